"""Scaling threshold of the degree-m Taylor polynomial of exp in double precision.

For T_m(x) = sum_{k<=m} x^k / k!, write exp(-x) T_m(x) = exp(h(x)) with
h(x) = sum_{k>m} c_k x^k.  Then T_m(X) = exp(X + dX) with dX = h(X), and
||dX|| / ||X|| <= sum_{k>m} |c_k| ||X||^(k-1).  theta_m is the largest ||X||
for which that bound is at most the unit roundoff 2^-53 (the construction of
Higham's and Al-Mohy and Higham's scaling-and-squaring thresholds).  The
coefficients c_k are computed exactly in rational arithmetic: the series of
exp(-x) T_m(x), then its logarithm by the recurrence for log of a power series.

Run as a script to print theta_m for a few degrees; the kernels use theta_18.
"""
from fractions import Fraction
import math


def log_series(m: int, terms: int = 160) -> list[Fraction]:
    """Coefficients c_0..c_{terms-1} of log(exp(-x) T_m(x))."""
    e = [Fraction((-1) ** k, math.factorial(k)) for k in range(terms)]
    t = [Fraction(1, math.factorial(k)) if k <= m else Fraction(0) for k in range(terms)]
    g = [sum(e[i] * t[n - i] for i in range(n + 1)) for n in range(terms)]
    # log g with g_0 = 1: n l_n = n g_n - sum_{k=1}^{n-1} k l_k g_{n-k}
    c = [Fraction(0)] * terms
    for n in range(1, terms):
        acc = g[n]
        for k in range(1, n):
            if c[k] and g[n - k]:
                acc -= Fraction(k, n) * c[k] * g[n - k]
        c[n] = acc
    return c


def theta(m: int, u: float = 2.0 ** -53, terms: int = 160) -> float:
    c = [abs(float(x)) for x in log_series(m, terms)]
    assert all(x == 0.0 for x in c[1:m + 1]), "exp(-x) T_m(x) = 1 + O(x^(m+1))"
    bound = lambda th: sum(c[k] * th ** (k - 1) for k in range(m + 1, terms))
    lo, hi = 0.0, 20.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if bound(mid) <= u:
            lo = mid
        else:
            hi = mid
    return lo


if __name__ == "__main__":
    for m in (12, 16, 18, 20, 24):
        print(m, repr(theta(m)))
