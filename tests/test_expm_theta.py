"""The scaling threshold of the GPU's small exponential (degree-18 Taylor
polynomial with scaling and squaring): the constant in the kernel source, the
script that derives it, the published value, and the scalar backward error at
the threshold computed in 80-digit arithmetic."""
import math
import os
import re
import runpy
import types
from decimal import Decimal, getcontext

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_0907_4631_amd", "csrc")
U = 2.0 ** -53


def _script():
    # run_path compiles without writing a bytecode cache beside the kernel sources
    return types.SimpleNamespace(**runpy.run_path(os.path.join(CSRC, "taylor_theta.py")))


def _kernel_theta() -> float:
    src = open(os.path.join(CSRC, "dense.hpp")).read()
    return float(re.search(r"TAYLOR18_THETA = ([0-9.eE+-]+);", src).group(1))


def _scalar_backward_error(x: float, m: int = 18) -> float:
    """|log(exp(-x) T_m(x))| / |x|, the relative backward error of T_m at the scalar x."""
    getcontext().prec = 80
    d = Decimal(x)
    t = sum(d ** k / Decimal(math.factorial(k)) for k in range(m + 1))
    return float(abs(((-d).exp() * t).ln())) / abs(x)


def test_kernel_constant_is_the_derived_threshold():
    assert abs(_kernel_theta() - _script().theta(18)) <= 1e-14


def test_threshold_matches_published_value():
    # Al-Mohy and Higham (2011), Table 3.1: theta_18 = 1.09 for double precision
    assert abs(_kernel_theta() - 1.09) < 5e-3
    # and the Pade-13 analogue the paper prints (5.37) is larger: two more squarings at most
    assert 2.0 < math.log2(5.37 / _kernel_theta()) < 2.5


def test_scalar_backward_error_at_threshold():
    th = _kernel_theta()
    # on the negative axis every term of the error series has one sign, so the
    # norm bound is attained: the backward error is the unit roundoff exactly
    assert abs(_scalar_backward_error(-th) / U - 1.0) < 1e-6
    assert _scalar_backward_error(-1.01 * th) > U
    assert _scalar_backward_error(th) <= U


def test_series_starts_after_the_degree():
    c = _script().log_series(18, terms=40)
    assert all(x == 0 for x in c[:19]) and c[19] != 0
    # leading term: exp(-x) T_m(x) = 1 - x^(m+1)/(m+1)! + ...
    assert c[19] == -1 / __import__("fractions").Fraction(math.factorial(19))
