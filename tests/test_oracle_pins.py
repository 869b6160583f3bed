"""Pins for the CPU oracle against facts that the paper and mathematics fix.

Each test names the passage it pins.  None of them retypes the oracle's own
formula: they use closed forms, high-precision quadrature, library routines,
brute force on tiny inputs, invariants and special cases.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
import workloads as W

mpmath.mp.dps = 40


# ----------------------------------------------------------- scalar phi_k

ZS = [-40.0, -7.5, -2.0, -1.0, -0.6, -1e-4, 0.0, 1e-6, 0.3, 0.99, 1.7, 6.0]


def _phi_mp(k, z):
    """phi_k from the integral definition (eq. phifunctions) by mpmath quadrature."""
    z = mpmath.mpf(z)
    if k == 0:
        return mpmath.e ** z
    f = lambda th: mpmath.e ** ((1 - th) * z) * th ** (k - 1)
    return mpmath.quad(f, [0, 1]) / mpmath.factorial(k - 1)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5])
def test_phi_matches_integral_definition(oracle_lib, k):
    for z in ZS:
        ref = float(_phi_mp(k, z))
        got = oracle.phi(k, z)
        assert abs(got - ref) <= 2e-13 * abs(ref) + 1e-300, (k, z, got, ref)


def test_phi_closed_forms_small_l(oracle_lib):
    # phi_1..phi_3 as printed after eq. phifunctions, in 40-digit arithmetic
    for z in ZS:
        if z == 0.0:
            continue
        e = mpmath.e ** mpmath.mpf(z)
        zz = mpmath.mpf(z)
        closed = [(e - 1) / zz, (e - 1 - zz) / zz ** 2, (e - 1 - zz - zz ** 2 / 2) / zz ** 3]
        for k, ref in enumerate(closed, start=1):
            assert oracle.phi(k, z) == pytest.approx(float(ref), rel=2e-13)


def test_phi_at_zero_and_recurrence(oracle_lib):
    for k in range(9):
        assert oracle.phi(k, 0.0) == pytest.approx(1.0 / math.factorial(k), rel=1e-15)
    # eq. phirelation: phi_l(z) = z phi_{l+1}(z) + 1/l!
    for l in range(1, 6):
        for z in ZS:
            lhs = oracle.phi(l, z)
            rhs = z * oracle.phi(l + 1, z) + 1.0 / math.factorial(l)
            assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-15)


# ---------------------------------------------------- dense exponential

def test_expm_closed_forms(oracle_lib):
    d = np.array([-30.0, -1.0, 0.0, 0.5, 3.0])
    assert np.allclose(oracle.expm(np.diag(d)), np.diag(np.exp(d)), rtol=1e-13, atol=0)
    # nilpotent shift: the exponential series terminates
    Nn = 6
    J = np.diag(np.ones(Nn - 1), 1) * 2.5
    ref = sum(np.linalg.matrix_power(J, k) / math.factorial(k) for k in range(Nn))
    assert np.allclose(oracle.expm(J), ref, rtol=1e-14, atol=1e-14)
    # rotation generator
    for th in (0.3, 7.0, 40.0):
        R = oracle.expm(np.array([[0.0, th], [-th, 0.0]]))
        ref = np.array([[math.cos(th), math.sin(th)], [-math.sin(th), math.cos(th)]])
        assert np.allclose(R, ref, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_expm_vs_library(oracle_lib, seed):
    g = np.random.default_rng(seed)
    for N, scale in ((5, 0.1), (17, 1.0), (40, 6.0), (70, 30.0)):
        A = g.standard_normal((N, N)) * scale / math.sqrt(N)
        E = oracle.expm(A)
        R = sla.expm(A)
        assert np.linalg.norm(E - R) <= 1e-13 * max(1.0, np.linalg.norm(R)) * N


def _augmented(H, tau, p):
    """tau*K with K = [[H, e1, 0], [0, 0, I_p], [0, 0, 0]] of size m+p+1."""
    m = H.shape[0]
    N = m + p + 1
    K = np.zeros((N, N))
    K[:m, :m] = tau * H
    K[0, m] = tau
    for i in range(p):
        K[m + i, m + i + 1] = tau
    return K


@pytest.mark.parametrize("p", [0, 1, 3])
def test_augmented_matrix_identity(oracle_lib, p):
    # eq. hathm: the top m entries of the columns appended to H hold
    # tau^k phi_k(tau H) e_1; checked through the eigen-decomposition of a
    # symmetric H with the (pinned) scalar phi_k.
    g = np.random.default_rng(7)
    m = 12
    d = -np.abs(g.standard_normal(m)) * 10
    e = g.standard_normal(m - 1) * 3
    H = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    lam, Q = np.linalg.eigh(H)
    tau = 0.7
    E = oracle.expm(_augmented(H, tau, p))
    for k in range(1, p + 2):
        ref = Q @ (np.array([tau ** k * oracle.phi(k, tau * l) for l in lam]) * Q[0, :])
        assert np.allclose(E[:m, m + k - 1], ref, rtol=1e-12, atol=1e-15)
    ref0 = Q @ (np.exp(tau * lam) * Q[0, :])
    assert np.allclose(E[:m, 0], ref0, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------- Krylov bases

def test_arnoldi_cgs2_orthonormal_and_relation(oracle_lib):
    A = W.random_sparse(300, 0.03, seed=3, shift=-2.0)
    v = np.random.default_rng(1).standard_normal(300)
    m = 40
    V, H, beta, mm = oracle.krylov(A, v, m, lanczos=False, reorth=1)
    assert mm == m
    assert beta == pytest.approx(np.linalg.norm(v), rel=1e-15)
    assert np.allclose(V[:, 0] * beta, v, rtol=1e-14, atol=1e-14)
    G = V.T @ V
    assert np.abs(G - np.eye(m + 1)).max() < 1e-13
    # Arnoldi relation A V_m = V_{m+1} Hbar_m, and H_m = V_m^T A V_m
    AV = A @ V[:, :m]
    assert np.linalg.norm(AV - V @ H) <= 1e-12 * sp.linalg.norm(A)
    assert np.allclose(V[:, :m].T @ AV, H[:m, :m], atol=1e-11)
    assert np.all(np.tril(H, -2) == 0.0)


def test_arnoldi_mgs_equals_cgs2(oracle_lib):
    # Algorithm 1 (modified Gram-Schmidt) spans the same basis
    A = W.random_sparse(200, 0.05, seed=4, shift=-1.0)
    v = np.random.default_rng(2).standard_normal(200)
    V1, H1, _, _ = oracle.krylov(A, v, 15, lanczos=False, reorth=0)
    V2, H2, _, _ = oracle.krylov(A, v, 15, lanczos=False, reorth=1)
    assert np.allclose(H1, H2, atol=1e-10)
    assert np.allclose(V1, V2, atol=1e-10)


@pytest.mark.parametrize("reorth", [0, 1])
def test_lanczos_tridiagonal(oracle_lib, reorth):
    A = W.laplace2d(20)
    v = np.random.default_rng(5).standard_normal(400)
    m = 25
    V, H, beta, mm = oracle.krylov(A, v, m, lanczos=True, reorth=reorth)
    assert mm == m
    band = np.triu(np.tril(H, 1), -1)
    assert np.all(H == band)
    Hm = H[:m, :m]
    assert np.allclose(Hm, Hm.T, rtol=1e-8, atol=1e-8 * np.abs(Hm).max())
    AV = A @ V[:, :m]
    assert np.linalg.norm(AV - V @ H) <= 1e-11 * sp.linalg.norm(A)
    # the same tridiagonal matrix as full Arnoldi for a short run
    V2, H2, _, _ = oracle.krylov(A, v, 8, lanczos=False, reorth=1)
    assert np.allclose(H[:9, :8], H2, atol=1e-9 * np.abs(H2).max())


def test_lanczos_full_reorth_keeps_orthogonality(oracle_lib):
    # Algorithm 2 with classical Gram-Schmidt applied twice against every
    # basis vector: orthonormal to rounding, and H tridiagonal up to rounding
    # (symmetric A), over a run long enough for the three-term recurrence
    # (and its local reorthogonalisation) to lose orthogonality: eigenvalues
    # spread over six decades, the largest ones well separated
    n = 1000
    A = sp.diags(-np.logspace(0.0, 6.0, n)).tocsr()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    v = np.random.default_rng(8).standard_normal(n)
    m = 80
    V, H, _, mm = oracle.krylov(A, v, m, lanczos=True, reorth=2)
    assert mm == m
    assert np.abs(V.T @ V - np.eye(m + 1)).max() < 1e-13
    off = H - np.triu(np.tril(H, 1), -1)
    assert np.abs(off).max() <= 1e-12 * np.abs(H).max()
    for r in (0, 1):   # the recurrence alone, and with the two-vector window, drift
        V0, _, _, _ = oracle.krylov(A, v, m, lanczos=True, reorth=r)
        assert np.abs(V0.T @ V0 - np.eye(m + 1)).max() > 1e-3


def test_lanczos_full_reorth_solve_is_the_arnoldi_solve(oracle_lib):
    # full reorthogonalisation runs the Arnoldi process on the symmetric
    # matrix and eq. 4 prices it as Arnoldi: the same solve, bit for bit
    A = W.laplace2d(24)
    b = np.random.default_rng(9).standard_normal((576, 3))
    u1, s1 = oracle.phipm(4e-3, A, b, tol=1e-8, symm=1, reorth=2)
    u2, s2 = oracle.phipm(4e-3, A, b, tol=1e-8, symm=0, reorth=1)
    assert np.array_equal(u1, u2) and s1 == s2
    u3, _ = oracle.phipm(4e-3, A, b, tol=1e-8, symm=1, reorth=1)
    assert np.linalg.norm(u1 - u3) <= 10 * 1e-8 * np.linalg.norm(u3)


# -------------------------------------------------------- controller pieces

def test_tau0_matches_stirling_free_form(oracle_lib):
    # eq. tau_0 is ten times the step at which 4 ||b|| ||A|| (tau ||A||)^m / (m+1)!
    # equals Tol once Stirling's formula replaces (m+1)!.
    for tol, a, b, m in ((1e-7, 7688.0, 3.2, 55.0), (1e-6, 2e5, 1.0, 20.0), (1e-3, 1.0, 1.0, 5.0)):
        t0 = oracle.tau0(tol, a, b, m) / 10.0
        lhs = math.log(4 * b * a) + m * math.log(t0 * a) - math.lgamma(m + 2)
        # Stirling's relative error for (m+1)! is about 1/(12(m+1))
        assert abs(lhs - math.log(tol)) < 1.5 / (12 * (m + 1)), (tol, a, b, m)
    # exponents: tau_0 ~ Tol^(1/m) ||b||^(-1/m) ||A||^(-1-1/m)
    m = 30.0
    base = oracle.tau0(1e-6, 100.0, 2.0, m)
    assert oracle.tau0(1e-6 * 2 ** m, 100.0, 2.0, m) == pytest.approx(2 * base, rel=1e-12)
    assert oracle.tau0(1e-6, 100.0, 2.0 * 3 ** m, m) == pytest.approx(base / 3, rel=1e-12)
    assert oracle.tau0(1e-6, 200.0, 2.0, m) == pytest.approx(base * 2 ** (-1 - 1 / m), rel=1e-12)


def test_cost_M_counts_the_expm_squarings(oracle_lib):
    # eq. 8: one division (8/3 N^3) and 6 + s products (2 N^3 each), with s
    # the squarings the Pade method performs.
    g = np.random.default_rng(11)
    for scale in (0.01, 1.0, 5.0, 5.5, 20.0, 300.0, 1e4):
        A = g.standard_normal((9, 9))
        A *= scale / np.abs(A).sum(axis=0).max()
        s = oracle.lib().oracle_expm(9, np.ascontiguousarray(A), np.empty((9, 9)))
        assert oracle.cost_M(np.abs(A).sum(axis=0).max()) == pytest.approx(8 / 3 + 2 * (6 + s))


def test_cost_C1_and_C(oracle_lib):
    n, nnz, M = 1000.0, 5000.0, 20.0
    for p in (0, 1, 3):
        for m in (1, 2, 3, 10, 40):
            la = oracle.cost_C1(True, m, p, nnz, n, M)
            ar = oracle.cost_C1(False, m, p, nnz, n, M)
            # Arnoldi orthogonalisation costs (m-1)(m-2) n more than Lanczos
            assert ar - la == pytest.approx((m - 1) * (m - 2) * n)
            # (m+p) products with A
            assert (oracle.cost_C1(True, m, p, nnz + 1, n, M) - la) == pytest.approx(m + p)
            # the small exponential of size m+p+1
            assert (oracle.cost_C1(True, m, p, nnz, n, M + 1) - la) == pytest.approx((m + p + 1) ** 3)
    assert oracle.cost_C(1.0, 0.3, 7.0) == pytest.approx(28.0)
    assert oracle.cost_C(1.0, 1.0, 7.0) == pytest.approx(7.0)
    assert oracle.cost_C(1.0, math.inf, 7.0) == pytest.approx(7.0)


def test_alg4_fixed_point_and_defaults(oracle_lib):
    s = oracle.Alg4State()
    tn, mn, q, k = oracle.alg4(s, 0.01, 12, 1e-9, 0.8)
    assert (q, k) == (3.0, 2.0)       # q = m/4, kappa = 2 without history
    assert tn == pytest.approx(0.01) and mn == 12.0
    s = oracle.Alg4State()
    tn, mn, q, k = oracle.alg4(s, 0.01, 12, 1e-9, 0.8 * 2 ** 5)
    assert mn == 17.0                 # eq. 3 with kappa = 2
    assert tn == pytest.approx(0.01 * 2 ** (-5 / 4))   # eq. 2 with q = 3


def test_alg4_recovers_order_after_tau_reduction(oracle_lib):
    # error model eps = C tau^(q+1) (Sect. 3.4): after a rejected attempt whose
    # tau was reduced, eq. 6 must return q itself.
    q_true, Cc = 2.5, 3e4
    s = oracle.Alg4State()
    tau1, m = 0.2, 16
    eps1 = Cc * tau1 ** (q_true + 1)
    oracle.alg4(s, tau1, m, eps1, 5.0)
    s.prev_rejected, s.prev_branch, s.eps_old, s.tau_old, s.m_old = 1, 1, eps1, tau1, m
    tau2 = 0.05
    eps2 = Cc * tau2 ** (q_true + 1)
    _, _, q, _ = oracle.alg4(s, tau2, m, eps2, 2.0)
    assert q == pytest.approx(q_true, rel=1e-12)
    assert s.q_valid == 1
    # a following m-change keeps that order (Algorithm 4, second branch)
    s.prev_rejected, s.prev_branch, s.eps_old, s.tau_old, s.m_old = 1, 2, eps2, tau2, m
    _, _, q2, _ = oracle.alg4(s, tau2, m + 3, eps2 / 8, 1.5)
    assert q2 == pytest.approx(q_true, rel=1e-12)


def test_alg4_recovers_kappa_after_m_change(oracle_lib):
    # error model eps = C kappa^(-m) (Sect. 3.4, eq. 7)
    kap, Cc = 3.7, 1.0
    s = oracle.Alg4State()
    m1, m2, tau = 10, 14, 0.1
    e1, e2 = Cc * kap ** (-m1), Cc * kap ** (-m2)
    oracle.alg4(s, tau, m1, e1, 9.0)
    s.prev_rejected, s.prev_branch, s.eps_old, s.tau_old, s.m_old = 1, 2, e1, tau, m1
    _, mn, _, k = oracle.alg4(s, tau, m2, e2, 3.0)
    assert k == pytest.approx(kap, rel=1e-12)
    assert mn == math.ceil(m2 + math.log(3.0 / 0.8) / math.log(kap))


# ------------------------------------------------------- whole solver

def brute_force(A, b, t):
    """u(t) from eq. phide: exp(t M) [b_0; e_p] with M = [[A, B], [0, J]],
    B = [b_p, ..., b_1] and J the upper shift (a library matrix exponential)."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A)
    n, p1 = b.shape
    p = p1 - 1
    M = np.zeros((n + p, n + p))
    M[:n, :n] = A
    for i in range(p):
        M[:n, n + i] = b[:, p - i]
        if i + 1 < p:
            M[n + i, n + i + 1] = 1.0
    x0 = np.zeros(n + p)
    x0[:n] = b[:, 0]
    if p > 0:
        x0[n + p - 1] = 1.0
    return (sla.expm(t * M) @ x0)[:n]


CASES = [
    # (seed, n, symmetric, p, t, tol)
    (0, 40, False, 0, 1.0, 1e-8),
    (1, 60, False, 2, 2.0, 1e-7),
    (2, 50, True, 1, 1.5, 1e-9),
    (3, 80, True, 4, 0.7, 1e-6),
    (4, 30, False, 3, -0.15, 1e-8),
]


@pytest.mark.parametrize("seed,n,symm,p,t,tol", CASES)
def test_phipm_vs_bruteforce(oracle_lib, seed, n, symm, p, t, tol):
    A = W.random_sparse(n, 0.1, seed=seed, symmetric=symm, shift=-3.0) * 6.0
    A = sp.csr_matrix(A)
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    b = np.random.default_rng(seed + 50).standard_normal((n, p + 1))
    u, st = oracle.phipm(t, A, b, tol=tol)
    ref = brute_force(A, b, t)
    err = np.linalg.norm(u - ref)
    assert err <= 4 * tol * max(1.0, abs(t)) + 1e-13 * np.linalg.norm(ref), (err, st)
    assert st["steps"] >= 1 and st["expms"] == st["steps"] + st["rejected"]
    assert st["matvecs"] >= p * st["steps"] + st["steps"]


def test_phipm_largest_sizes_vs_bruteforce(oracle_lib):
    """Krylov dimension 128 and p = 8 (a small exponential of order 137), two
    fixed substeps at tau ||A||_inf = 8, against the brute-force exponential of
    the augmented matrix (eq. phide)."""
    A = W.convdiff2d(32, 30.0, 30.0)
    tau = 8.0 / abs(A).sum(axis=1).max()
    b = np.random.default_rng(21).standard_normal((A.shape[0], 9))
    u, st = oracle.phipm(2 * tau, A, b, tau_fixed=tau, m_init=128, m_max=128, adapt_m=0)
    assert st["steps"] == 2 and st["m_last"] == 128 and st["matvecs"] == 2 * (128 + 8)
    ref = brute_force(A, b, 2 * tau)
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref)


def test_phipm_diagonal_closed_form(oracle_lib):
    n, p, t = 50, 3, 0.9
    d = -np.linspace(0.1, 40.0, n)
    A = sp.csr_matrix(sp.diags(d))
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    b = np.random.default_rng(9).standard_normal((n, p + 1))
    u, _ = oracle.phipm(t, A, b, tol=1e-10)
    ref = np.array([sum(t ** k * oracle.phi(k, t * d[i]) * b[i, k] for k in range(p + 1))
                    for i in range(n)])
    assert np.linalg.norm(u - ref) <= 4e-10


def test_phipm_zero_matrix_and_zero_time(oracle_lib):
    n, p, t = 20, 3, 1.7
    A = sp.csr_matrix((n, n))
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    b = np.random.default_rng(1).standard_normal((n, p + 1))
    u, _ = oracle.phipm(t, A, b)
    ref = sum(t ** k / math.factorial(k) * b[:, k] for k in range(p + 1))
    assert np.allclose(u, ref, rtol=1e-15, atol=1e-15)
    B = W.laplace2d(5)
    u0, st = oracle.phipm(0.0, B, np.random.default_rng(2).standard_normal((25, 2)))
    assert st["steps"] == 0


@pytest.mark.parametrize("p", [0, 1, 3])
def test_phipm_heat_decay_of_eigenvector(oracle_lib, p):
    # Eigenvector data: u(t) = sum_k t^k phi_k(t lam) c_k v exactly; the Krylov
    # space is invariant after one vector (happy breakdown), so one step suffices.
    N = 30
    A = W.laplace2d(N)
    v, lam = W.sine_mode2d(N, 2, 3)
    c = np.array([1.0, -0.5, 2.0, 0.25])[: p + 1]
    b = np.outer(v, c)
    t = 1e-3
    u, st = oracle.phipm(t, A, b, tol=1e-10)
    ref = sum(t ** k * oracle.phi(k, t * lam) * c[k] for k in range(p + 1)) * v
    assert np.linalg.norm(u - ref) <= 1e-12 * max(1.0, np.linalg.norm(ref))
    assert st["steps"] == 1 and st["rejected"] == 0


def test_stepping_identity_exact_krylov(oracle_lib):
    # With m = n every projection is exact; eq. step + eq. wrecurrence must then
    # give the same u whatever the substeps (the forcing is re-expanded at t_k).
    n, p, t = 24, 3, 1.3
    A = W.random_sparse(n, 0.2, seed=21, shift=-2.0)
    b = np.random.default_rng(3).standard_normal((n, p + 1))
    ref = brute_force(A, b, t)
    for tau in (t, t / 3, t / 7):
        u, st = oracle.phipm(t, A, b, tau_fixed=tau, m_init=n, m_max=n, adapt_m=0)
        assert np.linalg.norm(u - ref) <= 1e-11 * np.linalg.norm(ref), tau


def test_resume_identity(oracle_lib):
    # eq. steppre: restarting at t1 from u(t1) with b_i' = sum_j t1^j/j! b_{i+j}
    n, p, t, t1 = 60, 2, 1.0, 0.35
    A = W.random_sparse(n, 0.1, seed=8, shift=-3.0) * 5
    b = np.random.default_rng(4).standard_normal((n, p + 1))
    tol = 1e-9
    u_full, _ = oracle.phipm(t, A, b, tol=tol)
    u1, _ = oracle.phipm(t1, A, b, tol=tol)
    b2 = np.zeros_like(b)
    b2[:, 0] = u1
    for i in range(1, p + 1):
        b2[:, i] = sum(t1 ** j / math.factorial(j) * b[:, i + j] for j in range(p - i + 1))
    u2, _ = oracle.phipm(t - t1, A, b2, tol=tol)
    assert np.linalg.norm(u2 - u_full) <= 4 * tol


def test_forward_back_and_linearity(oracle_lib):
    A = W.laplace2d(30)
    b0 = np.random.default_rng(6).standard_normal(900)
    t = 1e-4
    fwd, _ = oracle.phipm(t, A, b0[:, None], tol=1e-12)
    back, _ = oracle.phipm(-t, A, fwd[:, None], tol=1e-12)
    assert np.linalg.norm(back - b0) <= 1e-9 * np.linalg.norm(b0)
    b1 = np.random.default_rng(7).standard_normal((900, 2))
    b2 = np.random.default_rng(8).standard_normal((900, 2))
    tol = 1e-9
    ua, _ = oracle.phipm(1e-3, A, b1, tol=tol)
    ub, _ = oracle.phipm(1e-3, A, b2, tol=tol)
    uc, _ = oracle.phipm(1e-3, A, 2.0 * b1 - 0.5 * b2, tol=tol)
    assert np.linalg.norm(uc - (2.0 * ua - 0.5 * ub)) <= 10 * tol


def test_error_estimate_tracks_uncorrected_error(oracle_lib):
    # eq. errest estimates the error of eq. phipapprox (first term of the
    # series eq. errorseries); the corrected eq. phipapprox2 is more accurate.
    A = W.laplace2d(12) * 1e-2
    n = A.shape[0]
    g = np.random.default_rng(12)
    for p in (0, 2):
        b = g.standard_normal((n, p + 1))
        u0 = g.standard_normal(n)
        b_loc = b.copy()
        b_loc[:, 0] = u0
        for m, tau in ((4, 0.1), (6, 0.2), (8, 0.3), (12, 0.5)):
            exact = brute_force(A, b_loc, tau)
            unc, eps = oracle.step(A, b_loc, 0.0, u0, tau, m, lanczos=True, corrector=0)
            cor, eps2 = oracle.step(A, b_loc, 0.0, u0, tau, m, lanczos=True, corrector=1)
            e_unc = np.linalg.norm(unc - exact)
            e_cor = np.linalg.norm(cor - exact)
            assert eps == pytest.approx(eps2, rel=1e-12)
            assert 0.5 <= e_unc / eps <= 2.0, (p, m, tau, e_unc, eps)
            assert e_cor < 0.5 * e_unc


def test_a_priori_bound(oracle_lib):
    # eq. 1: ||exp(tau A)v - beta V_m exp(tau H_m) e_1|| <= 2 beta (tau rho)^m / m!
    A = W.laplace2d(15)
    n = A.shape[0]
    rho = float(np.abs(np.linalg.eigvalsh(A.toarray())).max())
    v = np.random.default_rng(13).standard_normal(n)
    tau = 4.0 / rho
    exact = sla.expm(tau * A.toarray()) @ v
    for m in (10, 14, 18):
        unc, _ = oracle.step(A, v[:, None], 0.0, v, tau, m, lanczos=True, corrector=0)
        err = np.linalg.norm(unc - exact)
        bound = 2 * np.linalg.norm(v) * (tau * rho) ** m / math.factorial(m)
        assert err <= bound


def test_symmetry_detection(oracle_lib):
    assert oracle.is_symmetric(W.laplace2d(10))
    assert oracle.is_symmetric(W.laplace3d(6))
    assert not oracle.is_symmetric(W.convdiff2d(10, 5.0, 5.0))
    assert oracle.is_symmetric(W.convdiff2d(10, 0.0, 0.0))
    assert oracle.is_symmetric(W.reaction2d(16, 3))


@pytest.mark.parametrize("entries", [
    [],
    [(70, 3, -0.5), (3, 70, -0.5)],      # a mirrored pair added
    [(70, 3, -0.5)],                     # below the diagonal, no mirror
    [(3, 70, -0.5)],                     # above the diagonal, no mirror
    [(70, 3, 0.0)],                      # explicit zero, no mirror
    [(11, 1, -7.0)],                     # one value changed below the diagonal
    [(1, 11, -7.0)],                     # one value changed above the diagonal
    [(5, 5, -1.0)],                      # a diagonal value changed
])
def test_symmetry_detection_one_sided_edits(oracle_lib, entries):
    """Exact symmetry (same stored pattern, equal values) against its
    definition on the dense matrix and the set of stored positions."""
    A = W.laplace2d(10).tocoo()
    rows, cols, vals = list(A.row), list(A.col), list(A.data)
    where = {(int(r), int(c)): k for k, (r, c) in enumerate(zip(rows, cols))}
    for r, c, v in entries:
        if (r, c) in where:
            vals[where[(r, c)]] = v
        else:
            rows.append(r)
            cols.append(c)
            vals.append(v)
    B = sp.csr_matrix((np.array(vals), (np.array(rows), np.array(cols))), shape=A.shape)
    B.sort_indices()
    B.indptr = B.indptr.astype(np.int32)
    B.indices = B.indices.astype(np.int32)
    stored = {(i, int(j)) for i in range(B.shape[0])
              for j in B.indices[B.indptr[i]:B.indptr[i + 1]]}
    dense = B.toarray()
    want = stored == {(j, i) for i, j in stored} and np.array_equal(dense, dense.T)
    assert oracle.is_symmetric(B) == want


def test_oracle_spmv_matches_scipy(oracle_lib):
    A = W.convdiff2d(40, 30.0, 10.0)
    x = np.random.default_rng(0).standard_normal(A.shape[0])
    assert np.allclose(oracle.spmv(A, x), A @ x, rtol=1e-14, atol=1e-9)


@pytest.mark.parametrize("p", [0, 2])
def test_corrector_improves_fixed_steps(oracle_lib, p):
    # eq. phipapprox2 against eq. phipapprox inside the stepping loop: with a
    # fixed small m and fixed substeps the corrected scheme is far more accurate.
    A = W.laplace2d(12) * 1e-2
    n = A.shape[0]
    b = np.random.default_rng(31).standard_normal((n, p + 1))
    t = 1.2
    ref = brute_force(A, b, t)
    errs = []
    for corr in (1, 0):
        u, st = oracle.phipm(t, A, b, tau_fixed=0.2, m_init=6, m_max=6, adapt_m=0, corrector=corr)
        assert st["steps"] == 6
        errs.append(np.linalg.norm(u - ref))
    assert errs[0] < 0.5 * errs[1], errs


def test_heston_operator_is_exact_for_linear_prices():
    """The Heston discretisation (workloads.heston) with its boundary vector:
    for U = s every difference quotient is exact (U_s = 1, U_ss = U_v = U_vv =
    U_sv = 0) and the boundary values (U(0, v) = 0, U(s, V) = s, U_s(S, v) = 1)
    agree with U, so A s + b1 = (rd - rf) s - rd s = -rf s."""
    import workloads as W
    for rf in (0.0, 0.01):
        A, b0, b1 = W.heston(rf=rf)
        ds = 800.0 / 101
        s = np.tile(np.arange(1, 101) * ds, 51)
        r = A @ s + b1
        assert np.abs(r + rf * s).max() <= 1e-12 * np.abs(A @ s).max()
    # structure: 100 x 51 unknowns, the v = 0 line with the one-sided U_v
    assert A.shape == (5100, 5100)
    assert A.nnz == 44900
    assert np.all(b0[:12] == 0.0) and b0[12] == pytest.approx(13 * ds - 100.0)
