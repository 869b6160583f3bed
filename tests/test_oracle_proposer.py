"""Pins of the oracle's proposer references (CPU only): GELU, the network's
loss gradient, Adam and the hindsight label of a recorded step.

Each reference is checked against something other than itself: closed forms
and limits of GELU, central finite differences of the loss (independent of
backpropagation), Adam's closed-form first updates, and a brute-force scan
of omega(tau) with SciPy's matrix exponential for the label."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import workloads as W

NP = 5122


def test_gelu_closed_forms():
    assert oracle.gelu(0.0) == 0.0
    assert oracle.gelu_grad(0.0) == 0.5
    for z in (0.3, 1.7, 4.2):
        # tanh is odd, so gelu(z) - gelu(-z) = z exactly in real arithmetic
        assert oracle.gelu(z) - oracle.gelu(-z) == pytest.approx(z, rel=1e-15)
    assert oracle.gelu(12.0) == pytest.approx(12.0, rel=1e-15)
    assert abs(oracle.gelu(-12.0)) < 1e-30
    # value from the definition at z = 1: 0.5 (1 + tanh(sqrt(2/pi) 1.044715))
    assert oracle.gelu(1.0) == pytest.approx(0.5 * (1 + math.tanh(math.sqrt(2 / math.pi) * 1.044715)),
                                             rel=1e-15)
    for z in (-2.5, -0.4, 0.0, 0.9, 3.1):
        h = 1e-6
        fd = (oracle.gelu(z + h) - oracle.gelu(z - h)) / (2 * h)
        assert oracle.gelu_grad(z) == pytest.approx(fd, rel=1e-8, abs=1e-10)


def test_forward_of_a_hand_built_network():
    P = np.zeros(NP)
    W1, b1 = 0, 64 * 12
    W2, b2 = b1 + 64, b1 + 64 + 64 * 64
    W3, b3 = b2 + 64, b2 + 64 + 128
    P[W1 + 0 * 12 + 3] = 2.0          # unit 0 of layer 1 reads 2 x3
    P[b1 + 0] = -0.5
    P[W2 + 5 * 64 + 0] = 1.5          # unit 5 of layer 2 reads 1.5 a1_0
    P[W3 + 1 * 64 + 5] = -3.0         # output 1 reads -3 a2_5
    P[b3:b3 + 2] = [0.25, 1.0]
    x = np.linspace(-1, 1, 12)
    y = oracle.mlp_forward(P, x)[0]
    a1 = oracle.gelu(2.0 * x[3] - 0.5)
    a2_0 = oracle.gelu(0.0)           # units of layer 2 without inputs
    a2 = oracle.gelu(1.5 * a1)
    assert a2_0 == 0.0
    assert y[0] == 0.25
    assert y[1] == pytest.approx(1.0 - 3.0 * a2, rel=1e-15)


def test_loss_gradient_matches_finite_differences():
    g = np.random.default_rng(3)
    P = g.normal(0, 0.3, NP)
    X = g.normal(0, 1, (7, 12))
    T = g.normal(0, 1, (7, 2))
    L, grad = oracle.mlp_loss_grad(P, X, T)
    Y = oracle.mlp_forward(P, X)
    assert L == pytest.approx(np.sum((Y - T) ** 2) / (2 * 7), rel=1e-14)
    idx = np.concatenate([g.choice(NP, 300, replace=False), np.arange(768, 832),
                          np.arange(NP - 130, NP)])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (oracle.mlp_loss_grad(Pp, X, T, False) - oracle.mlp_loss_grad(Pm, X, T, False)) / (2 * h)
        assert grad[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_adam_first_updates_closed_form():
    g = np.random.default_rng(4)
    P0 = g.normal(size=50)
    grad = g.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 0.01
    P1, m1, v1 = oracle.adam_step(P0, m, v, grad, lr, 1)
    # bias-corrected moments equal g and g^2 after the first step
    assert np.allclose(P1, P0 - lr * grad / (np.abs(grad) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * grad, rtol=1e-15) and np.allclose(v1, 0.001 * grad ** 2, rtol=1e-15)
    P2, m2, v2 = oracle.adam_step(P1, m1, v1, grad, lr, 2)
    # with the same gradient again the corrected moments are still g and g^2
    assert np.allclose(P2, P1 - lr * grad / (np.abs(grad) + 1e-8), rtol=0, atol=1e-15)


def omega_scipy(Hs, mm, p, beta, tau, t_end, tol):
    N = mm + p + 1
    K = np.zeros((N, N))
    K[:mm, :mm] = tau * Hs[:mm, :mm]
    K[0, mm] = tau
    for i in range(p):
        K[mm + i, mm + i + 1] = tau
    E = sla.expm(K)
    c = E[mm - 1, mm + p]
    eps = beta * abs(Hs[mm, mm - 1]) * abs(c)
    return t_end * eps / (tau * tol), np.abs(K).sum(axis=0).max()


@pytest.mark.parametrize("p,lanczos,timed", [(0, 0, False), (2, 0, False), (1, 1, False),
                                             (2, 0, True), (1, 1, True)])
def test_label_against_brute_force_scan(p, lanczos, timed):
    costs = model_costs() if timed else None
    A = W.laplace2d(12) if lanczos else W.convdiff2d(12, 20.0, 20.0)
    n = A.shape[0]
    v = np.random.default_rng(p).standard_normal(n)
    m_have = 12
    V, Hb, beta, mm = oracle.krylov(A, v, m_have, lanczos=bool(lanczos))
    assert mm == m_have
    t_end, tol, t = 1e-2, 1e-7, 2e-3
    tau, m_use = 4e-4, 7
    ts, ms = oracle.label_step(Hb, m_use, m_have, p, lanczos, n, A.nnz, t, tau, beta, t_end, tol,
                               costs)
    lo, hi = 1, m_have          # every dimension up to 16 is a candidate
    assert lo <= ms <= hi
    grid = np.geomspace(tau / 4096, t_end - t, 3000)
    best = (np.inf, None, None)
    for m2 in range(lo, hi + 1):
        om = np.array([omega_scipy(Hb, m2, p, beta, tg, t_end, tol)[0] for tg in grid])
        ok = np.nonzero(om <= 0.8)[0]
        tg = grid[ok[-1]] if ok.size else grid[0]
        # omega is increasing in tau here, so the admissible set is an interval
        if ok.size:
            assert np.all(om[: ok[-1] + 1] <= 0.8 * (1 + 1e-9))
        kn = omega_scipy(Hb, m2, p, beta, tg, t_end, tol)[1]
        work = (oracle.step_time(m2, p, lanczos, n, A.nnz, costs) if costs else
                oracle.cost_C1(lanczos, m2, p, A.nnz, n, oracle.cost_M(kn)))
        cost = work / tg
        if cost < best[0]:
            best = (cost, m2, tg)
    step = grid[1] / grid[0]
    assert ms == best[1]
    assert best[2] <= ts <= best[2] * step * (1 + 1e-12)
    w, _ = oracle.step_omega(Hb, ms, p, beta, ts, t_end, tol)
    if ts < t_end - t:
        assert w == pytest.approx(0.8, rel=1e-9)


def model_costs():
    return oracle.label_costs(8e-6, 1e-6, 3e12, 25e9, 256,
                              [20e-6 + 3e-7 * N ** 2 for N in range(138)])


def test_step_time_hand_computed():
    c = model_costs()
    # n = 2048, nnz = 10000, p = 1, m = 2, Arnoldi: S = 12 nnz + 4 (n+1) + 16 n
    n, nnz = 2048, 10000
    S = 12 * nnz + 4 * (n + 1) + 16 * n
    byts = S + 8 * n * 1 + (S + 12 * 8 * n) + (S + 16 * 8 * n) + 16 * n + 16 * n + 24 * n
    G = 2
    want = (3 * 2 + 1 + 2) * 8e-6 + byts / min(3e12, G * 25e9) + c.expm_s[4]
    assert oracle.step_time(2, 1, 0, n, nnz, c) == pytest.approx(want, rel=1e-14)
    # a single workgroup uses the single-workgroup barrier and bandwidth
    want1 = (3 * 2 + 1 + 2) * 1e-6 + byts / 25e9 + c.expm_s[4]
    assert oracle.step_time(2, 1, 0, 1000, nnz, c) != want1   # different n, sanity
    n1 = 1000
    S1 = 12 * nnz + 4 * (n1 + 1) + 16 * n1
    b1 = S1 + 8 * n1 + (S1 + 12 * 8 * n1) + (S1 + 16 * 8 * n1) + 16 * n1 + 16 * n1 + 24 * n1
    assert oracle.step_time(2, 1, 0, n1, nnz, c) == pytest.approx(
        9 * 1e-6 + b1 / 25e9 + c.expm_s[4], rel=1e-14)
