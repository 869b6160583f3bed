"""Pins of Algorithm 3's decisions in the oracle (Sect. 3.4, Algorithm 3,
eqs. 2-5 and 8), CPU only.

Hand-computed cases fix acceptance at delta = 1.2, both clamps of tau
([tau/5, 2 tau] and t_end - t), the clamp of m to [floor(3m/4), ceil(4m/3)]
and to m_max, the cost comparison that picks the branch (ties take the
m-branch), and the forced tau-branch when m cannot move.  The arithmetic of
each expected value is written out in the comments, from the formulas of the
paper, not from the oracle's code.  Properties over every attempt of traced
solves tie the trajectory to the same rules, and the matrix-vector count to
the basis growth.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

GAMMA = 0.8
DELTA = 1.2


def fresh():
    return oracle.Alg4State()


# A common attempt: Lanczos, p = 0, n = 100, nnz = 500, ||tau K||_1 = 1 (no
# squarings, so M of eq. 8 is 44/3), m = 10, tau = 1/8, t_end - t = 1.
# Fresh Algorithm 4 memory: q = m/4 = 2.5, kappa = 2.
#   eq. 4 (Lanczos): C1(m) = (m+p) nnz + 3 (m+p) n + M (m+p+1)^3
#   C1(10) = 5000 + 3000 + (44/3) 1331 = 27521.33
#   C1(11) = 5500 + 3300 + (44/3) 1728 = 34144
#   C1(31) = 15500 + 9300 + (44/3) 32768 = 505397.33
BASE = dict(tau=0.125, knorm=1.0, rem=1.0, nnz=500.0, n=100.0, m_use=10, m_cap=100,
            lanczos=1, p=0)


def test_cost_pieces_by_hand():
    M = oracle.cost_M(1.0)
    assert M == pytest.approx(44.0 / 3.0, rel=1e-15)
    assert oracle.cost_C1(1, 10, 0, 500, 100, M) == pytest.approx(27521.333333333332, rel=1e-14)
    assert oracle.cost_C1(1, 11, 0, 500, 100, M) == pytest.approx(34144.0, rel=1e-14)
    # eq. 4 (Arnoldi): (m+p) nnz + (m^2 + 3p + 2) n + M (m+p+1)^3
    # m=10, p=2: 12*500 + 108*100 + M*2197 = 6000 + 10800 + 32222.67
    assert oracle.cost_C1(0, 10, 2, 500, 100, M) == pytest.approx(49022.666666666664, rel=1e-14)
    # eq. 8: ||.||_1 = 10.74 needs one squaring at theta 5.37 (10.74/5.37 = 2)
    assert oracle.cost_M(10.74) == pytest.approx(44.0 / 3.0 + 2.0, rel=1e-15)
    assert oracle.cost_M(10.75) == pytest.approx(44.0 / 3.0 + 4.0, rel=1e-15)
    # eq. 5: ceil((t_end - t)/tau) C1
    assert oracle.cost_C(1.0, 0.125, 10.0) == 80.0
    assert oracle.cost_C(1.0, 0.3, 10.0) == 40.0


def test_accept_at_delta_and_tau_branch():
    # omega = 1.2 = delta: accepted (Algorithm 3 accepts when omega <= delta).
    # tau_new = tau (gamma/omega)^(1/(q+1)) = 0.125 (2/3)^(1/3.5) = 0.1113264
    # m_new = ceil(10 + log(1.5)/log 2) = ceil(10.585) = 11
    # C(tau_new, 10) = ceil(1/0.111326) C1(10) = 9 * 27521.33 = 247692
    # C(tau, 11)     = ceil(1/0.125)    C1(11) = 8 * 34144    = 273152
    # the tau-branch is cheaper: tau_next = 0.111326 (inside [0.025, 0.25]), m stays 10
    d = oracle.decide(fresh(), eps=1.0, omega=DELTA, **BASE)
    assert d["accept"] is True
    assert d["branch"] == 1
    assert d["m_new"] == 11.0
    assert d["tau_next"] == pytest.approx(0.1113264, rel=1e-6)
    assert d["m_next"] == 10
    # the next double above delta is rejected, with the same proposal
    d = oracle.decide(fresh(), eps=1.0, omega=math.nextafter(DELTA, 2.0), **BASE)
    assert d["accept"] is False
    assert d["branch"] == 1
    assert d["tau_next"] == pytest.approx(0.1113264, rel=1e-6)
    # well inside: 1.19 accepts, 1.21 rejects
    assert oracle.decide(fresh(), eps=1.0, omega=1.19, **BASE)["accept"] is True
    assert oracle.decide(fresh(), eps=1.0, omega=1.21, **BASE)["accept"] is False


def test_m_branch_clamped_to_four_thirds():
    # omega = 1e6: tau_new = 0.125 (8e-7)^(1/3.5) = 0.125 exp(-14.03865/3.5)
    # = 0.0022643, m_new = ceil(10 + log(1.25e6)/log 2) = ceil(30.25) = 31.
    # C(tau_new, 10) = ceil(441.63) C1(10) = 442 * 27521.33 = 1.2164e7
    # C(tau, 31)     = 8 * C1(31)          = 8 * 505397.33 = 4.0432e6
    # the m-branch is cheaper; m_new = 31 is clamped to ceil(4*10/3) = 14,
    # tau is kept.
    d = oracle.decide(fresh(), eps=1.0, omega=1e6, **BASE)
    assert d["accept"] is False
    assert d["branch"] == 2
    assert d["m_new"] == 31.0
    assert d["tau_new"] == pytest.approx(0.0022643, rel=1e-4)
    assert d["m_next"] == 14
    assert d["tau_next"] == 0.125


def test_m_branch_clamped_to_three_quarters_and_m_max():
    # omega = 1e-6 on a long remaining interval (t_end - t = 100 tau):
    # m_new = ceil(10 + log(1.25e-6)/log 2) = ceil(-9.61) = -9, costed as m = 1:
    # C1(1) = 500 + 300 + (44/3) 8 = 917.33; tau_new = 0.125 (8e5)^(1/3.5) = 6.07.
    # C(tau_new, 10) = ceil(12.5/6.07) C1(10) = 3 * 27521.33 = 82564
    # C(tau, 1)      = 100 * 917.33 = 91733  -> tau-branch here; with rem = 1:
    # C(tau_new, 10) = 1 * 27521.33;  C(tau, 1) = 8 * 917.33 = 7338.67 -> m-branch,
    # and m_new = -9 is clamped up to floor(3*10/4) = 7.
    d = oracle.decide(fresh(), eps=1.0, omega=1e-6, **BASE)
    assert d["accept"] is True
    assert d["branch"] == 2
    assert d["m_new"] == -9.0
    assert d["m_next"] == 7
    assert d["tau_next"] == 0.125
    # m_max: omega = 1e6 wants 14 (above) but the cap is 12
    d = oracle.decide(fresh(), eps=1.0, omega=1e6, **{**BASE, "m_cap": 12})
    assert d["branch"] == 2 and d["m_next"] == 12


def test_tau_branch_clamped_to_twice_tau():
    # the same omega = 1e-6 with t_end - t = 12.5 (100 tau): C(tau_new, 10) =
    # 82564 < C(tau, 1) = 91733 (see above), so tau changes and tau_new =
    # 6.07 is clamped to 2 tau = 0.25.
    d = oracle.decide(fresh(), eps=1.0, omega=1e-6, **{**BASE, "rem": 12.5})
    assert d["accept"] is True
    assert d["branch"] == 1
    assert d["tau_new"] == pytest.approx(0.125 * (0.8e6) ** (1 / 3.5), rel=1e-12)
    assert d["tau_new"] == pytest.approx(6.0742, rel=1e-4)
    assert d["tau_next"] == 0.25
    assert d["m_next"] == 10


def test_tau_clamped_to_a_fifth_when_m_cannot_grow():
    # omega = 1e6 rejects and prefers m (above), but m is at its cap (m_cap =
    # m = 10): m cannot grow while rejecting, so tau changes instead, and
    # tau_new = 0.0022643 is clamped up to tau/5 = 0.025.
    d = oracle.decide(fresh(), eps=1.0, omega=1e6, **{**BASE, "m_cap": 10})
    assert d["accept"] is False
    assert d["branch"] == 1
    assert d["tau_next"] == 0.025
    assert d["m_next"] == 10


def test_tau_clamped_to_remaining_interval_and_fixed_m():
    # phip (m fixed): always the tau-branch.  omega = 1e-6, tau_new = 6.07,
    # 2 tau = 0.25, but only t_end - t = 0.1875 (1.5 tau) is left.
    d = oracle.decide(fresh(), eps=1.0, omega=1e-6, **{**BASE, "rem": 0.1875, "adapt_m": 0})
    assert d["branch"] == 1
    assert d["tau_next"] == 0.1875
    assert d["m_next"] == 10


def test_cost_tie_takes_m_branch():
    # omega = gamma: tau_new = tau and m_new = ceil(m + 0) = m, so
    # C(tau_new, m) = C(tau, m_new) exactly; ties go to m (strict comparison).
    d = oracle.decide(fresh(), eps=1.0, omega=GAMMA, **BASE)
    assert d["tau_new"] == 0.125 and d["m_new"] == 10.0
    assert d["branch"] == 2
    assert d["m_next"] == 10 and d["tau_next"] == 0.125


def test_breakdown_nonfinite_and_fixed_tau():
    # happy breakdown: the space is invariant, m is not adapted
    d = oracle.decide(fresh(), eps=0.0, omega=0.0, **{**BASE, "broke": 1, "m_req": 12})
    assert d["accept"] is True and d["branch"] == 1
    assert d["tau_next"] == 0.25
    # a non-finite ratio rejects and divides tau by 5, m as requested
    d = oracle.decide(fresh(), eps=float("inf"), omega=float("inf"), **{**BASE, "m_req": 12})
    assert d["accept"] is False and d["branch"] == 0
    assert d["tau_next"] == 0.025 and d["m_next"] == 12
    # a fixed substep accepts any omega
    d = oracle.decide(fresh(), eps=1.0, omega=1e9, **{**BASE, "tau_fixed": 1})
    assert d["accept"] is True and d["tau_next"] == 0.125


def test_memory_after_rejection_uses_estimated_order():
    # Reject with the tau-branch at omega = 2 (tau 1/8 -> tau_next), then
    # attempt again at tau_next with eps scaled as tau^(q+1), q = 3: Algorithm
    # 4 estimates q = 3 from the two attempts (eq. 6 read the right way up)
    # and proposes tau (gamma/omega)^(1/4).
    st = fresh()
    a = {**BASE, "m_cap": 10}
    d1 = oracle.decide(st, eps=2.0, omega=2.0, **a)
    assert d1["branch"] == 1 and not d1["accept"]
    t2 = d1["tau_next"]
    eps2 = 2.0 * (t2 / 0.125) ** 4
    om2 = 2.0 * (eps2 / 2.0) * (0.125 / t2)   # omega = t_end eps / (tau tol) scales as eps/tau
    d2 = oracle.decide(st, eps=eps2, omega=om2, **{**a, "tau": t2})
    assert d2["tau_new"] == pytest.approx(t2 * (GAMMA / om2) ** 0.25, rel=1e-12)


# ----------------------------------------------------- trajectory properties

def _problems():
    g = np.random.default_rng(11)
    pb = W.config1()
    yield "lap2d-30 p1", pb.A, pb.b, pb.t, pb.tol, {}
    A = W.convdiff2d(40, 30.0, 10.0)
    yield "convdiff-40 p2", A, g.standard_normal((A.shape[0], 3)), 5e-3, 1e-8, {}
    A = W.reaction2d(48, 5999)
    yield "reaction-48 p2", A, g.standard_normal((A.shape[0], 3)), 1e-3, 1e-6, {}
    A = W.laplace2d(40)
    yield "lap2d-40 p3 m_max 16", A, g.standard_normal((A.shape[0], 4)), 2e-3, 1e-8, \
        {"m_max": 16}
    A = W.convdiff2d(32, 10.0, 0.0)
    yield "convdiff-32 phip m 12", A, g.standard_normal((A.shape[0], 2)), 2e-3, 1e-8, \
        {"adapt_m": 0, "m_init": 12, "m_max": 12}


@pytest.mark.parametrize("case", list(range(5)))
def test_trace_follows_algorithm3(case):
    name, A, b, t, tol, kw = list(_problems())[case]
    u, st, tr = oracle.phipm(t, A, b, tol=tol, trace_cap=20000, **kw)
    assert len(tr) == st["steps"] + st["rejected"] > 0
    p = b.shape[1] - 1
    m_max = kw.get("m_max", 100)
    n_rej = 0
    matvecs = 0
    step_have = {}
    for i, r in enumerate(tr):
        # acceptance is exactly omega <= delta
        assert bool(r["accepted"]) == (r["omega"] <= DELTA), (name, i, r)
        n_rej += not r["accepted"]
        rem = t - r["t"] if t > 0 else abs(t) - r["t"]
        assert r["tau"] <= rem * (1 + 1e-15)
        if r["branch"] == 1:
            # tau changed within [tau/5, 2 tau] and not past t_end
            lo = min(r["tau"] / 5.0, rem)
            assert lo * (1 - 1e-15) <= r["tau_next"] <= 2.0 * r["tau"] * (1 + 1e-15), (name, i)
            assert r["tau_next"] <= rem * (1 + 1e-15)
            assert r["m_next"] == r["m"]
        elif r["branch"] == 2:
            # m changed within [floor(3m/4), ceil(4m/3)], at least 1, at most m_max
            m = r["m"]
            assert max(1, math.floor(0.75 * m)) <= r["m_next"] <= min(math.ceil(4 * m / 3),
                                                                        m_max), (name, i)
            assert r["tau_next"] == r["tau"]
        if not kw.get("adapt_m", 1):
            assert r["branch"] == 1 and r["m"] == kw["m_init"]
        # the next attempt starts from the decision (clipped to the interval left)
        if i + 1 < len(tr):
            nx = tr[i + 1]
            rem2 = (t if t > 0 else abs(t)) - nx["t"]
            if nx["hnext"] != 0.0:   # (a happy breakdown would stretch tau to the end)
                assert nx["tau"] == pytest.approx(min(r["tau_next"], rem2), rel=1e-15, abs=0)
            if nx["step"] == r["step"]:
                assert not r["accepted"]
                assert nx["t"] == r["t"]
            else:
                assert r["accepted"]
        step_have[r["step"]] = r["have"]
        assert r["have"] >= r["m"]
    assert n_rej == st["rejected"]
    # matrix-vector products: p per step for the w-recurrence plus every basis
    # vector built (the basis is reused across the rejections of a step)
    matvecs = sum(p + h for h in step_have.values())
    assert matvecs == st["matvecs"], (matvecs, st)
    assert st["expms"] == len(tr)
