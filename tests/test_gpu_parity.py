"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Kernel level: CSR product, small exponential, Krylov process.  Solver level:
fixed (tau, m) stepping (same arithmetic path, tight tolerance), adaptive
solves (relative 2-norm error <= 10 tol against the oracle), brute force on
tiny inputs, and the degenerate and error cases of the method.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0907_4631_amd as pk
    pk.lib()
    oracle.build(force=False)
    return pk


def say(*a):
    print(*a, flush=True)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def gpu_solve(pk, t, A, b, **kw):
    kw.setdefault("max_attempts", 200000)
    Ad = pk.DeviceCSR(A)
    bd = dev(np.asarray(b).T)
    u, st = pk.solve(t, Ad, bd, **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy(), st


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def ragged_matrix(n, seed):
    """Rows of very different lengths: empty rows, short rows and rows longer
    than one LDS tile can stage."""
    g = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        r = g.random()
        if r < 0.1:
            k = 0
        elif r < 0.97:
            k = int(g.integers(1, 9))
        else:
            k = int(g.integers(200, min(n, 6000)))
        c = np.unique(np.concatenate([[i], g.choice(n, size=k, replace=False)])) if k else []
        rows += [i] * len(c)
        cols += list(c)
    vals = g.standard_normal(len(rows))
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    return A


# ------------------------------------------------------------ kernel level

@pytest.mark.parametrize("case", ["laplace2d-30", "convdiff-512", "ragged-20000", "laplace3d-64"])
def test_spmv_matches_oracle(pk, case):
    say("spmv case", case)
    A = {"laplace2d-30": lambda: W.laplace2d(30),
         "convdiff-512": lambda: W.convdiff2d(512, 50.0, 50.0),
         "ragged-20000": lambda: ragged_matrix(20000, 5),
         "laplace3d-64": lambda: W.laplace3d(64)}[case]()
    x = np.random.default_rng(1).standard_normal(A.shape[0])
    y = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
    pk.spmv(pk.DeviceCSR(A), dev(x), y)
    torch.cuda.synchronize()
    ref = oracle.spmv(A, x)
    scale = abs(A) @ np.abs(x)
    assert np.all(np.abs(y.cpu().numpy() - ref) <= 1e-14 * scale + 1e-300)


@pytest.mark.parametrize("N,scale", [(1, 3.0), (2, 0.5), (5, 40.0), (16, 4.0), (17, 1.0),
                                     (41, 25.0), (42, 25.0), (44, 12.0), (45, 9.0),
                                     (64, 30.0), (70, 200.0), (80, 60.0), (81, 10.0),
                                     (92, 30.0), (93, 8.0), (103, 50.0),
                                     (128, 5.0), (129, 2.0), (137, 3.0)])
def test_expm_matches_oracle(pk, N, scale):
    say("expm case", N, scale)
    g = np.random.default_rng(N)
    H = g.standard_normal((N, N)) * scale / math.sqrt(N)
    E = pk.expm(dev(H)).cpu().numpy()
    R = oracle.expm(H)
    assert np.linalg.norm(E - R) <= 1e-13 * N * max(1.0, np.linalg.norm(R))


@pytest.mark.parametrize("lanczos", [0, 1])
def test_krylov_matches_oracle(pk, lanczos):
    say("krylov case lanczos", lanczos)
    A = W.laplace2d(40) if lanczos else W.convdiff2d(40, 20.0, 10.0)
    n = A.shape[0]
    v = np.random.default_rng(3).standard_normal(n)
    m = 30
    V, H, done = pk.krylov(pk.DeviceCSR(A), dev(v), m, lanczos)
    torch.cuda.synchronize()
    V, H = V.cpu().numpy(), H.cpu().numpy()
    Vr, Hr, _, mm = oracle.krylov(A, v, m, lanczos=bool(lanczos), reorth=1)
    assert done == mm == m
    hs = np.abs(Hr).max()
    assert np.abs(H - Hr).max() <= 1e-10 * hs
    assert np.abs(V - Vr).max() <= 1e-9
    G = V.T @ V
    if not lanczos:
        assert np.abs(G - np.eye(m + 1)).max() < 1e-13
    AV = A @ V[:, :m]
    assert np.linalg.norm(AV - V @ H) <= 1e-12 * sp.linalg.norm(A) * math.sqrt(m)


@pytest.mark.parametrize("case", ["convdiff-512 arnoldi m64", "laplace3d-128 lanczos m20"])
def test_krylov_full_grid_matches_oracle(pk, case):
    """The Krylov process on the full-size operators, where the library
    spreads it over one workgroup per CU (256 workgroups: the multi-level team
    reduction and the neighbour synchronisation), element by element against
    the oracle's CGS2."""
    say("krylov full grid", case)
    if case.startswith("convdiff"):
        A, m, lanczos = W.convdiff2d(512, 50.0, 50.0), 64, 0
    else:
        A, m, lanczos = W.laplace3d(128), 20, 1
    n = A.shape[0]
    v = np.random.default_rng(17).standard_normal(n)
    V, H, done = pk.krylov(pk.DeviceCSR(A), dev(v), m, lanczos)
    torch.cuda.synchronize()
    V, H = V.cpu().numpy(), H.cpu().numpy()
    Vr, Hr, _, mm = oracle.krylov(A, v, m, lanczos=bool(lanczos), reorth=1)
    assert done == mm == m
    eh = np.abs(H - Hr).max() / np.abs(Hr).max()
    ev = np.abs(V - Vr).max() / np.abs(Vr).max()
    say(f"  max |H - H_ref| / max |H_ref| = {eh:.2e}, max |V - V_ref| / max |V_ref| = {ev:.2e}")
    assert eh <= 1e-10
    assert ev <= 1e-8


# ------------------------------------------------------------ solver level

FIXED = [
    # name, matrix builder, p, t, tau, m
    ("lap2d-30 p1", lambda: W.laplace2d(30), 1, 1e-3, 1e-4, 12),
    ("convdiff-64 p3", lambda: W.convdiff2d(64, 30.0, 30.0), 3, 1e-3, 2.5e-4, 20),
    ("ragged-3000 p0", lambda: ragged_matrix(3000, 7) * 0.05, 0, 0.3, 0.1, 15),
    # ||tau H^||_1 of about 20: two squarings, the last one by columns only
    ("convdiff-64 p0 squarings", lambda: W.convdiff2d(64, 30.0, 30.0), 0, 2e-3, 1e-3, 20),
    ("lap2d-30 p2 squarings", lambda: W.laplace2d(30), 2, 4e-3, 2e-3, 16),
    # the largest Krylov dimension and p: exponential of order 137 (device-memory solve)
    ("convdiff-64 p8 m128", lambda: W.convdiff2d(64, 30.0, 30.0), 8, 4e-4, 2e-4, 128),
]


@pytest.mark.parametrize("name,build,p,t,tau,m", FIXED)
def test_fixed_tau_m_stepping_matches_oracle(pk, name, build, p, t, tau, m):
    """Same path on both sides: fixed substeps, fixed m, every step accepted."""
    say("fixed-step case", name)
    A = build()
    n = A.shape[0]
    b = np.random.default_rng(11).standard_normal((n, p + 1))
    kw = dict(tau_fixed=tau, m_init=m, m_max=m, adapt_m=0)
    u, st = gpu_solve(pk, t, A, b, **kw)
    ref, ost = oracle.phipm(t, A, b, **kw)
    assert st["status"] == 0
    assert st["lanczos"] == int(oracle.is_symmetric(A))
    assert st["steps"] == ost["steps"] and st["matvecs"] == ost["matvecs"]
    assert rel(u, ref) <= 1e-11, rel(u, ref)


ADAPTIVE = [
    # name, builder, p, t, tol
    ("config1 lap2d-30 p1", None, 1, 1e-3, 1e-7),
    ("lap2d-50 p0", lambda: W.laplace2d(50), 0, 2e-3, 1e-8),
    ("convdiff-48 p2", lambda: W.convdiff2d(48, 40.0, 20.0), 2, 5e-3, 1e-8),
    ("convdiff-32 p4 negative t", lambda: W.convdiff2d(32, 10.0, 0.0), 4, -2e-4, 1e-9),
    ("reaction-64 p2", lambda: W.reaction2d(64, 5999), 2, 1e-3, 1e-6),
    ("ragged-2000 p1", lambda: ragged_matrix(2000, 3) * 0.1, 1, 1.0, 1e-8),
]


@pytest.mark.parametrize("name,build,p,t,tol", ADAPTIVE)
def test_adaptive_matches_oracle(pk, name, build, p, t, tol):
    say("adaptive case", name)
    if build is None:
        pb = W.config1()
        A, b = pb.A, pb.b
    else:
        A = build()
        b = np.random.default_rng(5).standard_normal((A.shape[0], p + 1))
    u, st = gpu_solve(pk, t, A, b, tol=tol)
    ref, ost = oracle.phipm(t, A, b, tol=tol)
    say("  gpu", st, "\n  oracle", ost, "\n  rel", rel(u, ref))
    assert st["status"] == 0
    assert rel(u, ref) <= 10 * tol
    assert st["lanczos"] == int(oracle.is_symmetric(A))
    assert (st["setup_flags"] >> 2 & 1) == 1 - st["lanczos"]
    # the same trajectory of Algorithm 3: every accept/reject decision and
    # every change of tau and m agree with the oracle's
    assert (st["steps"], st["rejected"], st["matvecs"], st["expms"]) == \
        (ost["steps"], ost["rejected"], ost["matvecs"], ost["expms"])
    assert st["anorm"] == pytest.approx(abs(A).sum(axis=1).max(), rel=1e-14)


def _with_entries(A, entries):
    """A copy of CSR matrix A with the (row, col, value) entries set (added
    where absent, explicit zeros kept), columns sorted in each row."""
    M = A.tocoo()
    rows, cols, vals = list(M.row), list(M.col), list(M.data)
    where = {(int(r), int(c)): k for k, (r, c) in enumerate(zip(rows, cols))}
    for r, c, v in entries:
        if (r, c) in where:
            vals[where[(r, c)]] = v
        else:
            rows.append(r)
            cols.append(c)
            vals.append(v)
    B = sp.csr_matrix((np.array(vals, dtype=np.float64), (np.array(rows), np.array(cols))),
                      shape=A.shape)
    B.sort_indices()
    B.indptr = B.indptr.astype(np.int32)
    B.indices = B.indices.astype(np.int32)
    return B


_L30 = W.laplace2d(30)   # 900 rows; (31, 1) and (1, 31) are a coupled pair
SYMMETRY = [
    ("laplacian", [], True),
    ("mirrored pair added", [(700, 3, -0.5), (3, 700, -0.5)], True),
    ("entry below the diagonal without mirror", [(700, 3, -0.5)], False),
    ("entry above the diagonal without mirror", [(3, 700, -0.5)], False),
    ("explicit zero below the diagonal without mirror", [(700, 3, 0.0)], False),
    ("value changed below the diagonal", [(31, 1, -1.5)], False),
    ("value changed above the diagonal", [(1, 31, -1.5)], False),
]


@pytest.mark.parametrize("name,entries,symmetric", SYMMETRY)
def test_symmetry_decision_matches_oracle(pk, name, entries, symmetric):
    """The setup's exact symmetry test (same pattern, bitwise-equal values)
    picks Lanczos exactly when the oracle's entry-by-entry test does,
    including asymmetries present on one side of the diagonal only."""
    say("symmetry case", name)
    A = _with_entries(_L30, entries)
    assert oracle.is_symmetric(A) == symmetric
    b = np.random.default_rng(9).standard_normal((A.shape[0], 2))
    u, st = gpu_solve(pk, 1e-3, A, b, tol=1e-9)
    ref, _ = oracle.phipm(1e-3, A, b, tol=1e-9)
    assert st["lanczos"] == int(symmetric)
    assert (st["setup_flags"] >> 2 & 1) == int(not symmetric)
    assert rel(u, ref) <= 1e-8


@pytest.mark.parametrize("mode", ["fixed", "adaptive"])
def test_full_reorth_lanczos_matches_oracle(pk, mode):
    """Lanczos with CGS2 against every basis vector (Algorithm 2 with full
    reorthogonalisation) against the oracle's same flavour."""
    say("full-reorth lanczos", mode)
    A = W.laplace3d(20)
    b = np.random.default_rng(21).standard_normal((A.shape[0], 3))
    if mode == "fixed":
        kw = dict(tau_fixed=2e-4, m_init=40, m_max=40, adapt_m=0)
        t, gate = 1e-3, 1e-11
    else:
        kw = dict(tol=1e-8)
        t, gate = 4e-3, 10 * 1e-8
    u, st = gpu_solve(pk, t, A, b, reorth=pk.REORTH_FULL, **kw)
    ref, ost = oracle.phipm(t, A, b, reorth=2, **kw)
    loc, lst = oracle.phipm(t, A, b, reorth=1, **kw)
    say("  gpu", st, "\n  oracle", ost, "\n  rel", rel(u, ref))
    assert st["status"] == 0 and st["lanczos"] == 1
    assert rel(u, ref) <= gate
    assert (st["steps"], st["rejected"], st["matvecs"], st["expms"]) == \
        (ost["steps"], ost["rejected"], ost["matvecs"], ost["expms"])
    # the windowed flavour is a different computation of the same result
    assert rel(loc, ref) <= 10 * 1e-8 if mode == "adaptive" else True


def brute_force(A, b, t):
    import scipy.linalg as sla
    A = A.toarray()
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


@pytest.mark.parametrize("p", [0, 2, 4])
def test_tiny_vs_bruteforce(pk, p):
    say("tiny brute-force case p", p)
    A = W.random_sparse(60, 0.1, seed=p, shift=-3.0) * 6.0
    b = np.random.default_rng(p).standard_normal((60, p + 1))
    tol = 1e-8
    u, st = gpu_solve(pk, 1.0, A, b, tol=tol)
    ref = brute_force(A, b, 1.0)
    assert st["status"] == 0
    assert np.linalg.norm(u - ref) <= 10 * tol


def test_eigenvector_decay_is_exact(pk):
    say("eigenvector decay")
    A = W.laplace2d(30)
    v, lam = W.sine_mode2d(30, 2, 3)
    c = np.array([1.0, -0.5, 2.0])
    b = np.outer(v, c)
    t = 1e-3
    u, st = gpu_solve(pk, t, A, b, tol=1e-10)
    ref = sum(t ** k * oracle.phi(k, t * lam) * c[k] for k in range(3)) * v
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref)
    assert st["steps"] == 1 and st["rejected"] == 0


def test_degenerate_inputs(pk):
    say("degenerate inputs")
    A = W.laplace2d(10)
    n = 100
    b = np.random.default_rng(0).standard_normal((n, 3))
    u, st = gpu_solve(pk, 0.0, A, b)                      # t = 0: u = b0
    assert np.array_equal(u, b[:, 0]) and st["steps"] == 0
    Z = sp.csr_matrix((n, n))
    Z.indptr = Z.indptr.astype(np.int32)
    Z.indices = Z.indices.astype(np.int32)
    u, st = gpu_solve(pk, 0.7, Z, b)                      # A = 0
    ref = sum(0.7 ** k / math.factorial(k) * b[:, k] for k in range(3))
    assert np.allclose(u, ref, rtol=1e-15, atol=1e-15)
    u, st = gpu_solve(pk, 0.01, A, np.zeros((n, 3)))      # b = 0
    assert np.all(u == 0.0)
    one = sp.csr_matrix(np.array([[-2.0]]))               # n = 1
    one.indptr = one.indptr.astype(np.int32)
    one.indices = one.indices.astype(np.int32)
    bb = np.array([[1.5, 0.5]])
    u, st = gpu_solve(pk, 0.3, one, bb, tol=1e-12)
    ref = math.exp(-0.6) * 1.5 + 0.3 * oracle.phi(1, -0.6) * 0.5
    assert abs(u[0] - ref) <= 1e-13
    # largest p
    b8 = np.random.default_rng(1).standard_normal((n, 9))
    u, st = gpu_solve(pk, 2e-3, A, b8, tol=1e-9)
    ref, _ = oracle.phipm(2e-3, A, b8, tol=1e-9)
    assert rel(u, ref) <= 1e-8


def test_error_reporting(pk):
    say("error reporting")
    A = W.laplace2d(8)
    n = 64
    b = np.random.default_rng(0).standard_normal((n, 2))
    bn = b.copy()
    bn[5, 1] = np.nan
    with pytest.raises(pk.PhipmError) as e:
        gpu_solve(pk, 1e-3, A, bn)
    assert e.value.status == pk.ENONFINITE
    bad = A.copy()
    bad.indices = bad.indices.copy()
    bad.indices[3], bad.indices[4] = bad.indices[4], bad.indices[3]   # unsorted row
    with pytest.raises(pk.PhipmError) as e:
        gpu_solve(pk, 1e-3, bad, b)
    assert e.value.status == pk.EINVAL
    with pytest.raises(pk.PhipmError) as e:
        gpu_solve(pk, 1.0, A, b, max_attempts=2, tol=1e-12)
    assert e.value.status == pk.EMAXSTEPS
    with pytest.raises(pk.PhipmError) as e:
        gpu_solve(pk, 1.0, A, b, m_max=pk.M_CAP + 1)
    assert e.value.status == pk.EINVAL


@pytest.mark.parametrize("wg", [1, 3, 8, 64])
def test_workgroup_count_does_not_change_result(pk, wg):
    say("workgroups", wg)
    A = W.convdiff2d(96, 25.0, 5.0)
    b = np.random.default_rng(2).standard_normal((A.shape[0], 2))
    u, st = gpu_solve(pk, 2e-3, A, b, tol=1e-9, workgroups=wg)
    ref, _ = oracle.phipm(2e-3, A, b, tol=1e-9)
    assert st["workgroups"] == wg
    assert rel(u, ref) <= 1e-8


@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_heston_matches_oracle(pk, tol):
    """The paper's Heston example (n = 5100, p = 1, t = T = 1) in the
    benchmark's launch configuration."""
    say("heston tol", tol)
    pb = W.heston_problem(tol)
    u, st = gpu_solve(pk, pb.t, pb.A, pb.b, tol=tol)
    ref, ost = oracle.phipm(pb.t, pb.A, pb.b, tol=tol)
    say("  gpu", st, "\n  oracle", ost)
    assert st["status"] == 0 and st["lanczos"] == 0
    assert np.linalg.norm(u - ref) <= 10 * tol * max(1.0, np.linalg.norm(ref))


@pytest.mark.parametrize("name,build,p,t,tol,m", [
    ("lap2d-50 p1 m30", lambda: W.laplace2d(50), 1, 2e-3, 1e-8, 30),
    ("convdiff-64 p2 m30", lambda: W.convdiff2d(64, 30.0, 30.0), 2, 5e-3, 1e-8, 30),
    ("convdiff-48 p0 m8", lambda: W.convdiff2d(48, 40.0, 20.0), 0, 5e-3, 1e-7, 8),
])
def test_fixed_m_phip_matches_oracle(pk, name, build, p, t, tol, m):
    """The paper's phip: Krylov dimension fixed, only the step size adapted
    (Algorithm 4 without its m branch)."""
    say("phip case", name)
    A = build()
    b = np.random.default_rng(8).standard_normal((A.shape[0], p + 1))
    kw = dict(tol=tol, adapt_m=0, m_init=m, m_max=m)
    u, st = gpu_solve(pk, t, A, b, **kw)
    ref, ost = oracle.phipm(t, A, b, **kw)
    say("  gpu", st, "\n  oracle", ost)
    assert st["status"] == 0
    assert st["m_last"] == m
    assert rel(u, ref) <= 10 * tol


@pytest.mark.parametrize("symmetric", [False, True])
@pytest.mark.parametrize("wg", [3, 8, 37])
def test_long_range_couplings_match_oracle(pk, symmetric, wg):
    """Rows coupled across the whole index range: every workgroup's products
    read rows owned by every other one (the neighbour waits span the team;
    37 is not a multiple of 8, so slots equal ranks there)."""
    say("long-range", "symmetric" if symmetric else "nonsymmetric", "workgroups", wg)
    A = W.random_sparse(6000, 0.001, seed=21, symmetric=symmetric, shift=-4.0)
    b = np.random.default_rng(6).standard_normal((A.shape[0], 2))
    u, st = gpu_solve(pk, 0.6, A, b, tol=1e-9, workgroups=wg)
    ref, _ = oracle.phipm(0.6, A, b, tol=1e-9)
    assert st["status"] == 0 and st["workgroups"] == wg
    assert st["lanczos"] == int(symmetric)
    assert rel(u, ref) <= 1e-8


def test_corner_coupling_matches_oracle(pk):
    """A banded operator plus entries coupling the first and the last rows:
    the first and last workgroups depend on the whole slot range."""
    say("corner coupling")
    A = W.convdiff2d(64, 20.0, 10.0)
    n = A.shape[0]
    A = sp.csr_matrix(A + sp.csr_matrix(([500.0, -300.0], ([0, n - 1], [n - 1, 0])), shape=(n, n)))
    A.sort_indices()
    b = np.random.default_rng(7).standard_normal((n, 3))
    u, st = gpu_solve(pk, 2e-3, A, b, tol=1e-9, workgroups=4)
    ref, _ = oracle.phipm(2e-3, A, b, tol=1e-9)
    assert st["status"] == 0
    assert rel(u, ref) <= 1e-8


FP32_CASES = [
    # name, builder, p, t, tol, expected basis use: "fp32" (every step FP32),
    # "mixed" (some steps FP64), "fp64" (every step FP64)
    ("config1 lap2d-30 p1", None, 1, 1e-3, 1e-7, "fp64"),
    ("lap3d-40 p3", lambda: W.laplace3d(40), 3, 1e-4, 1e-6, "fp32"),
    ("convdiff-96 p0", lambda: W.convdiff2d(96, 40.0, 40.0), 0, 1e-2, 1e-7, "mixed"),
    ("convdiff-96 p2", lambda: W.convdiff2d(96, 40.0, 40.0), 2, 1e-2, 1e-7, "mixed"),
    ("reaction-128 p2", lambda: W.reaction2d(128, 5999), 2, 1e-3, 1e-6, "fp64"),
    ("lap2d-64 p1 smooth", None, 1, 2e-3, 1e-6, "fp32"),
]


def fp32_problem(name, build, p):
    if name.startswith("config1"):
        pb = W.config1()
        return pb.A, pb.b
    if name.startswith("lap2d-64 p1 smooth"):
        # smooth data: the phi-part stays small, every step fits in FP32
        A = W.laplace2d(64)
        x = np.arange(1, 65) / 65.0
        s = np.outer(np.sin(np.pi * x), np.sin(2 * np.pi * x)).ravel()
        return A, np.stack([s, 0.5 * s], axis=1)
    A = build()
    return A, np.random.default_rng(9).standard_normal((A.shape[0], p + 1))


@pytest.mark.parametrize("name,build,p,t,tol,use", FP32_CASES)
def test_fp32_basis_meets_gate(pk, name, build, p, t, tol, use):
    """FP32 Krylov basis with FP64 Taylor part, exponential and control: within
    10 tol (relative 2-norm) of the FP64 oracle.  Each step picks its basis
    type from the rounding budget; the cases cover solves that run wholly in
    FP32, wholly in FP64 (the phi-part of eq. step far larger than u, as with
    rough data and p >= 1) and mixed."""
    say("fp32 case", name)
    A, b = fp32_problem(name, build, p)
    u, st = gpu_solve(pk, t, A, b, tol=tol, precision=pk.FP32_BASIS)
    ref, ost = oracle.phipm(t, A, b, tol=tol)
    say("  gpu fp32", st, "rel", rel(u, ref))
    assert st["status"] == 0
    assert rel(u, ref) <= 10 * tol
    if use == "fp32":
        assert st["fp64_steps"] == 0 and st["steps"] >= 1
    elif use == "fp64":
        assert st["fp64_steps"] == st["steps"]
    else:
        assert 0 < st["fp64_steps"] < st["steps"]


def test_fp32_only_diagnostic_shows_the_rounding(pk):
    """With every step forced into FP32 (a diagnostic option) the rough-data
    p = 2 solve leaves the gate: the per-step choice above is what keeps
    FP32 results within it."""
    say("fp32-only diagnostic")
    A = W.convdiff2d(96, 40.0, 40.0)
    b = np.random.default_rng(9).standard_normal((A.shape[0], 3))
    ref, _ = oracle.phipm(1e-2, A, b, tol=1e-7)
    u, st = gpu_solve(pk, 1e-2, A, b, tol=1e-7, precision=pk.FP32_BASIS,
                      fp32_flags=pk.FP32_ONLY)
    u2, st2 = gpu_solve(pk, 1e-2, A, b, tol=1e-7, precision=pk.FP32_BASIS)
    say("  fp32-only rel", rel(u, ref), st, "\n  per-step rel", rel(u2, ref), st2)
    assert st["status"] == 0 and st["fp64_steps"] == 0
    assert rel(u, ref) > rel(u2, ref)


@pytest.mark.parametrize("case", ["ragged-3000", "convdiff-64", "lap2d-40"])
@pytest.mark.parametrize("wg", [0, 4])
def test_workspace_contents_do_not_matter(pk, case, wg):
    """Nothing is read from the workspace before it is written: a workspace
    filled with NaN bit patterns and one filled with zeros give bitwise
    identical results."""
    say("workspace fill", case, wg)
    A = {"ragged-3000": lambda: ragged_matrix(3000, 7) * 0.05,
         "convdiff-64": lambda: W.convdiff2d(64, 30.0, 30.0),
         "lap2d-40": lambda: W.laplace2d(40)}[case]()
    n = A.shape[0]
    b = np.random.default_rng(12).standard_normal((n, 3))
    Ad = pk.DeviceCSR(A)
    bd = dev(b.T)
    outs = []
    for fill in (0, 255):
        s = pk.Solver(Ad, 2, tol=1e-8, workgroups=wg)
        s.ws.fill_(fill)
        u = torch.empty(n, dtype=torch.float64, device="cuda")
        st = s(0.05, bd, u)
        assert st["status"] == 0
        outs.append(u.cpu().numpy())
    assert np.all(np.isfinite(outs[1])) and np.array_equal(outs[0], outs[1])
