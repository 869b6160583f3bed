"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only builds problems: sparse operators in CSR form (float64 values,
int32 indices, columns sorted within each row) and the vectors b_0..b_p.  It
contains none of the solver's arithmetic.

Grids use interior points only, lexicographic index i + N*j (+ N*N*k), mesh
width h = 1/(N+1) and homogeneous Dirichlet boundaries.  Every random draw
comes from ``numpy.random.Generator(PCG64(seed))``.

Workloads (the stand-ins for the paper's test matrices, which are not available):

* ``laplace2d``       5-point Laplacian (negative definite, symmetric).
* ``laplace3d``       7-point Laplacian.
* ``convdiff2d``      diffusion D times the 5-point Laplacian minus first-order
                      upwind convection with velocity (vx, vy) >= 0 (nonsymmetric).
* ``reaction2d``      Laplacian + diag(1 - 3 u^2) for a smooth random field u
                      (the Jacobian of an Allen-Cahn type right-hand side).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _csr(rows, cols, vals, n) -> sp.csr_matrix:
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    A.data = A.data.astype(np.float64)
    return A


def stencil2d(N: int, center: float, west: float, east: float, south: float,
              north: float, diag_extra: np.ndarray | None = None) -> sp.csr_matrix:
    """Constant-coefficient 5-point stencil on an N x N interior grid."""
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    i = idx % N
    j = idx // N
    rows = [idx]
    cols = [idx]
    c = np.full(n, center)
    if diag_extra is not None:
        c = c + diag_extra
    vals = [c]
    for di, dj, w in ((-1, 0, west), (1, 0, east), (0, -1, south), (0, 1, north)):
        ok = (i + di >= 0) & (i + di < N) & (j + dj >= 0) & (j + dj < N)
        rows.append(idx[ok])
        cols.append(idx[ok] + di + N * dj)
        vals.append(np.full(int(ok.sum()), w))
    return _csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)


def laplace2d(N: int) -> sp.csr_matrix:
    h2 = 1.0 / float(N + 1) ** 2
    return stencil2d(N, -4.0 / h2, 1.0 / h2, 1.0 / h2, 1.0 / h2, 1.0 / h2)


def laplace3d(N: int) -> sp.csr_matrix:
    n = N ** 3
    inv = float(N + 1) ** 2
    idx = np.arange(n, dtype=np.int64)
    i = idx % N
    j = (idx // N) % N
    k = idx // (N * N)
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, -6.0 * inv)]
    for di, dj, dk in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
        ok = ((i + di >= 0) & (i + di < N) & (j + dj >= 0) & (j + dj < N)
              & (k + dk >= 0) & (k + dk < N))
        rows.append(idx[ok])
        cols.append(idx[ok] + di + N * dj + N * N * dk)
        vals.append(np.full(int(ok.sum()), inv))
    return _csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)


def convdiff2d(N: int, vx: float, vy: float, D: float = 1.0) -> sp.csr_matrix:
    """D * Laplacian - (vx d/dx + vy d/dy) with backward (upwind) differences."""
    h = 1.0 / float(N + 1)
    d = D / (h * h)
    return stencil2d(N, -4.0 * d - (vx + vy) / h, d + vx / h, d, d + vy / h, d)


def smooth_field(N: int, seed: int, modes: int = 8) -> np.ndarray:
    """u(x,y) = sum_{k,l<=modes} a_kl sin(k pi x) sin(l pi y), a_kl ~ N(0,1)/(k^2+l^2),
    scaled so that max |u| = 1, sampled at the interior grid points."""
    g = rng(seed)
    a = g.standard_normal((modes, modes))
    x = np.arange(1, N + 1) / float(N + 1)
    kk = np.arange(1, modes + 1)
    a = a / (kk[:, None] ** 2 + kk[None, :] ** 2)
    Sx = np.sin(np.pi * np.outer(kk, x))           # modes x N
    U = Sx.T @ a @ Sx                               # U[i, j] = sum a_kl sin(k pi x_i) sin(l pi y_j)
    U = U / np.abs(U).max()
    return U.T.reshape(-1)                          # index i + N*j


def reaction2d(N: int, field_seed: int) -> sp.csr_matrix:
    h2 = 1.0 / float(N + 1) ** 2
    u = smooth_field(N, field_seed)
    return stencil2d(N, -4.0 / h2, 1.0 / h2, 1.0 / h2, 1.0 / h2, 1.0 / h2,
                     diag_extra=1.0 - 3.0 * u * u)


def sine_mode2d(N: int, k1: int, k2: int) -> tuple[np.ndarray, float]:
    """Unit-norm eigenvector of ``laplace2d(N)`` and its eigenvalue."""
    h = 1.0 / float(N + 1)
    x = np.arange(1, N + 1) * h
    v = np.outer(np.sin(k2 * math.pi * x), np.sin(k1 * math.pi * x)).reshape(-1)
    lam = -(4.0 / h ** 2) * (math.sin(k1 * math.pi * h / 2) ** 2 + math.sin(k2 * math.pi * h / 2) ** 2)
    return v / np.linalg.norm(v), lam


def heston(Ns: int = 100, Nv: int = 51, K: float = 100.0, S: float = 800.0, V: float = 5.0,
           kappa: float = 2.0, eta: float = 0.2, lam: float = 0.3, rho: float = 0.8,
           rd: float = 0.03, rf: float = 0.0):
    """Finite-difference Heston operator of the paper's Sect. 4.1: u' = A u + b1,
    u(0) = b0 (the call payoff).

    Grid: s_i = i ds (i = 1..Ns, ds = S/(Ns+1)) and v_j = j dv (j = 0..Nv-1,
    dv = V/Nv): v = 0 is a grid line, s = 0, s = S and v = V are not.  Unknown
    (i, j) has index (i-1) + Ns j.  Central second-order differences in the
    interior (the cross derivative by its four diagonal neighbours); on v = 0
    the boundary equation U_t = (rd - rf) s U_s + kappa eta U_v - rd U with
    the one-sided three-point U_v.  Boundary values: U(0, v) = 0, U(s, V) = s,
    and U(S, v) = U(s_Ns, v) + ds (the first-order form of U_s(S, v) = 1);
    known values go into b1.  Returns (A, b0, b1)."""
    ds = S / (Ns + 1)
    dv = V / Nv
    n = Ns * Nv
    rows, cols, vals = [], [], []
    b1 = np.zeros(n)

    def idx(i, j):
        return (i - 1) + Ns * j

    def add(k, i, j, c, s_i):
        # coefficient c on U(s_i, v_j); points off the grid are boundary values
        if c == 0.0:
            return
        if i == 0:                       # U(0, v) = 0
            return
        if j == Nv:                      # U(s, V) = s
            b1[k] += c * (i * ds if i <= Ns else S)
            return
        if i == Ns + 1:                  # U(S, v) = U(s_Ns, v) + ds
            rows.append(k); cols.append(idx(Ns, j)); vals.append(c)
            b1[k] += c * ds
            return
        rows.append(k); cols.append(idx(i, j)); vals.append(c)

    for j in range(Nv):
        v = j * dv
        for i in range(1, Ns + 1):
            s = i * ds
            k = idx(i, j)
            if j == 0:
                cs = (rd - rf) * s / (2 * ds)
                cv = kappa * eta / (2 * dv)
                add(k, i + 1, 0, cs, s)
                add(k, i - 1, 0, -cs, s)
                add(k, i, 0, -3 * cv - rd, s)
                add(k, i, 1, 4 * cv, s)
                add(k, i, 2, -cv, s)
                continue
            a_ss = 0.5 * v * s * s / (ds * ds)
            a_vv = 0.5 * lam * lam * v / (dv * dv)
            a_s = (rd - rf) * s / (2 * ds)
            a_v = kappa * (eta - v) / (2 * dv)
            a_sv = rho * lam * v * s / (4 * ds * dv)
            add(k, i, j, -2 * a_ss - 2 * a_vv - rd, s)
            add(k, i + 1, j, a_ss + a_s, s)
            add(k, i - 1, j, a_ss - a_s, s)
            add(k, i, j + 1, a_vv + a_v, s)
            add(k, i, j - 1, a_vv - a_v, s)
            add(k, i + 1, j + 1, a_sv, s)
            add(k, i - 1, j - 1, a_sv, s)
            add(k, i - 1, j + 1, -a_sv, s)
            add(k, i + 1, j - 1, -a_sv, s)
    A = _csr(np.array(rows), np.array(cols), np.array(vals), n)
    s_of = np.tile(np.arange(1, Ns + 1) * ds, Nv)
    b0 = np.maximum(s_of - K, 0.0)
    return A, b0, b1


# ------------------------------------------------------------------ configs

@dataclasses.dataclass
class Problem:
    name: str
    A: sp.csr_matrix
    b: np.ndarray          # n x (p+1)
    t: float
    tol: float
    symmetric: bool
    fp32_basis: bool = False

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def p(self) -> int:
        return self.b.shape[1] - 1


def config1() -> Problem:
    """2D Laplacian 30x30 (n=900), p=1, t=1e-3, tol=1e-7; b0 ~ N(0,1), b1 = 1."""
    A = laplace2d(30)
    g = rng(1000)
    b = np.stack([g.standard_normal(900), np.ones(900)], axis=1)
    return Problem("laplace2d-30x30-p1", A, b, 1e-3, 1e-7, True)


def config2() -> Problem:
    """Upwind convection-diffusion 512x512, D=1, v=(50,50), p=2, t=1e-2, tol=1e-8."""
    A = convdiff2d(512, 50.0, 50.0)
    g = rng(2000)
    b = g.standard_normal((A.shape[0], 3))
    return Problem("convdiff2d-512x512-p2", A, b, 1e-2, 1e-8, False)


def config3() -> Problem:
    """3D Laplacian 128^3 (n=2,097,152), p=3, t=1e-4, tol=1e-6, FP32 basis; b_k ~ U(-1,1)."""
    A = laplace3d(128)
    g = rng(3000)
    b = g.uniform(-1.0, 1.0, size=(A.shape[0], 4))
    return Problem("laplace3d-128^3-p3", A, b, 1e-4, 1e-6, True, fp32_basis=True)


def heston_problem(tol: float = 1e-6) -> Problem:
    """The paper's Heston example: u(1) = exp(A) b0 + phi_1(A) b1 on the 100 x 51
    grid (p = 1, t = T = 1)."""
    A, b0, b1 = heston()
    return Problem("heston-100x51", A, np.stack([b0, b1], axis=1), 1.0, tol, False)


def config5_matrix() -> sp.csr_matrix:
    return reaction2d(1024, 5999)


def config5_b(call: int, n: int = 1024 * 1024) -> np.ndarray:
    return rng(5000 + call).standard_normal((n, 3))


@dataclasses.dataclass
class BatchInstance:
    N: int
    peclet: float
    p: int
    t: float
    seed: int


def config4_specs(count: int = 256, seed0: int = 4000) -> list[BatchInstance]:
    out = []
    for i in range(count):
        g = rng(seed0 + i)
        N = int(g.integers(32, 257))
        pe = float(g.uniform(0.0, 100.0))
        p = int(g.integers(0, 4))
        t = float(10.0 ** g.uniform(-4.0, -1.0))
        out.append(BatchInstance(N, pe, p, t, seed0 + i))
    return out


def config4_problem(spec: BatchInstance, tol: float = 1e-7) -> Problem:
    v = spec.peclet / math.sqrt(2.0)
    A = convdiff2d(spec.N, v, v)
    g = rng(spec.seed + 100000)
    b = g.standard_normal((A.shape[0], spec.p + 1))
    return Problem(f"convdiff2d-{spec.N}-pe{spec.peclet:.1f}-p{spec.p}", A, b, spec.t, tol,
                   False, fp32_basis=True)


def random_sparse(n: int, density: float, seed: int, symmetric: bool = False,
                  shift: float = 0.0) -> sp.csr_matrix:
    """Small random sparse test matrix with a full diagonal (optionally symmetric)."""
    g = rng(seed)
    M = sp.random(n, n, density=density, random_state=g, data_rvs=g.standard_normal, format="csr")
    M = M + sp.diags(g.standard_normal(n) + shift)
    if symmetric:
        M = (M + M.T) * 0.5
    M = sp.csr_matrix(M)
    return _csr(*_coo(M), n)


def _coo(M):
    C = M.tocoo()
    return C.row, C.col, C.data
