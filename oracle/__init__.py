"""CPU oracle for the adaptive Krylov phi-function solver (Niesen & Wright).

TEST INFRASTRUCTURE ONLY.  A plain double-precision C implementation of
Algorithms 3 and 4 of the paper (with eqs. tau_0, taunew, 2-8, errest,
phipapprox2, step, wrecurrence), loaded through ctypes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package; the GPU library never does.  It shares no code with the GPU path.

Parity status per function is listed in ``oracle.h``.  The controller's
step-by-step trajectory has no printed worked example: parity unpinned.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "phipm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


# -O3 for an x86-64 baseline with AVX2 (every current server CPU; the library
# is built once and may run on another host); no contraction of a*b + c into
# fused multiply-adds, so the arithmetic is the plain one the source spells
# out on every machine.
CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-std=c11", "-D_GNU_SOURCE",
          "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP; CFLAGS)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("symm", C.c_int32), ("m_init", C.c_int32),
                ("m_max", C.c_int32), ("reorth", C.c_int32), ("adapt_m", C.c_int32),
                ("corrector", C.c_int32), ("pad_", C.c_int32), ("tau_fixed", C.c_double),
                ("max_attempts", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rejected", C.c_int64), ("matvecs", C.c_int64),
                ("expms", C.c_int64), ("t_reached", C.c_double), ("tau_last", C.c_double),
                ("m_last", C.c_int32), ("status", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TraceRec(C.Structure):
    _fields_ = [("t", C.c_double), ("tau", C.c_double), ("eps", C.c_double),
                ("omega", C.c_double), ("beta", C.c_double), ("hnext", C.c_double),
                ("anorm", C.c_double), ("tau_next", C.c_double), ("m", C.c_int32),
                ("accepted", C.c_int32), ("step", C.c_int32), ("m_next", C.c_int32),
                ("branch", C.c_int32), ("have", C.c_int32)]


class Attempt(C.Structure):
    _fields_ = [("tau", C.c_double), ("eps", C.c_double), ("omega", C.c_double),
                ("knorm", C.c_double), ("rem", C.c_double), ("nnz", C.c_double),
                ("n", C.c_double), ("m_use", C.c_int32), ("m_req", C.c_int32),
                ("m_cap", C.c_int32), ("lanczos", C.c_int32), ("p", C.c_int32),
                ("adapt_m", C.c_int32), ("broke", C.c_int32), ("tau_fixed", C.c_int32)]


class Decision(C.Structure):
    _fields_ = [("tau_next", C.c_double), ("tau_new", C.c_double), ("m_new", C.c_double),
                ("accept", C.c_int32), ("branch", C.c_int32), ("m_next", C.c_int32),
                ("pad_", C.c_int32)]


class Alg4State(C.Structure):
    _fields_ = [("prev_rejected", C.c_int32), ("prev_branch", C.c_int32),
                ("q_valid", C.c_int32), ("k_valid", C.c_int32), ("q_hat", C.c_double),
                ("k_hat", C.c_double), ("eps_old", C.c_double), ("tau_old", C.c_double),
                ("m_old", C.c_int32), ("pad_", C.c_int32)]


class LabelCosts(C.Structure):
    _fields_ = [("sync_s", C.c_double), ("sync1_s", C.c_double), ("bw_bytes_per_s", C.c_double),
                ("wg_bytes_per_s", C.c_double), ("workgroups", C.c_int32), ("pad_", C.c_int32),
                ("expm_s", C.c_double * 138)]


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.oracle_default_opts.argtypes = [C.POINTER(Opts)]
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_phi.argtypes = [C.c_int, C.c_double]
        L.oracle_phi.restype = C.c_double
        L.oracle_expm.argtypes = [C.c_int, _dp, _dp]
        L.oracle_expm.restype = C.c_int
        L.oracle_spmv.argtypes = [C.c_int, _ip, _ip, _dp, _dp, _dp]
        L.oracle_is_symmetric.argtypes = [C.c_int, _ip, _ip, _dp]
        L.oracle_is_symmetric.restype = C.c_int
        L.oracle_krylov.argtypes = [C.c_int, _ip, _ip, _dp, _dp, C.c_int, C.c_int, C.c_int,
                                    _dp, _dp, C.POINTER(C.c_double)]
        L.oracle_krylov.restype = C.c_int
        L.oracle_tau0.argtypes = [C.c_double] * 4
        L.oracle_tau0.restype = C.c_double
        L.oracle_cost_M.argtypes = [C.c_double]
        L.oracle_cost_M.restype = C.c_double
        L.oracle_cost_C1.argtypes = [C.c_int, C.c_double, C.c_int, C.c_double, C.c_double,
                                     C.c_double]
        L.oracle_cost_C1.restype = C.c_double
        L.oracle_cost_C.argtypes = [C.c_double] * 3
        L.oracle_cost_C.restype = C.c_double
        L.oracle_alg4.argtypes = [C.POINTER(Alg4State), C.c_double, C.c_int, C.c_double,
                                  C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_decide.argtypes = [C.POINTER(Alg4State), C.POINTER(Attempt),
                                    C.POINTER(Decision)]
        L.oracle_decide.restype = None
        L.oracle_phipm.argtypes = [C.c_double, C.c_int, _ip, _ip, _dp, C.c_int, _dp,
                                   C.POINTER(Opts), _dp, C.POINTER(Stats),
                                   C.c_void_p, C.c_int, C.POINTER(C.c_int)]
        L.oracle_phipm.restype = C.c_int
        L.oracle_step.argtypes = [C.c_int, _ip, _ip, _dp, C.c_int, _dp, C.c_double, _dp,
                                  C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, _dp,
                                  C.POINTER(C.c_double)]
        L.oracle_step.restype = C.c_int
        L.oracle_gelu.argtypes = [C.c_double]
        L.oracle_gelu.restype = C.c_double
        L.oracle_gelu_grad.argtypes = [C.c_double]
        L.oracle_gelu_grad.restype = C.c_double
        L.oracle_mlp_params.argtypes = []
        L.oracle_mlp_params.restype = C.c_int
        L.oracle_mlp_forward.argtypes = [_dp, _dp, C.c_int, _dp]
        L.oracle_mlp_forward.restype = None
        L.oracle_mlp_loss_grad.argtypes = [_dp, _dp, _dp, C.c_int, C.c_void_p]
        L.oracle_mlp_loss_grad.restype = C.c_double
        L.oracle_adam_step.argtypes = [_dp, _dp, _dp, _dp, C.c_int, C.c_double, C.c_longlong]
        L.oracle_adam_step.restype = None
        L.oracle_step_omega.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.POINTER(C.c_double)]
        L.oracle_step_omega.restype = C.c_double
        L.oracle_step_time.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                       C.POINTER(LabelCosts)]
        L.oracle_step_time.restype = C.c_double
        L.oracle_label_step.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                        C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.c_double,
                                        C.POINTER(LabelCosts), C.POINTER(C.c_double),
                                        C.POINTER(C.c_int)]
        L.oracle_label_step.restype = None
        _lib = L
    return _lib


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().oracle_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def phi(k: int, z: float) -> float:
    return lib().oracle_phi(int(k), float(z))


def expm(A: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    E = np.empty_like(A)
    lib().oracle_expm(A.shape[0], A, E)
    return E


def _csr(A):
    rp = np.ascontiguousarray(A.indptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.indices, dtype=np.int32)
    va = np.ascontiguousarray(A.data, dtype=np.float64)
    if va.size == 0:
        va = np.zeros(1)
        ci = np.zeros(1, dtype=np.int32)
    return rp, ci, va


def spmv(A, x) -> np.ndarray:
    rp, ci, va = _csr(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.shape[0])
    lib().oracle_spmv(A.shape[0], rp, ci, va, x, y)
    return y


def is_symmetric(A) -> bool:
    rp, ci, va = _csr(A)
    return bool(lib().oracle_is_symmetric(A.shape[0], rp, ci, va))


def krylov(A, v, m: int, lanczos: bool, reorth: int = 1):
    rp, ci, va = _csr(A)
    n = A.shape[0]
    v = np.ascontiguousarray(v, dtype=np.float64)
    V = np.zeros((m + 1) * n)
    H = np.zeros((m + 1) * m)
    beta = C.c_double()
    mm = lib().oracle_krylov(n, rp, ci, va, v, m, int(lanczos), int(reorth), V, H,
                             C.byref(beta))
    return V.reshape(m + 1, n).T.copy(), H.reshape(m + 1, m), beta.value, mm


def tau0(tol, anorm, bnorm, m_ave):
    return lib().oracle_tau0(tol, anorm, bnorm, m_ave)


def cost_M(norm1):
    return lib().oracle_cost_M(norm1)


def cost_C1(lanczos, m, p, nnz, n, M):
    return lib().oracle_cost_C1(int(lanczos), float(m), int(p), float(nnz), float(n), float(M))


def cost_C(remaining, tau, C1):
    return lib().oracle_cost_C(remaining, tau, C1)


def alg4(state: Alg4State, tau, m, eps, omega):
    tn, mn, q, k = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    lib().oracle_alg4(C.byref(state), tau, int(m), eps, omega, C.byref(tn), C.byref(mn),
                      C.byref(q), C.byref(k))
    return tn.value, mn.value, q.value, k.value


def decide(state: Alg4State, **attempt):
    """Algorithm 3's decision after one attempt; attempt fields as in
    ``Attempt`` (m_req defaults to m_use, m_cap to 100, adapt_m to 1).
    Returns a dict with accept, branch, tau_next, m_next, tau_new, m_new."""
    a = Attempt()
    a.m_cap, a.adapt_m = 100, 1
    for k, v in attempt.items():
        setattr(a, k, v)
    if "m_req" not in attempt:
        a.m_req = a.m_use
    d = Decision()
    lib().oracle_decide(C.byref(state), C.byref(a), C.byref(d))
    return {"accept": bool(d.accept), "branch": d.branch, "tau_next": d.tau_next,
            "m_next": d.m_next, "tau_new": d.tau_new, "m_new": d.m_new}


def threads() -> int:
    return lib().oracle_threads()


def set_threads(k: int) -> None:
    """Threads of the OpenMP loops from now on (results do not depend on it)."""
    lib().oracle_set_threads(int(k))


def phipm(t, A, b, opts: Opts | None = None, trace_cap: int = 0, allow_limit: bool = False,
          **kw):
    """u = sum_k t^k phi_k(tA) b_k; b is n x (p+1).  Returns (u, stats[, trace]).
    allow_limit: return normally when the attempt limit stops the solve."""
    if opts is None:
        opts = default_opts(**kw)
    rp, ci, va = _csr(A)
    n = A.shape[0]
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        b = b[:, None]
    p = b.shape[1] - 1
    bcm = np.ascontiguousarray(b.T).reshape(-1)
    u = np.empty(n)
    st = Stats()
    tl = C.c_int(0)
    tr = (TraceRec * trace_cap)() if trace_cap > 0 else None
    rc = lib().oracle_phipm(float(t), n, rp, ci, va, p, bcm, C.byref(opts), u, C.byref(st),
                            C.cast(tr, C.c_void_p) if tr is not None else None, trace_cap,
                            C.byref(tl))
    if rc != 0 and not (allow_limit and rc == -5):
        raise RuntimeError(f"oracle_phipm failed with status {rc}")
    if trace_cap > 0:
        recs = [{k: getattr(tr[i], k) for k, _ in TraceRec._fields_} for i in range(tl.value)]
        return u, st.as_dict(), recs
    return u, st.as_dict()


def step(A, b, t_k, u_k, tau, m, lanczos, reorth=1, corrector=1):
    rp, ci, va = _csr(A)
    n = A.shape[0]
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        b = b[:, None]
    p = b.shape[1] - 1
    bcm = np.ascontiguousarray(b.T).reshape(-1)
    out = np.empty(n)
    eps = C.c_double()
    lib().oracle_step(n, rp, ci, va, p, bcm, float(t_k),
                      np.ascontiguousarray(u_k, dtype=np.float64), float(tau), int(m),
                      int(lanczos), int(reorth), int(corrector), out, C.byref(eps))
    return out, eps.value


# ------------------------------------------------------------ proposer references

def gelu(z):
    return lib().oracle_gelu(float(z))


def gelu_grad(z):
    return lib().oracle_gelu_grad(float(z))


def mlp_forward(P, X):
    P = np.ascontiguousarray(P, dtype=np.float64)
    X = np.ascontiguousarray(np.atleast_2d(X), dtype=np.float64)
    Y = np.empty((X.shape[0], 2))
    lib().oracle_mlp_forward(P, X, X.shape[0], Y)
    return Y


def mlp_loss_grad(P, X, T, want_grad=True):
    P = np.ascontiguousarray(P, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    g = np.zeros(P.size) if want_grad else None
    L = lib().oracle_mlp_loss_grad(P, X, T, X.shape[0],
                                   g.ctypes.data_as(C.c_void_p) if want_grad else None)
    return (L, g) if want_grad else L


def adam_step(P, m, v, g, lr, t):
    P, m, v = (np.array(a, dtype=np.float64) for a in (P, m, v))
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().oracle_adam_step(P, m, v, g, P.size, float(lr), int(t))
    return P, m, v


def step_omega(H, mm, p, beta, tau, t_end, tol):
    H = np.ascontiguousarray(H, dtype=np.float64)
    kn = C.c_double()
    w = lib().oracle_step_omega(H, H.shape[1], int(mm), int(p), float(beta), float(tau),
                                float(t_end), float(tol), C.byref(kn))
    return w, kn.value


def label_costs(sync_s, sync1_s, bw, wg_bw, workgroups, expm_s):
    c = LabelCosts()
    c.sync_s, c.sync1_s, c.bw_bytes_per_s, c.wg_bytes_per_s = sync_s, sync1_s, bw, wg_bw
    c.workgroups = int(workgroups)
    for i, v in enumerate(expm_s):
        c.expm_s[i] = float(v)
    return c


def step_time(mm, p, lanczos, n, nnz, costs):
    return lib().oracle_step_time(int(mm), int(p), int(lanczos), float(n), float(nnz),
                                  C.byref(costs))


def label_step(H, m_use, m_have, p, lanczos, n, nnz, t, tau, beta, t_end, tol, costs=None):
    """H: (m_have+1) x ldh row-major array; costs: LabelCosts or None (eq. 4)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    ts, ms = C.c_double(), C.c_int()
    lib().oracle_label_step(H, H.shape[1], int(m_use), int(m_have), int(p), int(lanczos),
                            float(n), float(nnz), float(t), float(tau), float(beta),
                            float(t_end), float(tol), C.byref(costs) if costs else None,
                            C.byref(ts), C.byref(ms))
    return ts.value, ms.value
