"""phipm on MI355X: Python binding of the C ABI in ``include/phipm.h``.

Argument marshalling only: torch tensors supply device memory and the stream;
every step of the computation runs in the HIP library ``libphipm.so``.  The
binding raises if that library is missing; there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphipm.so")

OK, EINVAL, ENOMEM, EHIP, ENONFINITE, EMAXSTEPS, EUNSUPPORTED, EABORT = 0, -1, -2, -3, -4, -5, -6, -7
ESCRATCH = -8
FP64, FP32_BASIS = 0, 1
F64, F32 = 0, 1                        # CSR value types (phipm_csr.val_dtype)
REORTH_LOCAL, REORTH_FULL = 0, 1
FP32_ONLY = 1
M_CAP, P_MAX = 128, 8
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 12, 64, 2, 5122


class PhipmError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = status_string(status) if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


class CSR(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p), ("val_dtype", C.c_int32),
                ("pad_", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("symm", C.c_int32), ("m_init", C.c_int32),
                ("m_max", C.c_int32), ("precision", C.c_int32), ("adapt_m", C.c_int32),
                ("corrector", C.c_int32), ("tau_fixed", C.c_double),
                ("max_attempts", C.c_int64), ("workgroups", C.c_int32),
                ("validate", C.c_int32), ("proposer", C.c_void_p), ("history", C.c_void_p),
                ("trace", C.c_void_p), ("trace_cap", C.c_int32), ("reorth", C.c_int32),
                ("fp32_flags", C.c_int32), ("pad_", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rejected", C.c_int64), ("matvecs", C.c_int64),
                ("expms", C.c_int64), ("t_reached", C.c_double), ("tau_last", C.c_double),
                ("m_last", C.c_int32), ("status", C.c_int32), ("lanczos", C.c_int32),
                ("workgroups", C.c_int32), ("anorm", C.c_double), ("setup_flags", C.c_int32),
                ("pad_", C.c_int32), ("bytes", C.c_double), ("phi_ratio_max", C.c_double),
                ("precision_rejects", C.c_int64), ("fp32_error_estimate", C.c_double),
                ("fp64_steps", C.c_int32), ("trace_len", C.c_int32),
                ("proposals", C.c_int64), ("bytes_ref", C.c_double),
                ("krylov_bytes_ref", C.c_double), ("krylov_seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TraceStep(C.Structure):
    """phipm_trace_step (records live in device memory; this describes them)."""
    _fields_ = [("features", C.c_float * MLP_IN), ("m_use", C.c_int32), ("m_have", C.c_int32),
                ("p", C.c_int32), ("lanczos", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int32),
                ("attempts", C.c_int32), ("pad_", C.c_int32), ("t", C.c_double),
                ("tau", C.c_double), ("omega", C.c_double), ("beta", C.c_double),
                ("anorm", C.c_double), ("t_end", C.c_double), ("tol", C.c_double),
                ("pad2_", C.c_double), ("H", C.c_double * ((M_CAP + 1) * M_CAP))]


class LabelCosts(C.Structure):
    """phipm_label_costs: device time model of one step (hindsight labels)."""
    _fields_ = [("sync_s", C.c_double), ("sync1_s", C.c_double), ("bw_bytes_per_s", C.c_double),
                ("wg_bytes_per_s", C.c_double), ("workgroups", C.c_int32), ("pad_", C.c_int32),
                ("expm_s", C.c_double * (M_CAP + P_MAX + 2))]


class PlanOpts(C.Structure):
    _fields_ = [("autotune", C.c_int32), ("graph", C.c_int32), ("max_team", C.c_int32),
                ("pad_", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("count", C.c_int32), ("workgroups", C.c_int32), ("teams", C.c_int32),
                ("classes", C.c_int32), ("class_size", C.c_int32 * 8),
                ("class_teams", C.c_int32 * 8), ("graph", C.c_int32),
                ("cooperative", C.c_int32), ("candidates", C.c_int32), ("max_team", C.c_int32),
                ("alpha", C.c_double), ("tuned_ms", C.c_double), ("default_ms", C.c_double),
                ("device_bytes", C.c_uint64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        nc = self.classes
        d["class_size"] = list(self.class_size)[:nc]
        d["class_teams"] = list(self.class_teams)[:nc]
        return d


_lib = None

EXPORTS = ["phipm_default_opts", "phipm_workspace_bytes", "phipm", "phipm_last_status",
           "phipm_spmv", "phipm_expm", "phipm_krylov", "phipm_status_string",
           "phipm_default_plan_opts", "phipm_plan_create", "phipm_plan_execute",
           "phipm_plan_stats", "phipm_plan_get_info", "phipm_plan_destroy", "phipm_batched",
           "phipm_batch_layout", "phipm_mlp_forward", "phipm_mlp_grad", "phipm_mlp_train",
           "phipm_label_workspace_bytes", "phipm_label_steps", "phipm_allen_cahn_update",
           "phipm_noalloc", "phipm_noalloc_scratch_bytes"]


def lib():
    """Load libphipm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.phipm_default_opts.argtypes = [C.POINTER(Opts)]
        L.phipm_default_opts.restype = None
        L.phipm_workspace_bytes.argtypes = [C.POINTER(CSR), C.c_int, C.POINTER(Opts),
                                            C.POINTER(C.c_size_t)]
        L.phipm_workspace_bytes.restype = C.c_int
        L.phipm.argtypes = [C.c_double, C.POINTER(CSR), C.c_int, vp, C.POINTER(Opts), vp, vp,
                            C.c_size_t, C.POINTER(Stats), vp]
        L.phipm.restype = C.c_int
        L.phipm_noalloc.argtypes = [C.c_double, C.POINTER(CSR), C.c_int, vp, C.POINTER(Opts), vp,
                                    C.POINTER(Stats), vp]
        L.phipm_noalloc.restype = C.c_int
        L.phipm_noalloc_scratch_bytes.argtypes = []
        L.phipm_noalloc_scratch_bytes.restype = C.c_size_t
        L.phipm_last_status.argtypes = []
        L.phipm_last_status.restype = C.c_int
        L.phipm_spmv.argtypes = [C.POINTER(CSR), vp, vp, vp]
        L.phipm_spmv.restype = C.c_int
        L.phipm_expm.argtypes = [C.c_int, vp, vp, vp, vp]
        L.phipm_expm.restype = C.c_int
        L.phipm_krylov.argtypes = [C.POINTER(CSR), vp, C.c_int, C.c_int, vp, vp, vp, C.c_size_t,
                                   C.POINTER(C.c_int), vp]
        L.phipm_krylov.restype = C.c_int
        L.phipm_status_string.argtypes = [C.c_int]
        L.phipm_status_string.restype = C.c_char_p
        L.phipm_default_plan_opts.argtypes = [C.POINTER(PlanOpts)]
        L.phipm_default_plan_opts.restype = None
        plan_args = [C.c_int, C.POINTER(CSR), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                     C.POINTER(vp), C.POINTER(vp), C.POINTER(Opts)]
        L.phipm_plan_create.argtypes = plan_args + [C.POINTER(PlanOpts), vp, C.POINTER(vp)]
        L.phipm_plan_create.restype = C.c_int
        L.phipm_plan_execute.argtypes = [vp, vp]
        L.phipm_plan_execute.restype = C.c_int
        L.phipm_plan_stats.argtypes = [vp, C.POINTER(Stats)]
        L.phipm_plan_stats.restype = C.c_int
        L.phipm_plan_get_info.argtypes = [vp, C.POINTER(PlanInfo)]
        L.phipm_plan_get_info.restype = C.c_int
        L.phipm_plan_destroy.argtypes = [vp]
        L.phipm_plan_destroy.restype = C.c_int
        L.phipm_batched.argtypes = plan_args + [C.POINTER(Stats), vp]
        L.phipm_batched.restype = C.c_int
        ip = C.POINTER(C.c_int32)
        L.phipm_batch_layout.argtypes = [C.c_int, C.POINTER(C.c_double), C.c_int, C.c_int,
                                         C.c_double, ip, ip, ip, ip, ip, ip]
        L.phipm_batch_layout.restype = C.c_int
        L.phipm_mlp_forward.argtypes = [vp, vp, C.c_int, vp, vp]
        L.phipm_mlp_forward.restype = C.c_int
        L.phipm_mlp_grad.argtypes = [vp, vp, vp, C.c_int, vp, vp, vp]
        L.phipm_mlp_grad.restype = C.c_int
        L.phipm_mlp_train.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_float,
                                      C.c_int, vp, vp]
        L.phipm_mlp_train.restype = C.c_int
        L.phipm_label_workspace_bytes.argtypes = [C.c_int]
        L.phipm_label_workspace_bytes.restype = C.c_size_t
        L.phipm_label_steps.argtypes = [vp, C.c_int, vp, vp, vp, C.c_size_t,
                                        C.POINTER(LabelCosts), vp]
        L.phipm_label_steps.restype = C.c_int
        L.phipm_allen_cahn_update.argtypes = [C.POINTER(CSR), vp, vp, vp, vp, vp, vp, vp]
        L.phipm_allen_cahn_update.restype = C.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().phipm_status_string(int(status)).decode()


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().phipm_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class DeviceCSR:
    """A CSR matrix resident on the GPU (int32 indices; float64 values, or
    float32 with dtype=np.float32, which the solver then reads as they are:
    the matrix is the float32-rounded one)."""

    def __init__(self, A, device="cuda", dtype=np.float64):
        torch = _torch()
        dtype = np.dtype(dtype)
        if dtype not in (np.dtype(np.float64), np.dtype(np.float32)):
            raise ValueError("CSR values must be float64 or float32")
        self.val_dtype = F32 if dtype == np.float32 else F64
        self.n = int(A.shape[0])
        self.nnz = int(A.nnz)
        self.row_ptr = torch.as_tensor(np.asarray(A.indptr, dtype=np.int32), device=device)
        self.col_idx = torch.as_tensor(np.asarray(A.indices, dtype=np.int32), device=device)
        self.val = torch.as_tensor(np.asarray(A.data, dtype=dtype), device=device)
        if self.nnz == 0:   # keep non-null pointers
            self.col_idx = torch.zeros(1, dtype=torch.int32, device=device)
            self.val = torch.zeros(1, dtype=self.val.dtype, device=device)

    def c(self) -> CSR:
        return CSR(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                   self.val.data_ptr(), self.val_dtype, 0)


def workspace_bytes(A: DeviceCSR, p: int, opts: Opts) -> int:
    nb = C.c_size_t()
    rc = lib().phipm_workspace_bytes(C.byref(A.c()), int(p), C.byref(opts), C.byref(nb))
    if rc != OK:
        raise PhipmError(rc, "phipm_workspace_bytes")
    return nb.value


def alloc_workspace(nbytes: int, device="cuda"):
    torch = _torch()
    return torch.empty(nbytes + 256, dtype=torch.uint8, device=device)


def _aligned(ws):
    ptr = ws.data_ptr()
    return (ptr + 255) & ~255


class Solver:
    """Reusable solver: owns a workspace sized for (A, p, opts)."""

    def __init__(self, A: DeviceCSR, p: int, opts: Opts | None = None, **kw):
        self.A = A
        self.p = int(p)
        self.opts = opts if opts is not None else default_opts(**kw)
        self.ws_bytes = workspace_bytes(A, self.p, self.opts)
        self.ws = alloc_workspace(self.ws_bytes, device=A.row_ptr.device)
        self.csr = A.c()

    def __call__(self, t, b, u, stats: bool = True, stream=None):
        """u <- sum_k t^k phi_k(tA) b_k.  b: (p+1, n) float64 tensor, rows = b_k."""
        torch = _torch()
        assert b.dtype == torch.float64 and u.dtype == torch.float64
        assert b.is_contiguous() and b.shape == (self.p + 1, self.A.n) and u.numel() == self.A.n
        st = Stats()
        rc = lib().phipm(float(t), C.byref(self.csr), self.p, C.c_void_p(b.data_ptr()),
                         C.byref(self.opts), C.c_void_p(u.data_ptr()),
                         C.c_void_p(_aligned(self.ws)), self.ws_bytes,
                         C.byref(st) if stats else None, _stream_ptr(stream))
        if rc != OK:
            raise PhipmError(rc, "phipm")
        return st.as_dict() if stats else None


def solve(t, A: DeviceCSR, b, opts: Opts | None = None, **kw):
    """One-shot u = sum_k t^k phi_k(tA) b_k for b given as (p+1, n) tensor."""
    torch = _torch()
    p = b.shape[0] - 1
    s = Solver(A, p, opts, **kw)
    u = torch.empty(A.n, dtype=torch.float64, device=b.device)
    st = s(t, b, u)
    return u, st


def solve_noalloc(t, A: DeviceCSR, b, u, opts: Opts | None = None, stats: bool = True,
                  stream=None, **kw):
    """u <- sum_k t^k phi_k(tA) b_k with phipm_noalloc (the library's fixed
    device scratch, no allocation).  b: (p+1, n) float64 tensor."""
    torch = _torch()
    assert b.dtype == torch.float64 and u.dtype == torch.float64 and b.is_contiguous()
    o = opts if opts is not None else default_opts(**kw)
    st = Stats()
    rc = lib().phipm_noalloc(float(t), C.byref(A.c()), int(b.shape[0] - 1),
                             C.c_void_p(b.data_ptr()), C.byref(o), C.c_void_p(u.data_ptr()),
                             C.byref(st) if stats else None, _stream_ptr(stream))
    if rc != OK:
        raise PhipmError(rc, "phipm_noalloc")
    return st.as_dict() if stats else None


def spmv(A: DeviceCSR, x, y, stream=None):
    rc = lib().phipm_spmv(C.byref(A.c()), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                          _stream_ptr(stream))
    if rc != OK:
        raise PhipmError(rc, "phipm_spmv")


def allen_cahn_update(L: DeviceCSR, u, du=None, diag_pos=None, lap_diag=None, J_val=None,
                      F=None, stream=None):
    """phipm_allen_cahn_update: u += du, F = L u + (u - u^3), and the Jacobian's
    diagonal lap_diag + (1 - 3 u^2) into J_val at diag_pos (int32); None skips."""
    p = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    rc = lib().phipm_allen_cahn_update(C.byref(L.c()), p(u), p(du), p(diag_pos), p(lap_diag),
                                       p(J_val), p(F), _stream_ptr(stream))
    if rc != OK:
        raise PhipmError(rc, "phipm_allen_cahn_update")


def expm(H, stream=None):
    """exp(H) of a square float64 device tensor with the solver's small exponential."""
    torch = _torch()
    N = H.shape[0]
    H = H.contiguous()
    E = torch.empty_like(H)
    S = torch.empty(8 * N * N, dtype=torch.float64, device=H.device)
    rc = lib().phipm_expm(N, C.c_void_p(H.data_ptr()), C.c_void_p(E.data_ptr()),
                          C.c_void_p(S.data_ptr()), _stream_ptr(stream))
    if rc != OK:
        raise PhipmError(rc, "phipm_expm")
    return E


def krylov(A: DeviceCSR, v, m: int, lanczos: bool, stream=None):
    """m steps of the solver's Krylov process from v.  Returns (V n x (m+1), H (m+1) x m, done)."""
    torch = _torch()
    opts = default_opts(m_max=max(m, 10), m_init=1)
    nb = workspace_bytes(A, 0, opts)
    ws = alloc_workspace(nb, device=v.device)
    V = torch.zeros((m + 1) * A.n, dtype=torch.float64, device=v.device)
    H = torch.zeros((m + 1) * m, dtype=torch.float64, device=v.device)
    done = C.c_int()
    rc = lib().phipm_krylov(C.byref(A.c()), C.c_void_p(v.data_ptr()), int(m), int(lanczos),
                            C.c_void_p(V.data_ptr()), C.c_void_p(H.data_ptr()),
                            C.c_void_p(_aligned(ws)), nb, C.byref(done), _stream_ptr(stream))
    if rc != OK:
        raise PhipmError(rc, "phipm_krylov")
    return V.view(m + 1, A.n).T, H.view(m + 1, m), done.value


def default_plan_opts(**kw) -> PlanOpts:
    o = PlanOpts()
    lib().phipm_default_plan_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _batch_arrays(As, ps, ts, bs, us):
    torch = _torch()
    count = len(As)
    if not (len(ps) == len(ts) == len(bs) == len(us) == count):
        raise ValueError("instance lists differ in length")
    for A, p, b, u in zip(As, ps, bs, us):
        if b.dtype != torch.float64 or u.dtype != torch.float64:
            raise TypeError("b and u must be float64")
        if not b.is_contiguous() or tuple(b.shape) != (int(p) + 1, A.n) or u.numel() != A.n:
            raise ValueError("b must be a contiguous (p+1, n) tensor and u an n-vector")
    csr = (CSR * count)(*[A.c() for A in As])
    pa = (C.c_int32 * count)(*[int(p) for p in ps])
    ta = (C.c_double * count)(*[float(t) for t in ts])
    ba = (C.c_void_p * count)(*[b.data_ptr() for b in bs])
    ua = (C.c_void_p * count)(*[u.data_ptr() for u in us])
    return csr, pa, ta, ba, ua


class Plan:
    """Many solves in one persistent launch (``phipm_plan_*``).

    As: DeviceCSR list; ps: p_i; ts: t_i; bs: (p_i+1, n_i) float64 tensors;
    us: n_i float64 output tensors.  The plan keeps references to every
    tensor it was given, so they stay allocated while it lives."""

    def __init__(self, As, ps, ts, bs, us, opts: Opts | None = None,
                 plan_opts: PlanOpts | None = None, stream=None, **kw):
        self._keep = (list(As), list(bs), list(us))
        self.count = len(As)
        self.opts = opts if opts is not None else default_opts(**kw)
        self.plan_opts = plan_opts if plan_opts is not None else default_plan_opts()
        arrs = _batch_arrays(As, ps, ts, bs, us)
        self._arrs = arrs
        h = C.c_void_p()
        rc = lib().phipm_plan_create(self.count, *arrs, C.byref(self.opts),
                                     C.byref(self.plan_opts), _stream_ptr(stream), C.byref(h))
        if rc != OK:
            raise PhipmError(rc, "phipm_plan_create")
        self._h = h
        _LIVE_PLANS.add(self)

    def execute(self, stream=None):
        rc = lib().phipm_plan_execute(self._h, _stream_ptr(stream))
        if rc != OK:
            raise PhipmError(rc, "phipm_plan_execute")

    def stats(self, check: bool = True):
        st = (Stats * self.count)()
        rc = lib().phipm_plan_stats(self._h, st)
        if check and rc != OK:
            raise PhipmError(rc, "phipm_plan_stats")
        return [s.as_dict() for s in st]

    def info(self):
        inf = PlanInfo()
        rc = lib().phipm_plan_get_info(self._h, C.byref(inf))
        if rc != OK:
            raise PhipmError(rc, "phipm_plan_get_info")
        return inf.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib().phipm_plan_destroy(self._h)
            self._h = None
        _LIVE_PLANS.discard(self)

    def __del__(self):
        # no HIP calls while the interpreter shuts down: live plans are
        # released by _close_live_plans() while the runtime is still up
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


# Plans still open when the interpreter exits are released by an atexit
# handler, which runs before the C-level exit handlers tear down the HIP
# runtime (and any profiler attached to it).
_LIVE_PLANS = weakref.WeakSet()


@atexit.register
def _close_live_plans():
    for pl in list(_LIVE_PLANS):
        try:
            pl.close()
        except Exception:
            pass


def solve_batched(As, ps, ts, bs, us, opts: Opts | None = None, stream=None, **kw):
    """One-off batched solve (``phipm_batched``); returns per-instance stats."""
    o = opts if opts is not None else default_opts(**kw)
    arrs = _batch_arrays(As, ps, ts, bs, us)
    st = (Stats * len(As))()
    rc = lib().phipm_batched(len(As), *arrs, C.byref(o), st, _stream_ptr(stream))
    if rc != OK:
        raise PhipmError(rc, "phipm_batched")
    return [s.as_dict() for s in st]


def batch_layout(cost, workgroups: int, max_team: int, alpha: float):
    """The planner's team layout for per-instance costs (host only, no GPU).
    Returns dict(team_size, team_class, order, qbeg)."""
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    count = cost.size
    ts = np.zeros(max(1, workgroups), dtype=np.int32)
    tc = np.zeros_like(ts)
    order = np.zeros(max(1, count), dtype=np.int32)
    qbeg = np.zeros(max(1, workgroups) + 1, dtype=np.int32)
    nt, nc = C.c_int32(), C.c_int32()
    ip = C.POINTER(C.c_int32)
    rc = lib().phipm_batch_layout(int(count), cost.ctypes.data_as(C.POINTER(C.c_double)),
                                  int(workgroups), int(max_team), float(alpha),
                                  ts.ctypes.data_as(ip), tc.ctypes.data_as(ip), C.byref(nt),
                                  order.ctypes.data_as(ip), qbeg.ctypes.data_as(ip), C.byref(nc))
    if rc != OK:
        raise PhipmError(rc, "phipm_batch_layout")
    return {"team_size": ts[:nt.value].copy(), "team_class": tc[:nt.value].copy(),
            "order": order[:count].copy(), "qbeg": qbeg[:nc.value + 1].copy()}


# ------------------------------------------------------------ proposer kernels

def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _check_f32(*ts):
    torch = _torch()
    for t in ts:
        if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
            raise TypeError("expected contiguous float32 device tensors")


def mlp_forward(params, X, stream=None):
    """Y = MLP(X), X: (rows, 12) float32 device tensor."""
    torch = _torch()
    _check_f32(params, X)
    rows = X.shape[0]
    Y = torch.empty((rows, MLP_OUT), dtype=torch.float32, device=X.device)
    rc = lib().phipm_mlp_forward(_ptr(params), _ptr(X), rows, _ptr(Y), _stream_ptr(stream))
    if rc != OK:
        raise PhipmError(rc, "phipm_mlp_forward")
    return Y


def mlp_grad(params, X, T, stream=None):
    """(gradient, loss) of the mean squared error loss on (X, T)."""
    torch = _torch()
    _check_f32(params, X, T)
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    rc = lib().phipm_mlp_grad(_ptr(params), _ptr(X), _ptr(T), X.shape[0], _ptr(g), _ptr(loss),
                              _stream_ptr(stream))
    if rc != OK:
        raise PhipmError(rc, "phipm_mlp_grad")
    return g, loss


def mlp_train(params, adam_m, adam_v, X, T, epochs, lr=1e-3, batch=64, step0=0, stream=None):
    """Adam training in place; returns the per-epoch mean losses (device tensor)."""
    torch = _torch()
    _check_f32(params, adam_m, adam_v, X, T)
    loss = torch.empty(max(1, epochs), dtype=torch.float32, device=X.device)
    rc = lib().phipm_mlp_train(_ptr(params), _ptr(adam_m), _ptr(adam_v), _ptr(X), _ptr(T),
                               X.shape[0], int(batch), int(epochs), float(lr), int(step0),
                               _ptr(loss), _stream_ptr(stream))
    if rc != OK:
        raise PhipmError(rc, "phipm_mlp_train")
    return loss[:epochs]


def label_steps(trace, count, costs: LabelCosts | None = None, stream=None):
    """Hindsight labels of `count` recorded steps in the device buffer `trace`
    (cost per unit time from eq. 4, or from the time model `costs`).
    Returns (X, T) float32 device tensors."""
    torch = _torch()
    X = torch.empty((max(1, count), MLP_IN), dtype=torch.float32, device=trace.device)
    T = torch.empty((max(1, count), MLP_OUT), dtype=torch.float32, device=trace.device)
    nb = lib().phipm_label_workspace_bytes(int(count))
    ws = torch.empty(nb, dtype=torch.uint8, device=trace.device)
    rc = lib().phipm_label_steps(_ptr(trace), int(count), _ptr(X), _ptr(T), _ptr(ws), nb,
                                 C.byref(costs) if costs is not None else None,
                                 _stream_ptr(stream))
    if rc != OK:
        raise PhipmError(rc, "phipm_label_steps")
    return X[:count], T[:count]


def alloc_trace(cap, device="cuda"):
    """Device buffer for `cap` phipm_trace_step records."""
    torch = _torch()
    return torch.empty(cap * C.sizeof(TraceStep), dtype=torch.uint8, device=device)


def trace_records(trace, count):
    """Copy `count` records to the host as TraceStep structures."""
    raw = trace[: count * C.sizeof(TraceStep)].cpu().numpy().tobytes()
    return [TraceStep.from_buffer_copy(raw, i * C.sizeof(TraceStep)) for i in range(count)]
