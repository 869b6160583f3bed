// C ABI of the phipm library: argument checks, workspace layout, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/phipm.h"
#include "host_common.hpp"

using namespace pkr;

namespace {

// ------------------------------------------------------------ kernels

// Clears the team control block; keep_abort leaves the abort word as it is
// (between the chained launches of one solve, so that a launch that timed out
// stops the ones after it).
__global__ void k_zero_ctl(TeamCtl* ctl, int count, int keep_abort) {
  unsigned* w = reinterpret_cast<unsigned*>(ctl);
  const size_t words = (size_t)count * sizeof(TeamCtl) / sizeof(unsigned);
  const size_t abort_word = offsetof(TeamCtl, abort) / sizeof(unsigned);
  for (size_t i = threadIdx.x; i < words; i += blockDim.x)
    if (!(keep_abort && i == abort_word)) w[i] = 0u;
}

// One 1024-thread workgroup per CU (16 waves, at most 128 VGPRs each).
// T: basis type, VT: CSR value type.
template <typename T, typename VT>
__global__ __launch_bounds__(BLOCK) void k_solve(Problem P, Work<T> w, TeamCtl* ctl,
                                                 double* partials, double* result,
                                                 unsigned long long spin) {
  __shared__ Shared sh;
  const Team tm = make_team((int)blockIdx.x, (int)gridDim.x, &ctl->gen, &ctl->abort, partials,
                            result, spin);
  Work<T> wk = w;
  wk.Hm = w.H + (size_t)blockIdx.x * H_WORDS;
  solve<T, VT, true>(tm, P, wk, sh);
}

// The solver kernel of a (basis, values) type pair: index 2 * fp32 basis +
// float32 values.
const void* solve_kernel(int idx) {
  switch (idx) {
    case 0: return reinterpret_cast<const void*>(k_solve<double, double>);
    case 1: return reinterpret_cast<const void*>(k_solve<double, float>);
    case 2: return reinterpret_cast<const void*>(k_solve<float, double>);
    default: return reinterpret_cast<const void*>(k_solve<float, float>);
  }
}

template <typename VT>
__global__ __launch_bounds__(BLOCK) void k_spmv(int n, const int* rp, const int* ci,
                                                const VT* val, const double* x, double* y) {
  __shared__ SpmvSmem<VT> sm;
  auto ld = [&](int c) -> double { return x[c]; };
  for (long long r0 = (long long)blockIdx.x * BLOCK; r0 < n; r0 += (long long)gridDim.x * BLOCK) {
    const int r1 = (int)std::min<long long>(r0 + BLOCK, n);
    double acc = spmv_tile<VT, double>(rp, ci, val, (int)r0, r1, sm, ld);
    const int r = (int)r0 + threadIdx.x;
    if (r < r1) y[r] = acc;
  }
}

// u += du, elementwise.
__global__ __launch_bounds__(256) void k_add_to(int n, double* u, const double* du) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256)
    u[i] += du[i];
}

// Allen-Cahn step data, one row per thread: F = L u + (u - u^3) (the CSR
// product as in k_spmv) and the Jacobian's diagonal lap_diag + (1 - 3 u^2)
// at its positions in J's value array.  F or Jval may be null (skipped);
// both nulls are excluded by the caller.
__global__ __launch_bounds__(BLOCK) void k_allen_cahn(int n, const int* rp, const int* ci,
                                                      const double* val, const double* u,
                                                      const int* diag_pos,
                                                      const double* lap_diag, double* Jval,
                                                      double* F) {
  __shared__ SpmvSmem<double> sm;
  auto ld = [&](int c) -> double { return u[c]; };
  for (long long r0 = (long long)blockIdx.x * BLOCK; r0 < n; r0 += (long long)gridDim.x * BLOCK) {
    const int r1 = (int)std::min<long long>(r0 + BLOCK, n);
    // F is the same for every thread of the launch, so the product's
    // barriers are reached by all of them or by none
    const double acc = F ? spmv_tile<double, double>(rp, ci, val, (int)r0, r1, sm, ld) : 0.0;
    const int r = (int)r0 + threadIdx.x;
    if (r < r1) {
      const double ur = u[r];
      if (F) F[r] = acc + (ur - ur * ur * ur);
      if (Jval) Jval[diag_pos[r]] = lap_diag[r] + (1.0 - 3.0 * ur * ur);
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_expm(int N, const double* H, double* E, double* S) {
  __shared__ double s_norm;
  __shared__ int s_sq;
  __shared__ double L[DENSE_LDS];
  for (int e = threadIdx.x; e < N * N; e += BLOCK) S[e] = H[e];
  __syncthreads();
  const double* R = wg_expm(N, S, L, &s_norm, &s_sq);
  for (int e = threadIdx.x; e < N * N; e += BLOCK) E[e] = R[e];
}

// m Krylov steps from v with the solver's step routine (float64).
__global__ __launch_bounds__(BLOCK) void k_krylov(Problem P, Work<double> w0, const double* v,
                                                  int m, int lanczos, double* Hout,
                                                  int* m_done, TeamCtl* ctl, double* partials,
                                                  double* result, unsigned long long spin) {
  __shared__ Shared sh;
  const Team tm = make_team((int)blockIdx.x, (int)gridDim.x, &ctl->gen, &ctl->abort, partials,
                            result, spin);
  Work<double> w = w0;
  w.Hm = w0.H + (size_t)blockIdx.x * H_WORDS;
  const double* val = static_cast<const double*>(P.val);
  int rb, re;
  own_rows(tm, P.n, rb, re);
  // the column range of the own rows: every slot (this entry point skips
  // the solver's setup scan)
  if (threadIdx.x == 0) {
    sh.dep_lo = 0;
    sh.dep_hi = tm.size - 1;
  }
  for (size_t e = threadIdx.x; e < H_WORDS; e += BLOCK) w.Hm[e] = 0.0;
  __syncthreads();
  double a = 0.0;
  for (int r = rb + threadIdx.x; r < re; r += BLOCK) a += v[r] * v[r];
  double a1[1] = {a};
  block_reduce<1>(a1, RED_SUM, sh.blk);
  if (!team_sync(tm, sh.blk, 1, RED_SUM, sh.red)) return;
  const double beta = sqrt(sh.red[0]);
  KrylovCtl kc{0, 1, 0, 1};
  while (!kc.broke && kc.have < m && kc.have < P.n) {
    const bool ok = kc.have == 0
                        ? krylov_iter<double, double, double>(tm, P, w, val, 1.0, lanczos != 0,
                                                              0.0, kc, v, 1.0 / beta, rb, re, sh)
                        : krylov_iter<double, double, double>(tm, P, w, val, 1.0, lanczos != 0,
                                                              0.0, kc, nullptr, 0.0, rb, re, sh);
    if (!ok) return;
  }
  if (!krylov_finalize<double>(tm, P, w, lanczos != 0, 0.0, kc, rb, re, sh)) return;
  const int have = kc.have;
  if (tm.rank == 0) {
    for (int e = threadIdx.x; e < (m + 1) * m; e += BLOCK) {
      const int i = e / m, j = e - i * m;
      Hout[e] = j < have ? w.H[(long long)i * M_CAP + j] : 0.0;
    }
    if (threadIdx.x == 0) *m_done = have;
  }
}

// ----------------------------------------------------------- host side

struct DeviceInfo {
  int cus = 0;
  int coresident[4] = {0, 0, 0, 0};  // cooperative grid limit per solve_kernel() index
  unsigned long long spin_ticks = 0;
  double tick_s = 0.0;  // seconds per wall-clock tick
  bool ok = false;
};

DeviceInfo g_dev[64];
std::mutex g_mu;

const DeviceInfo* device_info() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceInfo& d = g_dev[dev];
  if (!d.ok) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return nullptr;
    d.cus = prop.multiProcessorCount;
    for (int k = 0; k < 4; ++k) {
      int b = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, solve_kernel(k), BLOCK, 0) !=
          hipSuccess)
        return nullptr;
      d.coresident[k] = std::min(TEAM_MAX, std::max(1, b) * d.cus);
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      khz = 100000;
    d.spin_ticks = (unsigned long long)khz * 1000ull * 20ull;  // 20 s per wait
    d.tick_s = wall_tick_seconds(dev);
    d.ok = true;
  }
  return &d;
}

// Work buffer of one solve followed by the team's control block, reduction
// partials and result.
struct Layout {
  WorkLayout w;
  size_t ctl, part, res, total;
};

Layout layout(int n, int p, int m_cap, int gmax, int groups) {
  Layout L{};
  L.w = work_layout(n, p, m_cap, groups);
  size_t off = L.w.total;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  L.ctl = take(sizeof(TeamCtl));
  L.part = take(sizeof(double) * team_partials(gmax));
  L.res = take(sizeof(double) * KMAX);
  L.total = off;
  return L;
}

// Device scratch of the allocation-free entry point phipm_noalloc(): a
// file-scope array that every GPU the library runs on holds until the
// process ends.  In host code its name is only a stand-in; the device
// address of each GPU's copy comes from hipGetSymbolAddress (once per device,
// kept in g_scratch) and only that address is passed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

struct DeviceScratch {
  void* ptr = nullptr;
  bool ok = false;
};
DeviceScratch g_scratch[64];

// This device's scratch address (null if it could not be obtained).
void* device_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceScratch& s = g_scratch[dev];
  if (!s.ok) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    s.ptr = ptr;
    s.ok = true;
  }
  return s.ptr;
}

thread_local hipStream_t t_last_stream = nullptr;
thread_local const Stats* t_last_stats = nullptr;
thread_local const TeamCtl* t_last_ctl = nullptr;
thread_local int t_last_host_status = 0;

int fail(int code) {
  t_last_host_status = code;
  t_last_stats = nullptr;
  return code;
}

// Library choice: one workgroup up to 2048 rows (a team's synchronisations
// would cost more than its streaming saves), else one per 320 rows up to the
// co-resident limit (measured on MI355X: the 100 x 51 Heston operator runs
// 15% faster on 16 workgroups than on 5, the 30 x 30 Laplacian fastest on 1).
int choose_workgroups(const phipm_opts* o, int n, int gmax) {
  int g = o->workgroups;
  if (g <= 0) {
    const long long want = n <= 2048 ? 1 : ((long long)n + 319) / 320;
    g = (int)std::min<long long>(want, gmax);
  }
  if (g > gmax) g = gmax;
  if (g < 1) g = 1;
  return g;
}

}  // namespace

extern "C" {

void phipm_default_opts(phipm_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-7;
  o->symm = -1;
  o->m_init = 10;
  o->m_max = 100;
  o->precision = PHIPM_FP64;
  o->adapt_m = 1;
  o->corrector = 1;
  o->tau_fixed = 0.0;
  o->max_attempts = 1000000;
  o->workgroups = 0;
  o->validate = 1;
}

int phipm_workspace_bytes(const phipm_csr* A, int p, const phipm_opts* o, size_t* bytes) {
  if (!csr_ok(A) || p < 0 || p > PHIPM_P_MAX || !opts_ok(o) || !bytes) return PHIPM_EINVAL;
  const DeviceInfo* d = device_info();
  if (!d) return PHIPM_EHIP;
  const bool fp32 = o->precision == PHIPM_FP32_BASIS;
  const int vf = A->val_dtype == PHIPM_F32;
  const int kidx = 2 * fp32 + vf;
  const int gmax = fp32 ? std::min(d->coresident[vf], d->coresident[kidx]) : d->coresident[kidx];
  const int m_cap = std::min(o->m_max, A->n);
  *bytes = layout(A->n, p, m_cap, gmax, choose_workgroups(o, A->n, gmax)).total;
  return PHIPM_OK;
}

int phipm(double t, const phipm_csr* A, int p, const double* b, const phipm_opts* o, double* u,
          void* workspace, size_t ws_bytes, phipm_stats* stats, phipm_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (!csr_ok(A) || p < 0 || p > PHIPM_P_MAX || !opts_ok(o) || !b || !u || !workspace)
    return fail(PHIPM_EINVAL);
  if (!std::isfinite(t)) return fail(PHIPM_ENONFINITE);
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(PHIPM_EINVAL);
  const DeviceInfo* d = device_info();
  if (!d) return fail(PHIPM_EHIP);
  const bool fp32 = o->precision == PHIPM_FP32_BASIS;
  const int vf = A->val_dtype == PHIPM_F32;
  const int kidx = 2 * fp32 + vf;
  // FP32 mode chains the FP64 and FP32 solvers: both must fit the grid
  const int gmax = fp32 ? std::min(d->coresident[vf], d->coresident[kidx]) : d->coresident[kidx];
  const int m_cap = std::min(o->m_max, A->n);
  const int G = choose_workgroups(o, A->n, gmax);
  const Layout L = layout(A->n, p, m_cap, gmax, G);
  if (ws_bytes < L.total) return fail(PHIPM_ENOMEM);
  // u must not overlap b or the workspace
  const size_t ub = sizeof(double) * (size_t)A->n;
  if (overlaps(u, ub, b, ub * (size_t)(p + 1)) || overlaps(u, ub, workspace, ws_bytes))
    return fail(PHIPM_EINVAL);

  char* ws = static_cast<char*>(workspace);
  Problem P{};
  P.n = A->n;
  P.nnz = A->nnz;
  P.p = p;
  P.rp = A->row_ptr;
  P.ci = A->col_idx;
  P.val = A->val;
  P.b = b;
  P.ldb = A->n;
  P.u = u;
  P.t = t;
  P.tol = o->tol;
  P.tau_fixed = o->tau_fixed;
  P.max_attempts = o->max_attempts;
  P.symm = o->symm;
  P.m_init = o->m_init;
  P.m_max = o->m_max;
  P.adapt_m = o->adapt_m;
  P.corrector = o->corrector;
  P.validate = o->validate;
  P.full_reorth = o->reorth == PHIPM_REORTH_FULL;
  P.fp32_flags = fp32 ? o->fp32_flags : 0;
  P.fp32mode = fp32;
  P.segment = SEG_WHOLE;
  P.proposer = o->proposer;
  P.history = o->history;
  P.trace = static_cast<TraceStep*>(o->trace);
  P.trace_cap = o->trace ? o->trace_cap : 0;

  TeamCtl* ctl = reinterpret_cast<TeamCtl*>(ws + L.ctl);
  double* part = reinterpret_cast<double*>(ws + L.part);
  double* res = reinterpret_cast<double*>(ws + L.res);
  Stats* dstats = reinterpret_cast<Stats*>(ws + L.w.stats);
  unsigned long long spin = d->spin_ticks;

  hipLaunchKernelGGL(k_zero_ctl, dim3(1), dim3(1024), 0, stream, ctl, 1, 0);
  if (hipGetLastError() != hipSuccess) return fail(PHIPM_EHIP);
  hipError_t e;
  if (fp32) {
    // FP64 steps from the start, FP32 steps, FP64 steps to the end
    Work<double> w64 = work_at<double>(ws, L.w);
    Work<float> w32 = work_at<float>(ws, L.w);
    const int seg[3] = {SEG_LEAD, SEG_FP32, SEG_TAIL};
    e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
      P.segment = seg[k];
      if (k > 0) {
        hipLaunchKernelGGL(k_zero_ctl, dim3(1), dim3(1024), 0, stream, ctl, 1, 1);
        if (hipGetLastError() != hipSuccess) return fail(PHIPM_EHIP);
      }
      void* args64[] = {&P, &w64, &ctl, &part, &res, &spin};
      void* args32[] = {&P, &w32, &ctl, &part, &res, &spin};
      e = hipLaunchCooperativeKernel(solve_kernel(seg[k] == SEG_FP32 ? kidx : vf), dim3(G),
                                     dim3(BLOCK), seg[k] == SEG_FP32 ? args32 : args64, 0,
                                     stream);
    }
  } else {
    Work<double> w = work_at<double>(ws, L.w);
    void* args[] = {&P, &w, &ctl, &part, &res, &spin};
    e = hipLaunchCooperativeKernel(solve_kernel(kidx), dim3(G), dim3(BLOCK), args, 0, stream);
  }
  if (e != hipSuccess) return fail(PHIPM_EHIP);
  t_last_stream = stream;
  t_last_stats = dstats;
  t_last_ctl = ctl;
  t_last_host_status = PHIPM_OK;
  if (stats) {
    Stats hs;
    TeamCtl hc;
    if (hipMemcpyAsync(&hs, dstats, sizeof(Stats), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(&hc, ctl, sizeof(TeamCtl), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return fail(PHIPM_EHIP);
    copy_stats(hs, hc.abort ? PHIPM_EABORT : hs.status, d->tick_s, stats);
    stats->workgroups = G;
    return stats->status;
  }
  return PHIPM_OK;
}

int phipm_noalloc(double t, const phipm_csr* A, int p, const double* b, const phipm_opts* o,
                  double* u, phipm_stats* stats, phipm_stream_t stream) {
  size_t need = 0;
  const int rc = phipm_workspace_bytes(A, p, o, &need);
  if (rc != PHIPM_OK) return fail(rc);
  if (need > NOALLOC_SCRATCH_BYTES) return fail(PHIPM_ESCRATCH);
  void* ws = device_scratch();
  if (!ws) return fail(PHIPM_EHIP);
  return phipm(t, A, p, b, o, u, ws, NOALLOC_SCRATCH_BYTES, stats, stream);
}

size_t phipm_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

int phipm_last_status(void) {
  if (t_last_host_status != PHIPM_OK || !t_last_stats) return t_last_host_status;
  Stats hs;
  TeamCtl hc;
  if (hipMemcpyAsync(&hs, t_last_stats, sizeof(Stats), hipMemcpyDeviceToHost, t_last_stream) !=
          hipSuccess ||
      hipMemcpyAsync(&hc, t_last_ctl, sizeof(TeamCtl), hipMemcpyDeviceToHost, t_last_stream) !=
          hipSuccess ||
      hipStreamSynchronize(t_last_stream) != hipSuccess)
    return PHIPM_EHIP;
  return hc.abort ? PHIPM_EABORT : hs.status;
}

int phipm_spmv(const phipm_csr* A, const double* x, double* y, phipm_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (!csr_ok(A) || !x || !y) return PHIPM_EINVAL;
  const DeviceInfo* d = device_info();
  if (!d) return PHIPM_EHIP;
  const long long tiles = ((long long)A->n + BLOCK - 1) / BLOCK;
  const int grid = (int)std::min<long long>(tiles, (long long)d->cus * 8);
  if (A->val_dtype == PHIPM_F32)
    hipLaunchKernelGGL(k_spmv<float>, dim3(grid), dim3(BLOCK), 0, stream, A->n, A->row_ptr,
                       A->col_idx, static_cast<const float*>(A->val), x, y);
  else
    hipLaunchKernelGGL(k_spmv<double>, dim3(grid), dim3(BLOCK), 0, stream, A->n, A->row_ptr,
                       A->col_idx, static_cast<const double*>(A->val), x, y);
  return hipGetLastError() == hipSuccess ? PHIPM_OK : PHIPM_EHIP;
}

int phipm_allen_cahn_update(const phipm_csr* L, double* u, const double* du,
                            const int32_t* diag_pos, const double* lap_diag, double* J_val,
                            double* F, phipm_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (!csr_ok(L) || L->val_dtype != PHIPM_F64 || !u || (J_val && (!diag_pos || !lap_diag)))
    return PHIPM_EINVAL;
  const DeviceInfo* d = device_info();
  if (!d) return PHIPM_EHIP;
  const long long tiles = ((long long)L->n + BLOCK - 1) / BLOCK;
  if (du) {
    const long long blocks = ((long long)L->n + 255) / 256;
    const int grid = (int)std::min<long long>(std::max<long long>(blocks, 1), (long long)d->cus * 16);
    hipLaunchKernelGGL(k_add_to, dim3(grid), dim3(256), 0, stream, L->n, u, du);
    if (hipGetLastError() != hipSuccess) return PHIPM_EHIP;
  }
  if (F || J_val) {
    const int grid = (int)std::min<long long>(std::max<long long>(tiles, 1), (long long)d->cus * 8);
    hipLaunchKernelGGL(k_allen_cahn, dim3(grid), dim3(BLOCK), 0, stream, L->n, L->row_ptr,
                       L->col_idx, static_cast<const double*>(L->val), u, diag_pos, lap_diag,
                       J_val, F);
    if (hipGetLastError() != hipSuccess) return PHIPM_EHIP;
  }
  return PHIPM_OK;
}

int phipm_expm(int N, const double* H, double* E, double* scratch, phipm_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (N < 1 || N > NMAX_EXPM || !H || !E || !scratch) return PHIPM_EINVAL;
  hipLaunchKernelGGL(k_expm, dim3(1), dim3(BLOCK), 0, stream, N, H, E, scratch);
  return hipGetLastError() == hipSuccess ? PHIPM_OK : PHIPM_EHIP;
}

int phipm_krylov(const phipm_csr* A, const double* v, int m, int lanczos, double* V, double* H,
                 void* workspace, size_t ws_bytes, int* m_done, phipm_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (!csr_ok(A) || A->val_dtype != PHIPM_F64 || !v || !V || !H || !workspace || !m_done ||
      m < 1 || m > PHIPM_M_CAP)
    return PHIPM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return PHIPM_EINVAL;
  const DeviceInfo* d = device_info();
  if (!d) return PHIPM_EHIP;
  phipm_opts o;
  phipm_default_opts(&o);
  const int G = choose_workgroups(&o, A->n, d->coresident[0]);
  const Layout L = layout(A->n, 0, m, d->coresident[0], G);
  if (ws_bytes < L.total) return PHIPM_ENOMEM;
  char* ws = static_cast<char*>(workspace);
  Problem P{};
  P.n = A->n;
  P.nnz = A->nnz;
  P.rp = A->row_ptr;
  P.ci = A->col_idx;
  P.val = A->val;
  Work<double> w{nullptr, 0, V, A->n, reinterpret_cast<double*>(ws + L.w.y0),
                 reinterpret_cast<double*>(ws + L.w.y1), reinterpret_cast<double*>(ws + L.w.H),
                 nullptr, reinterpret_cast<State*>(ws + L.w.st), nullptr,
                 reinterpret_cast<double*>(ws + L.w.H)};
  TeamCtl* ctl = reinterpret_cast<TeamCtl*>(ws + L.ctl);
  double* part = reinterpret_cast<double*>(ws + L.part);
  double* res = reinterpret_cast<double*>(ws + L.res);
  int* dm = reinterpret_cast<int*>(ws + L.w.stats);
  unsigned long long spin = d->spin_ticks;
  hipLaunchKernelGGL(k_zero_ctl, dim3(1), dim3(1024), 0, stream, ctl, 1, 0);
  void* args[] = {&P, &w, &v, &m, &lanczos, &H, &dm, &ctl, &part, &res, &spin};
  if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_krylov), dim3(G), dim3(BLOCK),
                                 args, 0, stream) != hipSuccess)
    return PHIPM_EHIP;
  if (hipMemcpyAsync(m_done, dm, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return PHIPM_EHIP;
  return PHIPM_OK;
}

const char* phipm_status_string(int s) {
  switch (s) {
    case PHIPM_OK: return "ok";
    case PHIPM_EINVAL: return "invalid argument or malformed CSR matrix";
    case PHIPM_ENOMEM: return "workspace too small";
    case PHIPM_EHIP: return "HIP runtime error";
    case PHIPM_ENONFINITE: return "non-finite value in A, b or t";
    case PHIPM_EMAXSTEPS: return "attempt limit reached";
    case PHIPM_EUNSUPPORTED: return "unsupported";
    case PHIPM_EABORT: return "device wait exceeded its time budget";
    case PHIPM_ESCRATCH:
      return "problem needs more device scratch than phipm_noalloc holds "
             "(phipm_noalloc_scratch_bytes()); use phipm() with a workspace";
    default: return "unknown status";
  }
}

}  // extern "C"
