// Many independent solves in one persistent launch.
//
// The grid (one 1024-thread workgroup per CU) is split into teams of
// power-of-two sizes.  Instances are grouped into size classes by predicted
// cost; each class has a queue in descending cost order (longest processing
// time first).  A team takes the next instance of its own class's queue and,
// when that is empty, the next one of the smaller classes' queues, solves it
// with the same routine as the single-solve kernel, and goes back for more.
// Queue heads are the only atomics; every team reuses one work buffer sized
// for the largest instance it may take.
//
// The team layout (team sizes, how many of each, the class thresholds) comes
// from an autotuner that times candidate layouts with the real kernel on the
// real instances, first with costs predicted from n, t and ||A||_inf, then
// with the per-instance times it measured.  The chosen launch (flag reset +
// persistent kernel) is captured in a hipGraph that execute() replays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/phipm.h"
#include "host_common.hpp"

using namespace pkr;

namespace {

// One instance (device array).
struct Inst {
  const int* rp;
  const int* ci;
  const void* val;  // of the plan's value type (every instance has the same)
  const double* b;
  double* u;
  double t;
  int n, nnz, p, val32;
};

// One team (device array).
struct TeamRec {
  int first, size, cls, pad;
  size_t ws;     // byte offset of the team's work buffer
  size_t flags;  // word offset of the team's barrier flags
  size_t part;   // double offset of the team's partials; its result follows them
};

struct BatchArgs {
  const Inst* inst;
  const int* order;   // queue entries (instance ids), class after class
  const int* qbeg;    // [ncls + 1] queue boundaries in order[]
  unsigned* qhead;    // [ncls] queue heads
  const TeamRec* teams;
  const int* team_of; // [grid] team of each workgroup
  char* ws;
  unsigned* flags;
  double* part;
  unsigned* abort;
  Stats* stats;       // [count]
  unsigned long long* clk;  // [2 count] start and end of each instance (wall clock)
  WorkLayout wl;      // layout of every team's work buffer
  double* hpool;      // [grid] copies of H, one per workgroup
  double tol, tau_fixed;
  long long max_attempts;
  int ncls, symm, m_init, m_max, adapt_m, corrector, validate, full_reorth;
  int fp32_flags, pad;
  unsigned long long spin;
  const float* proposer;
};

// Clears the barrier flags, the queue heads and the abort word (a kernel, so
// that the reset is an ordinary node of the captured graph).
__global__ void k_batch_reset(unsigned* flags, size_t nflags, unsigned* qhead, int ncls,
                              unsigned* abort) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nflags; i += stride)
    flags[i] = 0u;
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < ncls; i += blockDim.x) qhead[i] = 0u;
    if (threadIdx.x == 0) *abort = 0u;
  }
}

// ||A_i||_inf of every instance (one workgroup per instance).  Row bounds are
// clamped to [0, nnz] so that a malformed row pointer cannot send the loads
// out of range; the solver itself reports malformed input.
__global__ __launch_bounds__(256) void k_inst_norms(const Inst* inst, double* out) {
  __shared__ double s_w[256 / WAVE];
  const Inst in = inst[blockIdx.x];
  double mx = 0.0;
  for (int r = threadIdx.x; r < in.n; r += blockDim.x) {
    int k0 = in.rp[r], k1 = in.rp[r + 1];
    k0 = k0 < 0 ? 0 : (k0 > in.nnz ? in.nnz : k0);
    k1 = k1 < k0 ? k0 : (k1 > in.nnz ? in.nnz : k1);
    double s = 0.0;
    if (in.val32)
      for (int k = k0; k < k1; ++k) s += fabs((double)static_cast<const float*>(in.val)[k]);
    else
      for (int k = k0; k < k1; ++k) s += fabs(static_cast<const double*>(in.val)[k]);
    mx = nanmax(mx, s);
  }
  mx = wave_max(mx);
  if (threadIdx.x % WAVE == 0) s_w[threadIdx.x / WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = s_w[0];
    for (int w = 1; w < 256 / WAVE; ++w) a = nanmax(a, s_w[w]);
    out[blockIdx.x] = a;
  }
}

// T: basis type, VT: CSR value type.
template <typename T, typename VT>
__global__ __launch_bounds__(BLOCK) void k_batch(BatchArgs a) {
  __shared__ Shared sh;
  const int ti = a.team_of[blockIdx.x];
  const TeamRec tr = a.teams[ti];
  const int rank = (int)blockIdx.x - tr.first;
  double* part = a.part + tr.part;
  const Team tm = make_team(rank, tr.size, a.flags + tr.flags, a.abort, part,
                            part + team_partials(tr.size), a.spin);
  Work<T> w = {};
  {
    char* base = a.ws + tr.ws;
    w.W = reinterpret_cast<double*>(base + a.wl.W);
    w.ldw = a.wl.ld;
    w.V = reinterpret_cast<T*>(base + a.wl.V);
    w.ldv = a.wl.ld;
    w.y0 = reinterpret_cast<T*>(base + a.wl.y0);
    w.y1 = reinterpret_cast<T*>(base + a.wl.y1);
    w.H = a.hpool + (size_t)tr.first * H_WORDS;  // the team leader's copy
    w.Hm = a.hpool + (size_t)blockIdx.x * H_WORDS;
    w.ex = reinterpret_cast<double*>(base + a.wl.ex);
    w.st = reinterpret_cast<State*>(base + a.wl.st);
  }
  int qc = tr.cls;  // queue the team leader takes from next (used by rank 0 only)
  for (;;) {
    // the leader takes the next instance (-1: none left); the other members
    // contribute 0 to the team sum that hands the id to everyone
    if (threadIdx.x == 0) {
      int id = -1;
      if (rank == 0) {
        while (id < 0 && qc < a.ncls && ld_relaxed(a.abort) == 0u) {
          const unsigned k = atomicAdd(a.qhead + qc, 1u);
          if ((int)k < a.qbeg[qc + 1] - a.qbeg[qc]) id = a.order[a.qbeg[qc] + (int)k];
          else ++qc;
        }
      }
      sh.blk[0] = rank == 0 ? (double)id : 0.0;
    }
    if (!team_sync(tm, sh.blk, 1, RED_SUM, sh.red)) return;
    const int id = (int)sh.red[0];
    if (id < 0) return;
    const Inst in = a.inst[id];
    Problem P{};
    P.n = in.n;
    P.nnz = in.nnz;
    P.p = in.p;
    P.rp = in.rp;
    P.ci = in.ci;
    P.val = in.val;
    P.b = in.b;
    P.ldb = in.n;
    P.u = in.u;
    P.t = in.t;
    P.tol = a.tol;
    P.tau_fixed = a.tau_fixed;
    P.max_attempts = a.max_attempts;
    P.symm = a.symm;
    P.m_init = a.m_init;
    P.m_max = a.m_max;
    P.adapt_m = a.adapt_m;
    P.corrector = a.corrector;
    P.validate = a.validate;
    P.full_reorth = a.full_reorth;
    P.fp32_flags = a.fp32_flags;
    P.fp32mode = sizeof(T) == 4;
    P.segment = SEG_WHOLE;
    P.proposer = a.proposer;
    w.stats = a.stats + id;
    if (rank == 0 && threadIdx.x == 0) a.clk[2 * id] = wall_clock64();
    solve<T, VT, false>(tm, P, w, sh);
    if (rank == 0 && threadIdx.x == 0) a.clk[2 * id + 1] = wall_clock64();
  }
}

// ------------------------------------------------------------ host side

// The batched kernel of a (basis, values) type pair: index 2 * fp32 basis +
// float32 values.
const void* batch_kernel(int idx) {
  switch (idx) {
    case 0: return reinterpret_cast<const void*>(k_batch<double, double>);
    case 1: return reinterpret_cast<const void*>(k_batch<double, float>);
    case 2: return reinterpret_cast<const void*>(k_batch<float, double>);
    default: return reinterpret_cast<const void*>(k_batch<float, float>);
  }
}

struct BatchDevice {
  int cus = 0;
  int coresident[4] = {0, 0, 0, 0};  // per batch_kernel() index
  unsigned long long spin_ticks = 0;
  double clock_hz = 1e8;
  bool ok = false;
};

BatchDevice g_bdev[64];
std::mutex g_bmu;

const BatchDevice* batch_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_bmu);
  BatchDevice& d = g_bdev[dev];
  if (!d.ok) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return nullptr;
    d.cus = prop.multiProcessorCount;
    for (int k = 0; k < 4; ++k) {
      int b = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, batch_kernel(k), BLOCK, 0) !=
          hipSuccess)
        return nullptr;
      d.coresident[k] = std::min(TEAM_MAX, std::max(1, b) * d.cus);
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      khz = 100000;
    d.clock_hz = 1e3 * khz;
    d.spin_ticks = (unsigned long long)khz * 1000ull * 20ull;  // 20 s per wait
    d.ok = true;
  }
  return &d;
}

// A team layout: team sizes and classes, and the class queues.
struct TeamLayout {
  int smax = 1;
  double alpha = 1.0;
  std::vector<int> cls_size;   // team size of each class, largest first
  std::vector<int> cls_teams;  // teams per class
  std::vector<TeamRec> teams;
  std::vector<int> team_of;    // [grid]
  std::vector<int> order, qbeg;
};

// Layout for a grid of G workgroups from per-instance costs: an instance gets
// the smallest power-of-two team (at most smax) on which it costs no more
// than alpha times a workgroup's fair share; the workgroups are divided among
// the classes in proportion to the classes' total cost.
TeamLayout make_layout(const std::vector<double>& cost, int G, int smax, double alpha) {
  TeamLayout L;
  const int count = (int)cost.size();
  {
    // largest power of two not above min(smax, G)
    const int lim = std::max(1, std::min(smax, G));
    smax = 1;
    while (smax * 2 <= lim) smax *= 2;
  }
  L.smax = smax;
  L.alpha = alpha;
  double total = 0.0;
  for (double c : cost) total += c;
  if (!(total > 0.0)) total = 1.0;
  const double share = total / G;
  std::vector<int> s(count);
  for (int i = 0; i < count; ++i) {
    int si = 1;
    while (si < smax && cost[i] > alpha * share * si) si *= 2;
    s[i] = si;
  }
  std::vector<int> sizes(s);
  std::sort(sizes.begin(), sizes.end(), std::greater<int>());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  const int ncls = (int)sizes.size();
  std::vector<double> W(ncls, 0.0);
  std::vector<int> members(ncls, 0);
  auto cls_of = [&](int si) {
    return (int)(std::find(sizes.begin(), sizes.end(), si) - sizes.begin());
  };
  for (int i = 0; i < count; ++i) {
    W[cls_of(s[i])] += cost[i];
    members[cls_of(s[i])] += 1;
  }
  // instances a team of class c may take: its own class and the smaller ones
  std::vector<int> reach(ncls, 0);
  for (int c = ncls - 1, acc = 0; c >= 0; --c) reach[c] = (acc += members[c]);
  std::vector<int> nt(ncls);
  long long used = 0;
  for (int c = 0; c < ncls; ++c) {
    int k = (int)std::floor(G * W[c] / total / sizes[c]);
    k = std::max(1, std::min(k, reach[c]));
    nt[c] = k;
    used += (long long)k * sizes[c];
  }
  while (used > G) {
    int best = -1;
    for (int c = 0; c < ncls; ++c)
      if (nt[c] > 1 && (best < 0 || (long long)nt[c] * sizes[c] > (long long)nt[best] * sizes[best]))
        best = c;
    if (best < 0) break;
    nt[best] -= 1;
    used -= sizes[best];
  }
  if (used > G) {
    // too many classes for the grid: allow only smaller teams
    return make_layout(cost, G, smax / 2, alpha);
  }
  // leftover workgroups join the smallest class as teams of its size, then of 1
  int left = G - (int)used;
  const int last = ncls - 1;
  std::vector<int> extra1(ncls, 0);
  nt[last] += left / sizes[last];
  left -= (left / sizes[last]) * sizes[last];
  extra1[last] = left;
  int first = 0;
  for (int c = 0; c < ncls; ++c) {
    for (int k = 0; k < nt[c] + extra1[c]; ++k) {
      const int sz = k < nt[c] ? sizes[c] : 1;
      TeamRec tr{};
      tr.first = first;
      tr.size = sz;
      tr.cls = c;
      L.teams.push_back(tr);
      for (int r = 0; r < sz; ++r) L.team_of.push_back((int)L.teams.size() - 1);
      first += sz;
    }
  }
  L.cls_size = sizes;
  L.cls_teams.assign(ncls, 0);
  for (int c = 0; c < ncls; ++c) L.cls_teams[c] = nt[c] + extra1[c];
  // queues: class by class, descending cost (ties by index)
  L.qbeg.assign(ncls + 1, 0);
  for (int c = 0; c < ncls; ++c) {
    std::vector<int> q;
    for (int i = 0; i < count; ++i)
      if (s[i] == sizes[c]) q.push_back(i);
    std::stable_sort(q.begin(), q.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    L.order.insert(L.order.end(), q.begin(), q.end());
    L.qbeg[c + 1] = (int)L.order.size();
  }
  return L;
}

}  // namespace

struct phipm_plan {
  int device = 0;
  int count = 0;
  bool fp32 = false;
  int kidx = 0;  // batch_kernel() index
  int grid = 0;
  phipm_opts opts{};
  std::vector<Inst> inst;
  std::vector<double> anorm;
  // device memory (one allocation)
  void* mem = nullptr;
  size_t mem_bytes = 0;
  Inst* d_inst = nullptr;
  int* d_order = nullptr;
  int* d_qbeg = nullptr;
  unsigned* d_qhead = nullptr;
  TeamRec* d_teams = nullptr;
  int* d_team_of = nullptr;
  char* d_ws = nullptr;
  double* d_hpool = nullptr;
  unsigned* d_flags = nullptr;
  size_t nflags = 0;
  size_t npart = 0;
  double* d_part = nullptr;
  unsigned* d_abort = nullptr;
  Stats* d_stats = nullptr;
  unsigned long long* d_clk = nullptr;
  double* d_norms = nullptr;
  WorkLayout wl{};
  size_t team_ws = 0;
  TeamLayout layout;
  BatchArgs args{};
  unsigned long long spin = 0;
  double clock_hz = 1e8;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool graphed = false;
  bool coop_in_graph = false;
  hipStream_t last_stream = nullptr;
  bool executed = false;
  phipm_plan_info info{};
};

namespace {

// Upload a layout and fill the kernel arguments.
int set_layout(phipm_plan* pl, const TeamLayout& L, hipStream_t stream) {
  std::vector<TeamRec> teams = L.teams;
  size_t fw = 0, pw = 0;
  for (size_t t = 0; t < teams.size(); ++t) {
    teams[t].ws = pl->team_ws * t;
    teams[t].flags = fw;
    teams[t].part = pw;
    fw += team_flag_words(teams[t].size);
    pw += team_partials(teams[t].size) + KMAX;
  }
  const int ncls = (int)L.cls_size.size();
  if (fw > pl->nflags || pw > pl->npart || teams.size() > (size_t)pl->grid || ncls > pl->grid ||
      L.team_of.size() != (size_t)pl->grid || L.order.size() != (size_t)pl->count)
    return PHIPM_EINVAL;
  if (hipMemcpyAsync(pl->d_teams, teams.data(), sizeof(TeamRec) * teams.size(),
                     hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(pl->d_team_of, L.team_of.data(), sizeof(int) * L.team_of.size(),
                     hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(pl->d_order, L.order.data(), sizeof(int) * L.order.size(),
                     hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(pl->d_qbeg, L.qbeg.data(), sizeof(int) * L.qbeg.size(),
                     hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return PHIPM_EHIP;
  BatchArgs& a = pl->args;
  a = BatchArgs{};
  a.inst = pl->d_inst;
  a.order = pl->d_order;
  a.qbeg = pl->d_qbeg;
  a.qhead = pl->d_qhead;
  a.teams = pl->d_teams;
  a.team_of = pl->d_team_of;
  a.ws = pl->d_ws;
  a.flags = pl->d_flags;
  a.part = pl->d_part;
  a.abort = pl->d_abort;
  a.stats = pl->d_stats;
  a.clk = pl->d_clk;
  a.wl = pl->wl;
  a.hpool = pl->d_hpool;
  a.tol = pl->opts.tol;
  a.tau_fixed = pl->opts.tau_fixed;
  a.max_attempts = pl->opts.max_attempts;
  a.ncls = ncls;
  a.symm = pl->opts.symm;
  a.m_init = pl->opts.m_init;
  a.m_max = pl->opts.m_max;
  a.adapt_m = pl->opts.adapt_m;
  a.corrector = pl->opts.corrector;
  a.validate = pl->opts.validate;
  a.full_reorth = pl->opts.reorth == PHIPM_REORTH_FULL;
  a.fp32_flags = pl->fp32 ? pl->opts.fp32_flags : 0;
  a.spin = pl->spin;
  a.proposer = pl->opts.proposer;
  pl->layout = L;
  return PHIPM_OK;
}

hipError_t launch_reset(phipm_plan* pl, hipStream_t stream) {
  hipLaunchKernelGGL(k_batch_reset, dim3(64), dim3(256), 0, stream, pl->d_flags, pl->nflags,
                     pl->d_qhead, pl->args.ncls, pl->d_abort);
  return hipGetLastError();
}

hipError_t launch_batch(phipm_plan* pl, hipStream_t stream, bool cooperative) {
  void* args[] = {&pl->args};
  const void* fn = batch_kernel(pl->kidx);
  if (cooperative)
    return hipLaunchCooperativeKernel(fn, dim3(pl->grid), dim3(BLOCK), args, 0, stream);
  return hipLaunchKernel(fn, dim3(pl->grid), dim3(BLOCK), args, 0, stream);
}

// Run the current layout once (direct cooperative launch) and time it.
int timed_run(phipm_plan* pl, hipStream_t stream, double* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return PHIPM_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return PHIPM_EHIP;
  }
  int rc = PHIPM_OK;
  if (hipEventRecord(e0, stream) != hipSuccess || launch_reset(pl, stream) != hipSuccess ||
      launch_batch(pl, stream, true) != hipSuccess || hipEventRecord(e1, stream) != hipSuccess ||
      hipEventSynchronize(e1) != hipSuccess)
    rc = PHIPM_EHIP;
  float f = 0.f;
  if (rc == PHIPM_OK && hipEventElapsedTime(&f, e0, e1) != hipSuccess) rc = PHIPM_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != PHIPM_OK) return rc;
  unsigned ab = 0;
  if (hipMemcpy(&ab, pl->d_abort, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess)
    return PHIPM_EHIP;
  if (ab) return PHIPM_EABORT;
  *ms = f;
  return PHIPM_OK;
}

// Per-instance cost measured in the last run: workgroup-seconds.
int measured_costs(phipm_plan* pl, std::vector<double>& cost) {
  std::vector<unsigned long long> clk(2 * (size_t)pl->count);
  std::vector<Stats> st(pl->count);
  if (hipMemcpy(clk.data(), pl->d_clk, sizeof(unsigned long long) * clk.size(),
                hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(st.data(), pl->d_stats, sizeof(Stats) * st.size(), hipMemcpyDeviceToHost) !=
          hipSuccess)
    return PHIPM_EHIP;
  cost.resize(pl->count);
  for (int i = 0; i < pl->count; ++i) {
    const double sec = (double)(clk[2 * i + 1] - clk[2 * i]) / pl->clock_hz;
    cost[i] = std::max(1e-7, sec) * std::max(1, st[i].workgroups);
  }
  return PHIPM_OK;
}

// Predicted cost before anything was measured: rows times the number of
// products, which grows like the square root of t ||A||_inf for these
// stepping methods, plus a floor of ten products.
std::vector<double> predicted_costs(const phipm_plan* pl) {
  std::vector<double> c(pl->count);
  for (int i = 0; i < pl->count; ++i) {
    const double ta = std::fabs(pl->inst[i].t) * (std::isfinite(pl->anorm[i]) ? pl->anorm[i] : 0.0);
    c[i] = (double)pl->inst[i].n * (10.0 + 13.0 * std::sqrt(ta)) * (1.0 + 0.25 * pl->inst[i].p);
  }
  return c;
}

bool same_layout(const TeamLayout& a, const TeamLayout& b) {
  if (a.teams.size() != b.teams.size() || a.order != b.order || a.qbeg != b.qbeg) return false;
  for (size_t t = 0; t < a.teams.size(); ++t)
    if (a.teams[t].size != b.teams[t].size || a.teams[t].cls != b.teams[t].cls) return false;
  return true;
}

// Candidates: team-size caps 1..32 with the threshold factor 0.5 or 1 on the
// predicted costs; then the three fastest parameter pairs again on the costs
// measured in the fastest layout so far.
int autotune(phipm_plan* pl, hipStream_t stream, int default_smax) {
  const std::vector<double> pred = predicted_costs(pl);
  std::vector<int> smaxes;
  for (int s = 1; s <= std::min(pl->grid, 32); s *= 2) smaxes.push_back(s);
  const double alphas[] = {0.5, 1.0};
  struct Cand { TeamLayout L; double ms; };
  std::vector<Cand> tried;
  auto run = [&](const TeamLayout& L, double* ms) -> int {
    for (const Cand& c : tried)
      if (same_layout(c.L, L)) { *ms = c.ms; return PHIPM_OK; }
    int rc = set_layout(pl, L, stream);
    if (rc != PHIPM_OK) return rc;
    rc = timed_run(pl, stream, ms);
    if (rc != PHIPM_OK) return rc;
    tried.push_back(Cand{L, *ms});
    return PHIPM_OK;
  };
  // the untuned default first
  double ms = 0.0;
  int rc = run(make_layout(pred, pl->grid, default_smax, 1.0), &ms);
  if (rc != PHIPM_OK) return rc;
  pl->info.default_ms = ms;
  std::vector<double> meas;
  rc = measured_costs(pl, meas);
  if (rc != PHIPM_OK) return rc;
  // pass 1 with the predicted costs
  for (int s : smaxes)
    for (double al : alphas) {
      rc = run(make_layout(pred, pl->grid, s, al), &ms);
      if (rc != PHIPM_OK) return rc;
    }
  std::vector<size_t> rank(tried.size());
  std::iota(rank.begin(), rank.end(), 0);
  std::sort(rank.begin(), rank.end(), [&](size_t x, size_t y) { return tried[x].ms < tried[y].ms; });
  // measured costs from the fastest layout so far
  rc = set_layout(pl, tried[rank[0]].L, stream);
  if (rc == PHIPM_OK) rc = timed_run(pl, stream, &ms);
  if (rc == PHIPM_OK) rc = measured_costs(pl, meas);
  if (rc != PHIPM_OK) return rc;
  // pass 2: the best parameter pairs on the measured costs
  const size_t top = std::min<size_t>(3, rank.size());
  std::vector<std::pair<int, double>> params;
  for (size_t k = 0; k < top; ++k) params.push_back({tried[rank[k]].L.smax, tried[rank[k]].L.alpha});
  for (const auto& pa : params) {
    rc = run(make_layout(meas, pl->grid, pa.first, pa.second), &ms);
    if (rc != PHIPM_OK) return rc;
  }
  size_t b = 0;
  for (size_t i = 1; i < tried.size(); ++i)
    if (tried[i].ms < tried[b].ms) b = i;
  pl->info.candidates = (int)tried.size();
  pl->info.tuned_ms = tried[b].ms;
  return set_layout(pl, tried[b].L, stream);
}

// Capture reset + persistent kernel in a graph.  A cooperative launch is
// tried first; if the runtime does not accept one under capture, the kernel
// is captured as an ordinary launch of the same co-resident grid size (the
// team barriers then rely on the whole grid being resident, which holds on
// an otherwise idle device; a wait that times out aborts the run with
// PHIPM_EABORT instead of hanging).
int capture(phipm_plan* pl) {
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return PHIPM_EHIP;
  int rc = PHIPM_EHIP;
  for (int attempt = 0; attempt < 2 && rc != PHIPM_OK; ++attempt) {
    const bool coop = attempt == 0;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) break;
    const bool ok = launch_reset(pl, cs) == hipSuccess && launch_batch(pl, cs, coop) == hipSuccess;
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &g);
    (void)hipGetLastError();
    if (ok && ee == hipSuccess && g) {
      hipGraphExec_t ex = nullptr;
      if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
        pl->graph = g;
        pl->exec = ex;
        pl->graphed = true;
        pl->coop_in_graph = coop;
        rc = PHIPM_OK;
        continue;
      }
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
  }
  (void)hipStreamDestroy(cs);
  return rc;
}

void release(phipm_plan* pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->mem) (void)hipFree(pl->mem);
  delete pl;
}

}  // namespace

extern "C" {

void phipm_default_plan_opts(phipm_plan_opts* po) {
  if (!po) return;
  std::memset(po, 0, sizeof(*po));
  po->autotune = 1;
  po->graph = 1;
  po->max_team = 0;
}

int phipm_plan_create(int count, const phipm_csr* A, const int32_t* p, const double* t,
                      const double* const* b, double* const* u, const phipm_opts* o,
                      const phipm_plan_opts* po, phipm_stream_t stream_, phipm_plan** out) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (!out) return PHIPM_EINVAL;
  *out = nullptr;
  if (count < 1 || !A || !p || !t || !b || !u || !opts_ok(o) || !po) return PHIPM_EINVAL;
  if (po->max_team < 0 || (po->max_team & (po->max_team - 1)) != 0) return PHIPM_EINVAL;
  int nmax = 1, pmax = 0;
  for (int i = 0; i < count; ++i) {
    if (!csr_ok(&A[i]) || p[i] < 0 || p[i] > PHIPM_P_MAX || !b[i] || !u[i]) return PHIPM_EINVAL;
    if (A[i].val_dtype != A[0].val_dtype) return PHIPM_EINVAL;  // one value type per plan
    if (!std::isfinite(t[i])) return PHIPM_ENONFINITE;
    const size_t ub = sizeof(double) * (size_t)A[i].n;
    if (overlaps(u[i], ub, b[i], ub * (size_t)(p[i] + 1))) return PHIPM_EINVAL;
    nmax = std::max(nmax, A[i].n);
    pmax = std::max(pmax, (int)p[i]);
  }
  // outputs must not overlap each other
  {
    std::vector<std::pair<uintptr_t, uintptr_t>> r(count);
    for (int i = 0; i < count; ++i)
      r[i] = {reinterpret_cast<uintptr_t>(u[i]),
              reinterpret_cast<uintptr_t>(u[i]) + sizeof(double) * (size_t)A[i].n};
    std::sort(r.begin(), r.end());
    for (int i = 1; i < count; ++i)
      if (r[i].first < r[i - 1].second) return PHIPM_EINVAL;
  }
  const BatchDevice* d = batch_device();
  if (!d) return PHIPM_EHIP;
  phipm_plan* pl = new (std::nothrow) phipm_plan();
  if (!pl) return PHIPM_ENOMEM;
  (void)hipGetDevice(&pl->device);
  pl->count = count;
  pl->opts = *o;
  pl->fp32 = o->precision == PHIPM_FP32_BASIS;
  pl->kidx = 2 * pl->fp32 + (A[0].val_dtype == PHIPM_F32);
  const int gmax = d->coresident[pl->kidx];
  pl->grid = o->workgroups > 0 ? std::min(o->workgroups, gmax) : gmax;
  pl->spin = d->spin_ticks;
  pl->clock_hz = d->clock_hz;
  pl->inst.resize(count);
  for (int i = 0; i < count; ++i) {
    Inst& in = pl->inst[i];
    in.rp = A[i].row_ptr;
    in.ci = A[i].col_idx;
    in.val = A[i].val;
    in.b = b[i];
    in.u = u[i];
    in.t = t[i];
    in.n = A[i].n;
    in.nnz = A[i].nnz;
    in.p = p[i];
    in.val32 = A[i].val_dtype == PHIPM_F32;
  }
  // one allocation for everything the plan keeps on the device
  const int G = pl->grid;
  pl->wl = work_layout(nmax, pmax, std::min(o->m_max, nmax), 0);
  pl->team_ws = pl->wl.total;
  pl->nflags = (size_t)FLAG_STRIDE * 3 * (size_t)G;
  // >= sum over teams of team_partials(size) + KMAX (teams of one: 1 + TEAM_GBUF + 1 rows)
  pl->npart = (size_t)KMAX * (2 + TEAM_GBUF) * (size_t)G;
  const size_t npart = pl->npart;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o2 = off; off = align256(off + bytes); return o2; };
  const size_t o_inst = take(sizeof(Inst) * count);
  const size_t o_order = take(sizeof(int) * count);
  const size_t o_qbeg = take(sizeof(int) * (G + 1));
  const size_t o_qhead = take(sizeof(unsigned) * G);
  const size_t o_teams = take(sizeof(TeamRec) * G);
  const size_t o_team_of = take(sizeof(int) * G);
  const size_t o_flags = take(sizeof(unsigned) * pl->nflags);
  const size_t o_part = take(sizeof(double) * npart);
  const size_t o_abort = take(sizeof(unsigned) * FLAG_STRIDE);
  const size_t o_stats = take(sizeof(Stats) * count);
  const size_t o_clk = take(sizeof(unsigned long long) * 2 * count);
  const size_t o_norms = take(sizeof(double) * count);
  const size_t o_hpool = take(sizeof(double) * H_WORDS * (size_t)G);
  const size_t o_ws = take(pl->team_ws * (size_t)G);
  pl->mem_bytes = off;
  if (hipMalloc(&pl->mem, off) != hipSuccess) {
    (void)hipGetLastError();
    pl->mem = nullptr;
    release(pl);
    return PHIPM_ENOMEM;
  }
  char* base = static_cast<char*>(pl->mem);
  pl->d_inst = reinterpret_cast<Inst*>(base + o_inst);
  pl->d_order = reinterpret_cast<int*>(base + o_order);
  pl->d_qbeg = reinterpret_cast<int*>(base + o_qbeg);
  pl->d_qhead = reinterpret_cast<unsigned*>(base + o_qhead);
  pl->d_teams = reinterpret_cast<TeamRec*>(base + o_teams);
  pl->d_team_of = reinterpret_cast<int*>(base + o_team_of);
  pl->d_flags = reinterpret_cast<unsigned*>(base + o_flags);
  pl->d_part = reinterpret_cast<double*>(base + o_part);
  pl->d_abort = reinterpret_cast<unsigned*>(base + o_abort);
  pl->d_stats = reinterpret_cast<Stats*>(base + o_stats);
  pl->d_clk = reinterpret_cast<unsigned long long*>(base + o_clk);
  pl->d_norms = reinterpret_cast<double*>(base + o_norms);
  pl->d_ws = base + o_ws;
  pl->d_hpool = reinterpret_cast<double*>(base + o_hpool);
  int rc = PHIPM_OK;
  pl->anorm.assign(count, 0.0);
  if (hipMemcpyAsync(pl->d_inst, pl->inst.data(), sizeof(Inst) * count, hipMemcpyHostToDevice,
                     stream) != hipSuccess)
    rc = PHIPM_EHIP;
  if (rc == PHIPM_OK) {
    hipLaunchKernelGGL(k_inst_norms, dim3(count), dim3(256), 0, stream, pl->d_inst, pl->d_norms);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(pl->anorm.data(), pl->d_norms, sizeof(double) * count,
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      rc = PHIPM_EHIP;
  }
  const int default_smax = po->max_team > 0 ? po->max_team : 16;
  if (rc == PHIPM_OK) {
    if (po->autotune) {
      rc = autotune(pl, stream, default_smax);
    } else {
      rc = set_layout(pl, make_layout(predicted_costs(pl), G, default_smax, 1.0), stream);
    }
  }
  if (rc == PHIPM_OK && po->graph) rc = capture(pl);
  if (rc != PHIPM_OK) {
    (void)hipStreamSynchronize(stream);
    release(pl);
    return rc;
  }
  phipm_plan_info& inf = pl->info;
  inf.count = count;
  inf.workgroups = G;
  inf.teams = (int)pl->layout.teams.size();
  inf.classes = std::min<int>(8, (int)pl->layout.cls_size.size());
  for (int c = 0; c < inf.classes; ++c) {
    inf.class_size[c] = pl->layout.cls_size[c];
    inf.class_teams[c] = pl->layout.cls_teams[c];
  }
  inf.graph = pl->graphed ? 1 : 0;
  inf.cooperative = pl->graphed ? (pl->coop_in_graph ? 1 : 0) : 1;
  inf.max_team = pl->layout.smax;
  inf.alpha = pl->layout.alpha;
  inf.device_bytes = pl->mem_bytes;
  *out = pl;
  return PHIPM_OK;
}

int phipm_plan_execute(phipm_plan* pl, phipm_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (!pl) return PHIPM_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl->device) return PHIPM_EINVAL;
  if (pl->graphed) {
    if (hipGraphLaunch(pl->exec, stream) != hipSuccess) return PHIPM_EHIP;
  } else {
    if (launch_reset(pl, stream) != hipSuccess || launch_batch(pl, stream, true) != hipSuccess)
      return PHIPM_EHIP;
  }
  pl->last_stream = stream;
  pl->executed = true;
  return PHIPM_OK;
}

int phipm_plan_stats(phipm_plan* pl, phipm_stats* stats) {
  if (!pl || !stats) return PHIPM_EINVAL;
  std::vector<Stats> hs(pl->count);
  unsigned ab = 0;
  hipStream_t s = pl->last_stream;
  if (hipMemcpyAsync(hs.data(), pl->d_stats, sizeof(Stats) * hs.size(), hipMemcpyDeviceToHost,
                     s) != hipSuccess ||
      hipMemcpyAsync(&ab, pl->d_abort, sizeof(unsigned), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return PHIPM_EHIP;
  int first = PHIPM_OK;
  const double tick_s = wall_tick_seconds(pl->device);
  for (int i = 0; i < pl->count; ++i) {
    const int st = ab ? PHIPM_EABORT : hs[i].status;
    copy_stats(hs[i], st, tick_s, &stats[i]);
    if (first == PHIPM_OK && st != PHIPM_OK) first = st;
  }
  return first;
}

int phipm_plan_get_info(const phipm_plan* pl, phipm_plan_info* info) {
  if (!pl || !info) return PHIPM_EINVAL;
  *info = pl->info;
  return PHIPM_OK;
}

int phipm_plan_destroy(phipm_plan* pl) {
  if (!pl) return PHIPM_EINVAL;
  if (pl->executed) (void)hipStreamSynchronize(pl->last_stream);
  release(pl);
  return PHIPM_OK;
}

int phipm_batch_layout(int count, const double* cost, int workgroups, int max_team,
                       double alpha, int32_t* team_size, int32_t* team_class, int32_t* nteams,
                       int32_t* order, int32_t* qbeg, int32_t* nclasses) {
  if (count < 1 || !cost || workgroups < 1 || workgroups > TEAM_MAX || max_team < 1 ||
      (max_team & (max_team - 1)) != 0 || !(alpha > 0.0) || !std::isfinite(alpha) ||
      !team_size || !team_class || !nteams || !order || !qbeg || !nclasses)
    return PHIPM_EINVAL;
  std::vector<double> c(cost, cost + count);
  for (double x : c)
    if (!(x >= 0.0) || !std::isfinite(x)) return PHIPM_EINVAL;
  const TeamLayout L = make_layout(c, workgroups, max_team, alpha);
  *nteams = (int32_t)L.teams.size();
  for (size_t t = 0; t < L.teams.size(); ++t) {
    team_size[t] = L.teams[t].size;
    team_class[t] = L.teams[t].cls;
  }
  for (int i = 0; i < count; ++i) order[i] = L.order[i];
  *nclasses = (int32_t)L.cls_size.size();
  for (size_t c2 = 0; c2 < L.qbeg.size(); ++c2) qbeg[c2] = L.qbeg[c2];
  return PHIPM_OK;
}

int phipm_batched(int count, const phipm_csr* A, const int32_t* p, const double* t,
                  const double* const* b, double* const* u, const phipm_opts* o,
                  phipm_stats* stats, phipm_stream_t stream) {
  phipm_plan_opts po;
  phipm_default_plan_opts(&po);
  po.autotune = 0;
  po.graph = 0;
  phipm_plan* pl = nullptr;
  int rc = phipm_plan_create(count, A, p, t, b, u, o, &po, stream, &pl);
  if (rc != PHIPM_OK) return rc;
  rc = phipm_plan_execute(pl, stream);
  if (rc == PHIPM_OK) {
    if (stats) {
      rc = phipm_plan_stats(pl, stats);
    } else {
      std::vector<phipm_stats> tmp(count);
      rc = phipm_plan_stats(pl, tmp.data());
    }
  }
  phipm_plan_destroy(pl);
  return rc;
}

}  // extern "C"
