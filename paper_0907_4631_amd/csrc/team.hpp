// Workgroup teams: the workgroups of one persistent (cooperatively launched)
// grid that solve one problem together.  A team owns a control block in
// device memory (arrival counter, generation, abort flag) and a partials
// buffer used by the fused "reduce and synchronise" primitive below.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pkr {

constexpr int BLOCK = 512;               // threads per workgroup
constexpr int WAVE = 64;                 // CDNA wavefront
constexpr int NWAVES = BLOCK / WAVE;
constexpr int M_CAP = 128;               // largest Krylov dimension
constexpr int P_MAX = 8;                 // largest p
constexpr int KMAX = M_CAP + 8;          // widest team reduction
constexpr int NMAX_EXPM = M_CAP + P_MAX + 1;

constexpr int TEAM_GROUP = 16;            // workgroups per arrival group
constexpr int TEAM_MAX = 1024;            // largest team
constexpr int TEAM_NGROUPS = TEAM_MAX / TEAM_GROUP;

// Team control block in device memory.  Arrivals are counted per group of
// TEAM_GROUP workgroups (each counter on its own 128-byte line); the last
// arrival of a group then arrives at the top counter.  This keeps the number
// of serialized atomics on any one address at TEAM_GROUP or the group count.
struct TeamCtl {
  unsigned count;    // group arrivals at the top in the current generation
  unsigned gen;      // generation number
  unsigned abort;    // set when a wait exceeded its time budget
  unsigned pad[29];
  unsigned grp[TEAM_NGROUPS][32];  // per-group arrival counters
};

struct Team {
  int rank;            // this workgroup's index in the team
  int size;            // workgroups in the team
  TeamCtl* ctl;
  double* partials;    // [KMAX][size] per-workgroup values, then [KMAX][groups] group sums
  double* result;      // [KMAX]
  uint64_t spin_ticks; // wall-clock budget of one wait
};

enum RedOp { RED_SUM = 0, RED_MAX = 1 };

__device__ __forceinline__ double nanmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, WAVE));
  return v;
}

// Block-wide reduction of KB values held by every thread; the result lands in
// out[0..KB) (shared memory, visible to all threads on return).  The order of
// operations is fixed, so results are bitwise reproducible.
template <int KB>
__device__ __forceinline__ void block_reduce(double (&v)[KB], int op, double* out) {
  __shared__ double s_wave[NWAVES][8];
  static_assert(KB <= 8, "at most 8 values per block reduction");
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
#pragma unroll
  for (int k = 0; k < KB; ++k) v[k] = (op == RED_SUM) ? wave_sum(v[k]) : wave_max(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < KB; ++k) s_wave[wv][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < KB) {
    double a = s_wave[0][threadIdx.x];
    for (int w = 1; w < NWAVES; ++w)
      a = (op == RED_SUM) ? a + s_wave[w][threadIdx.x] : nanmax(a, s_wave[w][threadIdx.x]);
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

__device__ __forceinline__ unsigned ld_acquire(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_relaxed(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned add_relaxed(unsigned* p, unsigned v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reduce src[0..cnt) (stride 1) for K rows of length ld, writing dst[k*dld+di].
__device__ __forceinline__ void reduce_rows(const double* src, int ld, int cnt, int K, int op,
                                            double* dst, int dld, int di) {
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  for (int k = wv; k < K; k += NWAVES) {
    const double* row = src + (size_t)k * ld;
    double a = (op == RED_SUM) ? 0.0 : -INFINITY;
    for (int r = lane; r < cnt; r += WAVE) a = (op == RED_SUM) ? a + row[r] : nanmax(a, row[r]);
    a = (op == RED_SUM) ? wave_sum(a) : wave_max(a);
    if (lane == 0) dst[(size_t)k * dld + di] = a;
  }
}

// Synchronise the team and reduce K per-workgroup values.  blk (shared memory)
// holds this workgroup's K values; on return out (shared memory) holds the
// team-wide reduction, identical in every workgroup.  K = 0 is a plain
// barrier.  The last arrival of each group sums that group's values (in rank
// order), the last group to arrive sums the group sums (in group order), so
// the result does not depend on arrival order.  Waiters poll the generation
// word with relaxed loads and acquire once.  Returns false if the team was
// aborted (a wait ran past its time budget); callers then leave the kernel.
__device__ __forceinline__ bool team_sync(const Team& tm, const double* blk, int K, int op,
                                          double* out) {
  __shared__ int s_role;  // 0 = waiter, 1 = last of its group, 2 = last overall
  __shared__ int s_ok;
  const int tid = threadIdx.x;
  if (tm.size == 1) {
    __syncthreads();
    for (int k = tid; k < K; k += BLOCK) out[k] = blk[k];
    __syncthreads();
    return true;
  }
  const int ngroups = (tm.size + TEAM_GROUP - 1) / TEAM_GROUP;
  const int grp = tm.rank / TEAM_GROUP;
  const int g0 = grp * TEAM_GROUP;
  const int gsz = tm.size - g0 < TEAM_GROUP ? tm.size - g0 : TEAM_GROUP;
  double* gsum = tm.partials + (size_t)KMAX * tm.size;  // [KMAX][ngroups]
  for (int k = tid; k < K; k += BLOCK) tm.partials[(size_t)k * tm.size + tm.rank] = blk[k];
  __syncthreads();
  unsigned g = 0;
  if (tid == 0) {
    g = ld_relaxed(&tm.ctl->gen);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned old = add_relaxed(&tm.ctl->grp[grp][0], 1u);
    s_role = (old == (unsigned)gsz - 1u) ? 1 : 0;
    s_ok = 1;
    if (s_role) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (s_role) {
    reduce_rows(tm.partials + g0, tm.size, gsz, K, op, gsum, ngroups, grp);
    __syncthreads();
    if (tid == 0) {
      st_relaxed(&tm.ctl->grp[grp][0], 0u);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned old = add_relaxed(&tm.ctl->count, 1u);
      s_role = (old == (unsigned)ngroups - 1u) ? 2 : 1;
      if (s_role == 2) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (s_role == 2) {
      reduce_rows(gsum, ngroups, ngroups, K, op, tm.result, 1, 0);
      __syncthreads();
      if (tid == 0) {
        st_relaxed(&tm.ctl->count, 0u);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        st_relaxed(&tm.ctl->gen, g + 1u);
      }
    }
  }
  if (s_role != 2 && tid == 0) {
    const uint64_t t0 = wall_clock64();
    int ok = 1;
    while (ok && ld_relaxed(&tm.ctl->gen) == g) {
      __builtin_amdgcn_s_sleep(1);
      if (ld_relaxed(&tm.ctl->abort)) ok = 0;
      else if (wall_clock64() - t0 > tm.spin_ticks) {
        st_relaxed(&tm.ctl->abort, 1u);
        ok = 0;
      }
    }
    s_ok = ok;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (!s_ok) return false;
  for (int k = tid; k < K; k += BLOCK) out[k] = tm.result[k];
  __syncthreads();
  return true;
}

}  // namespace pkr
