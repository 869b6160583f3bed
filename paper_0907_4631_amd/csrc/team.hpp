// Workgroup teams: the workgroups of one persistent (cooperatively launched)
// grid that solve one problem together.  A team owns a control block in
// device memory (arrival counter, generation, abort flag) and a partials
// buffer used by the fused "reduce and synchronise" primitive below.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pkr {

constexpr int BLOCK = 1024;              // threads per workgroup (one per CU)
constexpr int WAVE = 64;                 // CDNA wavefront
constexpr int NWAVES = BLOCK / WAVE;
constexpr int M_CAP = 128;               // largest Krylov dimension
constexpr int P_MAX = 8;                 // largest p
constexpr int KMAX = M_CAP + 8;          // widest team reduction
constexpr int NMAX_EXPM = M_CAP + P_MAX + 1;

constexpr int TEAM_GROUP = 16;            // workgroups per arrival group
constexpr int TEAM_MAX = 1024;            // largest team
constexpr int TEAM_NGROUPS = TEAM_MAX / TEAM_GROUP;
constexpr int FLAG_STRIDE = 32;           // one flag per 128-byte line

// Team control block in device memory (zeroed before every launch).  Every
// workgroup posts the epoch it reached in its own flag; the first workgroup
// of each group of TEAM_GROUP (the group leader) waits for its members'
// flags, and workgroup 0 waits for the group leaders' flags and then
// publishes the generation.  There are no read-modify-write atomics, so
// nothing serializes on one address.
struct TeamCtl {
  unsigned gen;      // generation number (last completed barrier)
  unsigned abort;    // set when a wait exceeded its time budget
  unsigned pad[FLAG_STRIDE - 2];
  unsigned garr[TEAM_NGROUPS][FLAG_STRIDE];  // group leaders' epochs
  unsigned arr[TEAM_MAX][FLAG_STRIDE];       // members' epochs
};

struct Team {
  int rank;            // this workgroup's index in the team
  int size;            // workgroups in the team
  unsigned* gen;       // the team's generation word
  unsigned* abort;     // abort flag shared by every team of the launch
  unsigned* garr;      // group leaders' epochs, FLAG_STRIDE apart
  unsigned* arr;       // members' epochs, FLAG_STRIDE apart
  double* partials;    // [KMAX][size] per-workgroup values, then [KMAX][groups] group sums
  double* result;      // [KMAX]
  uint64_t spin_ticks; // wall-clock budget of one wait
};

// Flag words a team of `size` workgroups needs (generation line, group lines,
// member lines).
__host__ __device__ inline size_t team_flag_words(int size) {
  return (size_t)FLAG_STRIDE * (1 + (size + TEAM_GROUP - 1) / TEAM_GROUP + size);
}

// A team whose flags live in `flags` (team_flag_words(size) zeroed words).
__device__ __forceinline__ Team make_team(int rank, int size, unsigned* flags, unsigned* abort,
                                          double* partials, double* result, uint64_t spin) {
  const int ngroups = (size + TEAM_GROUP - 1) / TEAM_GROUP;
  Team tm;
  tm.rank = rank;
  tm.size = size;
  tm.gen = flags;
  tm.abort = abort;
  tm.garr = flags + FLAG_STRIDE;
  tm.arr = flags + FLAG_STRIDE * (1 + ngroups);
  tm.partials = partials;
  tm.result = result;
  tm.spin_ticks = spin;
  return tm;
}

// Partials a team needs (doubles).
__host__ __device__ inline size_t team_partials(int size) {
  return (size_t)KMAX * (size + (size + TEAM_GROUP - 1) / TEAM_GROUP);
}

enum RedOp { RED_SUM = 0, RED_MAX = 1 };

__device__ __forceinline__ double nanmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

// Move a double between lanes with a DPP pattern (row_mask/bank_mask
// select the rows/banks written; other lanes keep `old`).
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ double dpp(double old, double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL,
                                             ROW_MASK, BANK_MASK, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL,
                                             ROW_MASK, BANK_MASK, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Wave-wide sum / max with DPP: quad swaps, half-row and row mirrors, then
// the row broadcasts 15 and 31; the total ends in lane 63 and is returned to
// every lane.  Fixed order of operations.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp<0xB1>(0.0, v);                 // quad_perm [1,0,3,2]
  v += dpp<0x4E>(0.0, v);                 // quad_perm [2,3,0,1]
  v += dpp<0x141>(0.0, v);                // row_half_mirror
  v += dpp<0x140>(0.0, v);                // row_mirror: row sums in every lane
  v += dpp<0x142, 0xa>(0.0, v);           // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xc>(0.0, v);           // row_bcast:31 into rows 2 and 3
  return lane_value(v, 63);
}

__device__ __forceinline__ double wave_max(double v) {
  v = nanmax(v, dpp<0xB1>(v, v));
  v = nanmax(v, dpp<0x4E>(v, v));
  v = nanmax(v, dpp<0x141>(v, v));
  v = nanmax(v, dpp<0x140>(v, v));
  v = nanmax(v, dpp<0x142, 0xa>(v, v));
  v = nanmax(v, dpp<0x143, 0xc>(v, v));
  return lane_value(v, 63);
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

// Reduce src rows: dst[k*dld+di] = op over src[k*ld + 0..cnt) for k < K.
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

// Wave 0 of the calling workgroup waits until flags[base .. base+cnt) (cnt <=
// 64, one per lane, FLAG_STRIDE apart) have all reached epoch e.  Returns 0
// if the team was aborted or the wait ran out of time (then sets abort).
__device__ __forceinline__ int wait_flags(const Team& tm, unsigned* flags, int cnt, unsigned e) {
  const int lane = threadIdx.x % WAVE;
  const uint64_t t0 = wall_clock64();
  int ok = 1;
  int all = 0;
  while (ok && !all) {
    const unsigned f = lane < cnt ? ld_relaxed(flags + (size_t)lane * FLAG_STRIDE) : e;
    all = __all((int)(f - e) >= 0);
    if (!all) {
      __builtin_amdgcn_s_sleep(1);
      if (ld_relaxed(tm.abort)) ok = 0;
      else if (wall_clock64() - t0 > tm.spin_ticks) {
        st_relaxed(tm.abort, 1u);
        ok = 0;
      }
    }
  }
  return ok;
}

// Synchronise the team and reduce K per-workgroup values.  blk (shared memory)
// holds this workgroup's K values; on return out (shared memory) holds the
// team-wide reduction, identical in every workgroup.  K = 0 is a plain
// barrier.  Group leaders sum their group's values in rank order and
// workgroup 0 sums the group sums in group order, so the result does not
// depend on timing.  Returns false if the team was aborted (a wait ran past
// its time budget); callers then leave the kernel.
__device__ __forceinline__ bool team_sync(const Team& tm, const double* blk, int K, int op,
                                          double* out) {
  __shared__ unsigned s_epoch;
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
  const bool leader = tm.rank == g0;
  double* gsum = tm.partials + (size_t)KMAX * tm.size;  // [KMAX][ngroups]
  for (int k = tid; k < K; k += BLOCK) tm.partials[(size_t)k * tm.size + tm.rank] = blk[k];
  __syncthreads();
  if (tid == 0) {
    const unsigned e = ld_relaxed(tm.gen) + 1u;
    s_epoch = e;
    s_ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    st_relaxed(tm.arr + (size_t)tm.rank * FLAG_STRIDE, e);
  }
  __syncthreads();
  const unsigned e = s_epoch;
  if (leader) {
    if (tid < WAVE) {
      const int ok = wait_flags(tm, tm.arr + (size_t)g0 * FLAG_STRIDE, gsz, e);
      if (tid == 0) {
        s_ok = ok;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
    }
    __syncthreads();
    if (!s_ok) return false;
    reduce_rows(tm.partials + g0, tm.size, gsz, K, op, gsum, ngroups, grp);
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      st_relaxed(tm.garr + (size_t)grp * FLAG_STRIDE, e);
    }
    if (tm.rank == 0) {
      if (tid < WAVE) {
        const int ok = wait_flags(tm, tm.garr, ngroups, e);
        if (tid == 0) {
          s_ok = ok;
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
      }
      __syncthreads();
      if (!s_ok) return false;
      reduce_rows(gsum, ngroups, ngroups, K, op, tm.result, 1, 0);
      __syncthreads();
      if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        st_relaxed(tm.gen, e);
      }
    }
  }
  if (tm.rank != 0 && tid == 0) {
    const uint64_t t0 = wall_clock64();
    int ok = 1;
    while (ok && (int)(ld_relaxed(tm.gen) - e) < 0) {
      __builtin_amdgcn_s_sleep(1);
      if (ld_relaxed(tm.abort)) ok = 0;
      else if (wall_clock64() - t0 > tm.spin_ticks) {
        st_relaxed(tm.abort, 1u);
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
