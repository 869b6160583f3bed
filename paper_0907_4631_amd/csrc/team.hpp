// Workgroup teams: the workgroups of one persistent (cooperatively launched)
// grid that solve one problem together.  A team owns flags in device memory
// (one epoch per member and per group, a generation, the abort word) and a
// partials buffer used by the fused "reduce and synchronise" primitive below.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pkr {

constexpr int BLOCK = 1024;              // threads per workgroup (one per CU)
constexpr int WAVE = 64;                 // CDNA wavefront
constexpr int NWAVES = BLOCK / WAVE;
constexpr int M_CAP = 128;               // largest Krylov dimension
constexpr int P_MAX = 8;                 // largest p
constexpr int KMAX = 2 * M_CAP + 8;      // widest team reduction
constexpr int NMAX_EXPM = M_CAP + P_MAX + 1;

constexpr int TEAM_GROUP = 16;            // workgroups per arrival group
constexpr int TEAM_MAX = 1024;            // largest team
constexpr int TEAM_NGROUPS = TEAM_MAX / TEAM_GROUP;
constexpr int FLAG_STRIDE = 32;           // one flag per 128-byte line
constexpr int TEAM_GBUF = 4;              // group-sum buffers, used round robin by epoch

// Team control block in device memory (zeroed before every launch).  Every
// workgroup posts the epoch it reached in its own flag.  In a reduction of a
// few values (and a plain barrier) workgroup 0 waits for all flags and
// publishes the generation; in a wider one the first workgroup of each group
// of TEAM_GROUP (the group leader) waits for its members' flags and posts a
// group flag, which every workgroup waits for; a neighbour synchronisation
// waits for the flags of a range of workgroups only.  There are no
// read-modify-write atomics, so nothing serializes on one address.
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
  double* partials;    // [size][KMAX] per-workgroup values, then TEAM_GBUF x [groups][KMAX] group sums
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
  return (size_t)KMAX * (size + TEAM_GBUF * ((size + TEAM_GROUP - 1) / TEAM_GROUP));
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

// Agent-coherent data accesses (relaxed agent-scope atomics: written
// through to, and read from, the level shared by all XCDs) for the values of
// a light reduction, which publishes nothing else and so needs no cache-wide
// write-back or invalidation.
__device__ __forceinline__ void st_coh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Waves 0..ceil(cnt/64)-1 of the calling workgroup wait until the cnt flags
// at flags, FLAG_STRIDE apart (one per lane), have all reached epoch e; the
// workgroup then takes an agent-scope acquire (not when LIGHT: the caller
// reads only agent-coherent data published with the flags).  Returns false
// (in every thread) if the team was aborted or a wait ran out of time (then
// it sets abort).
template <bool LIGHT = false>
__device__ __forceinline__ bool wait_flags(const Team& tm, const unsigned* flags, int cnt,
                                           unsigned e) {
  __shared__ int s_bad;
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  if (wv * WAVE < cnt) {
    const int i = wv * WAVE + lane;
    const uint64_t t0 = wall_clock64();
    int all = 0, bad = 0;
    while (!all && !bad) {
      const unsigned f = i < cnt ? ld_relaxed(const_cast<unsigned*>(flags) + (size_t)i * FLAG_STRIDE)
                                 : e;
      all = __all((int)(f - e) >= 0);
      if (!all) {
        __builtin_amdgcn_s_sleep(1);
        if (ld_relaxed(tm.abort)) bad = 1;
        else if (wall_clock64() - t0 > tm.spin_ticks) {
          st_relaxed(tm.abort, 1u);
          bad = 1;
        }
      }
    }
    if (bad && lane == 0) s_bad = 1;
  }
  __syncthreads();
  if (!LIGHT) {
    if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __syncthreads();
  }
  return s_bad == 0;
}

// Synchronise the team and reduce K (<= KMAX) per-workgroup values.  blk
// (shared memory) holds this workgroup's K values; on return out (shared
// memory) holds the team-wide reduction, identical in every workgroup (sums
// in a fixed order, so bitwise reproducible for a given team size).  K = 0
// is a plain barrier.  Every workgroup writes its values contiguously and
// posts its epoch in its own 128-byte flag line; there are no
// read-modify-write atomics.
//  * K <= 8 (and plain barriers): workgroup 0 polls every flag, reduces the
//    values (one wave per value, lanes over workgroups) and publishes the
//    generation word, which the others poll.
//  * K > 8: the first workgroup of each group of TEAM_GROUP polls its members,
//    reduces their values in rank order and posts a group flag; every
//    workgroup then polls the group flags and reduces the group sums itself
//    in group order (no further publication step).
// Returns false if the team was aborted (a wait ran past its time budget);
// callers then leave the kernel.
// LIGHT: the values travel by agent-coherent stores and loads and the flags
// carry no release or acquire, so the sync publishes nothing but the values
// (no write-back of this workgroup's other global writes, no invalidation
// before later reads of other workgroups' data).  For reductions whose
// surrounding code reads only its own rows until a full synchronisation.
// nmax > 0: values k < nmax are reduced with RED_MAX whatever op is.
template <bool LIGHT = false>
__device__ __forceinline__ bool team_sync(const Team& tm, const double* blk, int K, int op,
                                          double* out, int nmax = 0) {
  __shared__ unsigned s_epoch;
  const int tid = threadIdx.x;
  if (tm.size == 1) {
    __syncthreads();
    for (int k = tid; k < K; k += BLOCK) out[k] = blk[k];
    __syncthreads();
    return true;
  }
  const int PS = KMAX;
  const int ngroups = (tm.size + TEAM_GROUP - 1) / TEAM_GROUP;
  unsigned* my = tm.arr + (size_t)tm.rank * FLAG_STRIDE;
  for (int k = tid; k < K; k += BLOCK) {
    double* dst = tm.partials + (size_t)tm.rank * PS + k;
    if (LIGHT) st_coh(dst, blk[k]);
    else *dst = blk[k];
  }
  // (LIGHT: every wave's coherent stores have completed at this barrier)
  if (LIGHT) __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) {
    const unsigned e = ld_relaxed(my) + 1u;  // this workgroup's own epoch count
    s_epoch = e;
    if (!LIGHT) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    st_relaxed(my, e);
  }
  __syncthreads();
  const unsigned e = s_epoch;
  if (K <= 8) {
    if (tm.rank == 0) {
      if (!wait_flags<LIGHT>(tm, tm.arr, tm.size, e)) return false;
      const int lane = tid % WAVE, wv = tid / WAVE;
      for (int k = wv; k < K; k += NWAVES) {
        const int opk = k < nmax ? RED_MAX : op;
        double a = (opk == RED_SUM) ? 0.0 : -INFINITY;
        for (int r = lane; r < tm.size; r += WAVE) {
          const double* src = tm.partials + (size_t)r * PS + k;
          const double v = LIGHT ? ld_coh(src) : *src;
          a = (opk == RED_SUM) ? a + v : nanmax(a, v);
        }
        a = (opk == RED_SUM) ? wave_sum(a) : wave_max(a);
        if (lane == 0) {
          if (LIGHT) st_coh(tm.result + k, a);
          else tm.result[k] = a;
        }
      }
      if (LIGHT) __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid == 0) {
        if (!LIGHT) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        st_relaxed(tm.gen, e);
      }
    } else {
      if (!wait_flags<LIGHT>(tm, tm.gen, 1, e)) return false;
    }
    for (int k = tid; k < K; k += BLOCK) out[k] = LIGHT ? ld_coh(tm.result + k) : tm.result[k];
    __syncthreads();
    return true;
  }
  // group sums rotate over TEAM_GBUF buffers by epoch: a leader may write a
  // later sync's sums while a slower workgroup of another group still reads
  // this one's, as long as only neighbour synchronisations (which do not
  // wait for that workgroup) lie between the two.  Between two reductions of
  // more than eight values the solver has at most one (the w-recurrence's
  // run of them ends in a one-value reduction, which waits for every
  // workgroup)
  double* gsum =
      tm.partials + ((size_t)tm.size + (size_t)(e % (unsigned)TEAM_GBUF) * ngroups) * PS;
  const int grp = tm.rank / TEAM_GROUP;
  const int g0 = grp * TEAM_GROUP;
  const int gsz = tm.size - g0 < TEAM_GROUP ? tm.size - g0 : TEAM_GROUP;
  if (tm.rank == g0) {
    if (!wait_flags<LIGHT>(tm, tm.arr + (size_t)g0 * FLAG_STRIDE, gsz, e)) return false;
    for (int k = tid; k < K; k += BLOCK) {
      double v[TEAM_GROUP];
#pragma unroll
      for (int r = 0; r < TEAM_GROUP; ++r) {
        const double* src = tm.partials + (size_t)(g0 + r) * PS + k;
        v[r] = r < gsz ? (LIGHT ? ld_coh(src) : *src) : 0.0;
      }
      const int opk = k < nmax ? RED_MAX : op;
      double a = v[0];
#pragma unroll
      for (int r = 1; r < TEAM_GROUP; ++r)
        if (r < gsz) a = (opk == RED_SUM) ? a + v[r] : nanmax(a, v[r]);
      if (LIGHT) st_coh(gsum + (size_t)grp * PS + k, a);
      else gsum[(size_t)grp * PS + k] = a;
    }
    if (LIGHT) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      if (!LIGHT) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      st_relaxed(tm.garr + (size_t)grp * FLAG_STRIDE, e);
    }
  }
  if (!wait_flags<LIGHT>(tm, tm.garr, ngroups, e)) return false;
  for (int k = tid; k < K; k += BLOCK) {
    double a = 0.0;
    bool first = true;
    for (int gb = 0; gb < ngroups; gb += 16) {
      double v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double* src = gsum + (size_t)(gb + q) * PS + k;
        v[q] = gb + q < ngroups ? (LIGHT ? ld_coh(src) : *src) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        if (gb + q < ngroups) {
          a = first ? v[q] : ((k < nmax || op != RED_SUM) ? nanmax(a, v[q]) : a + v[q]);
          first = false;
        }
      }
    }
    out[k] = a;
  }
  __syncthreads();
  return true;
}

// Row-block slot of a team rank and its inverse.  With a team size that is
// a multiple of 8, ranks with equal rank mod 8 (the workgroups of one XCD
// when the team starts at a multiple of 8) get neighbouring slots.
__host__ __device__ inline int team_slot(int rank, int size) {
  return size % 8 == 0 ? (rank % 8) * (size / 8) + rank / 8 : rank;
}
__host__ __device__ inline int team_rank_of_slot(int slot, int size) {
  return size % 8 == 0 ? (slot % (size / 8)) * 8 + slot / (size / 8) : slot;
}

// Neighbour synchronisation: this workgroup posts its next epoch, then waits
// until the workgroups owning row-block slots [slo, shi] have posted it too
// (an empty range waits for nobody).  Publishes this workgroup's earlier
// global writes to those that wait for it; it orders nothing else, so it
// replaces a barrier only where the data that follows depends on those
// slots alone.  Returns false if the team was aborted.
__device__ __forceinline__ bool team_neighbor_sync(const Team& tm, int slo, int shi) {
  __shared__ unsigned s_epoch;
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  if (tm.size == 1) {
    __syncthreads();
    return true;
  }
  unsigned* my = tm.arr + (size_t)tm.rank * FLAG_STRIDE;
  __syncthreads();
  if (tid == 0) {
    const unsigned e = ld_relaxed(my) + 1u;
    s_epoch = e;
    s_bad = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    st_relaxed(my, e);
  }
  __syncthreads();
  const unsigned e = s_epoch;
  const int cnt = shi - slo + 1;
  const int lane = tid % WAVE, wv = tid / WAVE;
  if (cnt > 0 && wv * WAVE < cnt) {
    const int i = wv * WAVE + lane;
    const unsigned* f =
        i < cnt ? tm.arr + (size_t)team_rank_of_slot(slo + i, tm.size) * FLAG_STRIDE : nullptr;
    const uint64_t t0 = wall_clock64();
    int all = 0, bad = 0;
    while (!all && !bad) {
      const unsigned v = f ? ld_relaxed(const_cast<unsigned*>(f)) : e;
      all = __all((int)(v - e) >= 0);
      if (!all) {
        __builtin_amdgcn_s_sleep(1);
        if (ld_relaxed(tm.abort)) bad = 1;
        else if (wall_clock64() - t0 > tm.spin_ticks) {
          st_relaxed(tm.abort, 1u);
          bad = 1;
        }
      }
    }
    if (bad && lane == 0) s_bad = 1;
  }
  __syncthreads();
  if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
  return s_bad == 0;
}

}  // namespace pkr
