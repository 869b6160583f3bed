// CSR sparse matrix-vector product for one workgroup's tile of rows, with the
// tile's column indices and values staged through LDS by coalesced loads.
//
// A tile is BLOCK consecutive rows, one row per thread.  The nonzeros of the
// tile form one contiguous range [row_ptr[r0], row_ptr[r1]) of col_idx/val;
// the workgroup copies that range into LDS with unit-stride loads (every
// global load instruction of a wave covers 64 consecutive entries), then each
// thread walks its own row in LDS and gathers x.  Tiles whose range does not
// fit the LDS buffer fall back to direct loads.
#pragma once
#include "team.hpp"

namespace pkr {

constexpr int TILE_NNZ = 8 * BLOCK;  // staged nonzeros per tile (7-point rows fit)

template <typename VT>
struct SpmvSmem {
  int col[TILE_NNZ];
  VT val[TILE_NNZ];
};

// Returns sum_k val[k] * load(col[k]) for row r0 + threadIdx.x (0 for threads
// past r1).  load(c) must return the source entry c already in the
// accumulation type.  Contains two workgroup barriers; every thread of the
// workgroup must call it with the same r0, r1.
// GATHER > 0: the row walk loads GATHER entries of x together (predicated
// tail); GATHER = 0: one at a time.  The row's sum is formed in the same
// order either way.
template <typename VT, typename AT, int GATHER = 0, typename Load>
__device__ __forceinline__ AT spmv_tile(const int* __restrict__ rp, const int* __restrict__ ci,
                                        const VT* __restrict__ val, int r0, int r1,
                                        SpmvSmem<VT>& sm, Load load) {
  constexpr int SLOTS = TILE_NNZ / BLOCK;
  const int tid = threadIdx.x;
  const int r = r0 + tid;
  const int base = rp[r0];
  const int cnt = rp[r1] - base;
  AT acc = AT(0);
  if (cnt <= TILE_NNZ) {
    if constexpr (GATHER > 0) {
      // the row bounds and every staged entry are loaded before the first
      // LDS store
      int k0 = 0, k1 = 0;
      if (r < r1) {
        k0 = rp[r];
        k1 = rp[r + 1];
      }
      int cc[SLOTS];
      VT vv[SLOTS];
#pragma unroll
      for (int q = 0; q < SLOTS; ++q) {
        const int e = tid + q * BLOCK;
        if (e < cnt) {
          cc[q] = ci[base + e];
          vv[q] = val[base + e];
        }
      }
#pragma unroll
      for (int q = 0; q < SLOTS; ++q) {
        const int e = tid + q * BLOCK;
        if (e < cnt) {
          sm.col[e] = cc[q];
          sm.val[e] = vv[q];
        }
      }
      __syncthreads();
      if (r < r1) {
        k0 -= base;
        k1 -= base;
        for (int k = k0; k < k1; k += GATHER) {
          AT xv[GATHER], av[GATHER];
#pragma unroll
          for (int q = 0; q < GATHER; ++q) {
            const int kk = k + q < k1 ? k + q : k;
            av[q] = AT(sm.val[kk]);
            xv[q] = load(sm.col[kk]);
          }
#pragma unroll
          for (int q = 0; q < GATHER; ++q)
            if (k + q < k1) acc += av[q] * xv[q];
        }
      }
    } else {
      for (int e = tid; e < cnt; e += BLOCK) {
        sm.col[e] = ci[base + e];
        sm.val[e] = val[base + e];
      }
      __syncthreads();
      if (r < r1) {
        const int k0 = rp[r] - base, k1 = rp[r + 1] - base;
        for (int k = k0; k < k1; ++k) acc += AT(sm.val[k]) * load(sm.col[k]);
      }
    }
    __syncthreads();
  } else if (r < r1) {
    const int k0 = rp[r], k1 = rp[r + 1];
    for (int k = k0; k < k1; ++k) acc += AT(val[k]) * load(ci[k]);
  }
  return acc;
}

}  // namespace pkr
