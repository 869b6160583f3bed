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
template <typename VT, typename AT, typename Load>
__device__ __forceinline__ AT spmv_tile(const int* __restrict__ rp, const int* __restrict__ ci,
                                        const VT* __restrict__ val, int r0, int r1,
                                        SpmvSmem<VT>& sm, Load load) {
  const int tid = threadIdx.x;
  const int base = rp[r0];
  const int cnt = rp[r1] - base;
  const int r = r0 + tid;
  AT acc = AT(0);
  if (cnt <= TILE_NNZ) {
    for (int e = tid; e < cnt; e += BLOCK) {
      sm.col[e] = ci[base + e];
      sm.val[e] = val[base + e];
    }
    __syncthreads();
    if (r < r1) {
      const int k0 = rp[r] - base, k1 = rp[r + 1] - base;
      for (int k = k0; k < k1; ++k) acc += AT(sm.val[k]) * load(sm.col[k]);
    }
    __syncthreads();
  } else if (r < r1) {
    const int k0 = rp[r], k1 = rp[r + 1];
    for (int k = k0; k < k1; ++k) acc += AT(val[k]) * load(ci[k]);
  }
  return acc;
}

}  // namespace pkr
