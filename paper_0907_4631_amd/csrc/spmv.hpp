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

// ---------------------------------------------------------------------------
// The same product over a workgroup's consecutive tiles with the staging
// double-buffered through the LDS DMA path (global_load_lds): the staged
// entries never pass through registers, so the next tile's indices (and, for
// float32 values, its values) are in flight while the current tile's rows
// gather x.  float64 values are read by each row straight from memory (two
// float64 staging buffers would not fit the LDS).  Per tile one workgroup
// barrier, which also waits for the DMA of the next tile.

template <typename VT>
struct SpmvPipe {
  static constexpr bool kStageVal = sizeof(VT) == 4;
  int col[2][TILE_NNZ];
  VT val[kStageVal ? 2 : 1][kStageVal ? TILE_NNZ : 1];
};

// Issue the DMA of tile [r0, r1)'s column indices (and float32 values) into
// buffer b.  One wave instruction copies 64 consecutive dwords; lanes past
// the range re-read its last dword (in bounds) into slots past it, which
// stay below TILE_NNZ.  A tile with more than TILE_NNZ entries is not staged.
template <typename VT>
__device__ __forceinline__ void spmv_pipe_stage(const int* __restrict__ rp,
                                                const int* __restrict__ ci,
                                                const VT* __restrict__ val, int r0, int r1,
                                                SpmvPipe<VT>& sp, int b) {
  const int base = rp[r0];
  const int cnt = rp[r1] - base;
  if (cnt > TILE_NNZ || cnt <= 0) return;
  const int lane = threadIdx.x % WAVE, e00 = (threadIdx.x / WAVE) * WAVE;
  for (int e0 = e00; e0 < cnt; e0 += BLOCK) {
    const int e = e0 + lane < cnt ? e0 + lane : cnt - 1;
    __builtin_amdgcn_global_load_lds(ci + base + e, &sp.col[b][e0], 4, 0, 0);
  }
  if constexpr (SpmvPipe<VT>::kStageVal) {
    for (int e0 = e00; e0 < cnt; e0 += BLOCK) {
      const int e = e0 + lane < cnt ? e0 + lane : cnt - 1;
      __builtin_amdgcn_global_load_lds(val + base + e, &sp.val[b][e0], 4, 0, 0);
    }
  }
}

// y_r = sum_k val[k] * load(col[k]) for the workgroup's rows [rb, re) in
// tiles of BLOCK rows; store(r, acc) receives each row's sum (threads past
// the end of a tile call nothing).  Every thread of the workgroup must call
// it with the same rb, re.  The row's sum is formed in the same order as
// spmv_tile's.
template <typename VT, typename AT, int GATHER, typename Load, typename Store>
__device__ __forceinline__ void spmv_pipelined(const int* __restrict__ rp,
                                               const int* __restrict__ ci,
                                               const VT* __restrict__ val, int rb, int re,
                                               SpmvPipe<VT>& sp, Load load, Store store) {
  static_assert(GATHER > 0, "gathered row walk");
  if (rb < re) spmv_pipe_stage<VT>(rp, ci, val, rb, rb + BLOCK < re ? rb + BLOCK : re, sp, 0);
  int b = 0;
  for (int r0 = rb; r0 < re; r0 += BLOCK, b ^= 1) {
    const int r1 = r0 + BLOCK < re ? r0 + BLOCK : re;
    const int r = r0 + threadIdx.x;
    int k0 = 0, k1 = 0;
    if (r < r1) {
      k0 = rp[r];
      k1 = rp[r + 1];
    }
    const int base = rp[r0];
    const int cnt = rp[r1] - base;
    // tile r0's DMA has landed and every wave is done with the other buffer
    __syncthreads();
    if (r1 < re) spmv_pipe_stage<VT>(rp, ci, val, r1, r1 + BLOCK < re ? r1 + BLOCK : re, sp, b ^ 1);
    if (r >= r1) continue;
    AT acc = AT(0);
    if (cnt <= TILE_NNZ) {
      const int* col = sp.col[b];
      for (int k = k0; k < k1; k += GATHER) {
        AT xv[GATHER], av[GATHER];
#pragma unroll
        for (int q = 0; q < GATHER; ++q) {
          const int kk = k + q < k1 ? k + q : k;
          if constexpr (SpmvPipe<VT>::kStageVal) av[q] = AT(sp.val[b][kk - base]);
          else av[q] = AT(val[kk]);
          xv[q] = load(col[kk - base]);
        }
#pragma unroll
        for (int q = 0; q < GATHER; ++q)
          if (k + q < k1) acc += av[q] * xv[q];
      }
    } else {
      for (int k = k0; k < k1; ++k) acc += AT(val[k]) * load(ci[k]);
    }
    store(r, acc);
  }
  // the last tile's buffer is free again
  __syncthreads();
}

}  // namespace pkr
