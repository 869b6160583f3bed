// Exponential of a small dense matrix by one workgroup, in float64: the
// degree-13 diagonal Pade approximant with scaling and squaring that the
// paper prescribes for the augmented matrix (Sect. 3.1, following Higham).
// Matrices are row-major N x N in device memory (a per-team scratch region
// that stays in L2); the linear system of the Pade step is solved by
// Gauss-Jordan elimination with partial pivoting.
#pragma once
#include "team.hpp"

namespace pkr {

constexpr int DENSE_LDS = 17408;  // doubles of LDS available to the dense routines

// C = A B for N x N row-major matrices in device memory (an L2-resident
// scratch).  When both operands fit, A is staged transposed and B as is in
// LDS, zero-padded to a multiple of 4, and every thread accumulates a 4 x 4
// block of C in registers from 16-byte LDS reads.  Up to N = 128 (at most one
// 4 x 4 block per thread) the same runs over panels of MM_KC values of k
// staged in turn; beyond that, one output entry per thread straight from
// memory.
__device__ __forceinline__ void wg_matmul(int N, const double* __restrict__ A,
                                          const double* __restrict__ B, double* __restrict__ C,
                                          double* L) {
  const int NN = N * N;
  const int N4 = (N + 3) & ~3;
  if (2 * N4 * N4 <= DENSE_LDS) {
    double* At = L;             // At[k][i] = A[i][k]
    double* Bs = L + N4 * N4;   // Bs[k][j] = B[k][j]
    for (int e = threadIdx.x; e < N4 * N4; e += BLOCK) {
      const int r = e / N4, c = e - r * N4;
      const bool in = r < N && c < N;
      At[c * N4 + r] = in ? A[r * N + c] : 0.0;
      Bs[e] = in ? B[r * N + c] : 0.0;
    }
    __syncthreads();
    const int nb = N4 >> 2;
    for (int t = threadIdx.x; t < nb * nb; t += BLOCK) {
      const int ib = t / nb, jb = t - ib * nb;
      const int i0 = 4 * ib, j0 = 4 * jb;
      double c[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) c[a][b] = 0.0;
#pragma unroll 4
      for (int k = 0; k < N; ++k) {
        const double2 x01 = *reinterpret_cast<const double2*>(At + k * N4 + i0);
        const double2 x23 = *reinterpret_cast<const double2*>(At + k * N4 + i0 + 2);
        const double2 y01 = *reinterpret_cast<const double2*>(Bs + k * N4 + j0);
        const double2 y23 = *reinterpret_cast<const double2*>(Bs + k * N4 + j0 + 2);
        const double x[4] = {x01.x, x01.y, x23.x, x23.y};
        const double y[4] = {y01.x, y01.y, y23.x, y23.y};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) c[a][b] = fma(x[a], y[b], c[a][b]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (i0 + a < N && j0 + b < N) C[(i0 + a) * N + j0 + b] = c[a][b];
    }
    __syncthreads();
    return;
  }
  constexpr int MM_KC = 32;
  if ((N4 >> 2) * (N4 >> 2) <= BLOCK && 2 * MM_KC * N4 <= DENSE_LDS) {
    double* At = L;              // At[kk][i] = A[i][k0 + kk]
    double* Bs = L + MM_KC * N4; // Bs[kk][j] = B[k0 + kk][j]
    const int nb = N4 >> 2;
    const int t = threadIdx.x;
    const bool mine = t < nb * nb;
    const int ib = mine ? t / nb : 0, jb = mine ? t - ib * nb : 0;
    const int i0 = 4 * ib, j0 = 4 * jb;
    double c[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) c[a][b] = 0.0;
    for (int k0 = 0; k0 < N; k0 += MM_KC) {
      const int kc = N - k0 < MM_KC ? N - k0 : MM_KC;
      __syncthreads();  // the previous panel has been consumed
      for (int e = threadIdx.x; e < MM_KC * N4; e += BLOCK) {
        const int kk = e / N4, r = e - kk * N4;
        const bool in = r < N && kk < kc;
        At[e] = in ? A[r * N + k0 + kk] : 0.0;
        Bs[e] = in ? B[(k0 + kk) * N + r] : 0.0;
      }
      __syncthreads();
      if (mine) {
        for (int kk = 0; kk < kc; ++kk) {
          const double2 x01 = *reinterpret_cast<const double2*>(At + kk * N4 + i0);
          const double2 x23 = *reinterpret_cast<const double2*>(At + kk * N4 + i0 + 2);
          const double2 y01 = *reinterpret_cast<const double2*>(Bs + kk * N4 + j0);
          const double2 y23 = *reinterpret_cast<const double2*>(Bs + kk * N4 + j0 + 2);
          const double x[4] = {x01.x, x01.y, x23.x, x23.y};
          const double y[4] = {y01.x, y01.y, y23.x, y23.y};
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) c[a][b] = fma(x[a], y[b], c[a][b]);
        }
      }
    }
    if (mine) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (i0 + a < N && j0 + b < N) C[(i0 + a) * N + j0 + b] = c[a][b];
    }
    __syncthreads();
    return;
  }
  for (int e = threadIdx.x; e < NN; e += BLOCK) {
    const int i = e / N, j = e - i * N;
    const double* a = A + i * N;
    double s = 0.0;
#pragma unroll 2
    for (int k = 0; k < N; ++k) s = fma(a[k], B[k * N + j], s);
    C[e] = s;
  }
  __syncthreads();
}

// Pivot key: |v| as a float with the 8 low mantissa bits replaced by
// 255 - row, so that an unsigned max picks the largest |v| (to 2^-15
// relative) and, among equals, the smallest row.  Needs N <= 256.
__device__ __forceinline__ unsigned pivot_key(double v, int row) {
  const unsigned f = __float_as_uint((float)fabs(v));
  return (f & 0xffffff00u) | (255u - (unsigned)row);
}

// Wave-wide unsigned max with DPP (same pattern as wave_sum); the result is
// returned to every lane.
__device__ __forceinline__ unsigned wave_umax(unsigned v) {
  auto mx = [](unsigned a, int b) { return a > (unsigned)b ? a : (unsigned)b; };
  v = mx(v, __builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false));
  v = mx(v, __builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false));
  v = mx(v, __builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false));
  v = mx(v, __builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false));
  v = mx(v, __builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
  v = mx(v, __builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Gauss-Jordan elimination with P by columns in LDS (M, stride ld) and Q in
// registers (N <= 128), so that LDS and vector ALU work side by side.  Lanes
// own rows l and l+64 (the second half only when HI, i.e. N > 64).  P: the
// columns right of k are split over the wavefronts and updated in LDS;
// wavefront 0, which owns column k+1, posts the next pivot as the wave-wide
// maximum of its candidates' pivot keys.  Q: wavefront wv owns columns wv,
// wv+16, ... (at most 8) in registers and takes their pivot row and row k by
// lane reads.  One barrier per column; every entry gets the same update
// expression, the row exchange folded in.
template <bool HI>
__device__ __forceinline__ void gj_hybrid(int N, double* M, int ld, double* Q, unsigned* s_key) {
  constexpr int SL = 2 * WAVE / NWAVES;  // Q columns per wavefront for N = 128
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
  const int i0 = lane, i1 = lane + WAVE;
  const bool r0 = i0 < N, r1 = HI && i1 < N;
  double x0[SL], x1[SL];
#pragma unroll
  for (int sl = 0; sl < SL; ++sl) {
    const int c = wv + sl * NWAVES;
    x0[sl] = (c < N && r0) ? Q[i0 * N + c] : 0.0;
    x1[sl] = (c < N && r1) ? Q[i1 * N + c] : 0.0;
  }
  for (int k = 0; k < N; ++k) {
    const int piv = 255 - (int)(s_key[k & 1] & 0xffu);
    const double* colk = M + k * ld;
    const double inv = 1.0 / colk[piv];
    const double kk = colk[k];
    const double f0 = r0 ? colk[i0] : 0.0;
    const double f1 = r1 ? colk[i1] : 0.0;
    auto update = [&](double* col, bool cand) {
      const double pr = col[piv] * inv;
      const double kj = col[k];
      const double a0 = r0 ? col[i0] : 0.0;
      const double a1 = r1 ? col[i1] : 0.0;
      const double v0 = i0 == k ? pr : (i0 == piv ? kj - kk * pr : a0 - f0 * pr);
      const double v1 = i1 == k ? pr : (i1 == piv ? kj - kk * pr : a1 - f1 * pr);
      if (cand) {  // candidates for the next pivot: rows > k (one wavefront)
        const unsigned c0 = (r0 && i0 > k) ? pivot_key(v0, i0) : 0u;
        const unsigned c1 = (r1 && i1 > k) ? pivot_key(v1, i1) : 0u;
        const unsigned m = wave_umax(c0 > c1 ? c0 : c1);
        if (lane == 0) s_key[(k + 1) & 1] = m;
      }
      if (r0) col[i0] = v0;
      if (r1) col[i1] = v1;
    };
    for (int j = k + 1 + wv; j < N; j += NWAVES) update(M + j * ld, j == k + 1);
    const int pl = piv % WAVE, kl = k % WAVE;
    const bool phi = piv >= WAVE, khi = k >= WAVE;
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      if (wv + sl * NWAVES < N) {
        const double pr = lane_value(HI && phi ? x1[sl] : x0[sl], pl) * inv;
        const double kj = lane_value(HI && khi ? x1[sl] : x0[sl], kl);
        const double v0 = i0 == k ? pr : (i0 == piv ? kj - kk * pr : x0[sl] - f0 * pr);
        const double v1 = i1 == k ? pr : (i1 == piv ? kj - kk * pr : x1[sl] - f1 * pr);
        if (r0) x0[sl] = v0;
        if (HI && r1) x1[sl] = v1;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int sl = 0; sl < SL; ++sl) {
    const int c = wv + sl * NWAVES;
    if (c < N) {
      if (r0) Q[i0 * N + c] = x0[sl];
      if (r1) Q[i1 * N + c] = x1[sl];
    }
  }
  __syncthreads();
}

// Solve P X = Q in place (X overwrites Q) by Gauss-Jordan elimination with
// partial pivoting (P, Q row-major N x N in device memory).  Pivots are
// chosen with pivot keys, ties to the smallest row; the row exchange is
// folded into the update of each column (row k takes the scaled pivot row,
// the pivot row takes the eliminated old row k).  N <= 128: P by columns in
// LDS and Q in registers (gj_hybrid); larger N: in device memory.  L:
// DENSE_LDS doubles of shared memory.
__device__ __forceinline__ void wg_gauss_jordan(int N, double* P, double* Q, double* L) {
  const int tid = threadIdx.x;
  const int ld = (N + 1) & ~1;  // column stride of the transposed system in LDS
  if (N <= 2 * WAVE) {
    __shared__ unsigned s_key[2];
    double* M = L;  // P stored by columns: entry (i, j) at M[j * ld + i]
    if (tid == 0) { s_key[0] = 0u; s_key[1] = 0u; }
    for (int e = tid; e < N * N; e += BLOCK) {
      const int i = e / N, j = e - i * N;
      M[j * ld + i] = P[e];
    }
    __syncthreads();
    for (int i = tid; i < N; i += BLOCK) atomicMax(&s_key[0], pivot_key(M[i], i));
    __syncthreads();
    if (N <= WAVE) gj_hybrid<false>(N, M, ld, Q, s_key);
    else gj_hybrid<true>(N, M, ld, Q, s_key);
    return;
  }
  __shared__ int s_pivg;
  // large systems: the same elimination on the matrices in device memory
  __shared__ double s_fac[NMAX_EXPM];
  for (int k = 0; k < N; ++k) {
    if (tid < WAVE) {
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < N; i += WAVE) {
        double v = fabs(P[i * N + k]);
        if (v > best) { best = v; bi = i; }
      }
      for (int off = WAVE / 2; off > 0; off >>= 1) {
        double ob = __shfl_xor(best, off, WAVE);
        int oi = __shfl_xor(bi, off, WAVE);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) s_pivg = bi;
    }
    __syncthreads();
    const int piv = s_pivg;
    if (piv != k) {
      for (int j = tid; j < 2 * N; j += BLOCK) {
        double* M = j < N ? P : Q;
        const int c = j < N ? j : j - N;
        double t = M[k * N + c];
        M[k * N + c] = M[piv * N + c];
        M[piv * N + c] = t;
      }
      __syncthreads();
    }
    for (int i = tid; i < N; i += BLOCK) s_fac[i] = P[i * N + k];
    __syncthreads();
    const double inv = 1.0 / s_fac[k];
    for (int j = tid; j < 2 * N; j += BLOCK) {
      if (j < N) { if (j > k) P[k * N + j] *= inv; }
      else Q[k * N + (j - N)] *= inv;
    }
    __syncthreads();
    const int W = (N - k - 1) + N;
    for (int e = tid; e < N * W; e += BLOCK) {
      const int i = e / W;
      if (i == k) continue;
      const int jj = e - i * W;
      const double f = s_fac[i];
      if (f == 0.0) continue;
      if (jj < N - k - 1) {
        const int j = k + 1 + jj;
        P[i * N + j] -= f * P[k * N + j];
      } else {
        const int j = jj - (N - k - 1);
        Q[i * N + j] -= f * Q[k * N + j];
      }
    }
    __syncthreads();
  }
}

// C[:, c] = A B[:, c] for the two columns c0 and c1 of N x N row-major
// matrices (every row of those two columns; the rest of C is not written).
// The columns of B are staged in LDS; eight consecutive lanes share one
// output entry and add their partial sums with shuffles.
__device__ __forceinline__ void wg_matcols(int N, const double* __restrict__ A,
                                           const double* __restrict__ B, double* __restrict__ C,
                                           int c0, int c1, double* L) {
  for (int e = threadIdx.x; e < 2 * N; e += BLOCK)
    L[e] = B[(e < N ? e : e - N) * N + (e < N ? c0 : c1)];
  __syncthreads();
  for (int t0 = 0; t0 < 16 * N; t0 += BLOCK) {  // same trip count on every lane
    const int t = t0 + threadIdx.x;
    const int o = t >> 3, q = t & 7;
    const bool valid = o < 2 * N;
    const int i = valid ? (o < N ? o : o - N) : 0;
    const double* col = L + (o < N ? 0 : N);
    double acc = 0.0;
    if (valid)
      for (int j = q; j < N; j += 8) acc = fma(A[i * N + j], col[j], acc);
    acc += __shfl_xor(acc, 1, WAVE);
    acc += __shfl_xor(acc, 2, WAVE);
    acc += __shfl_xor(acc, 4, WAVE);
    if (valid && q == 0) C[i * N + (o < N ? c0 : c1)] = acc;
  }
  __syncthreads();
}

// E = exp(A) for the N x N matrix in S[0] (overwritten).  S must hold 8
// matrices of N*N doubles; L is DENSE_LDS doubles of shared memory.  Returns
// (in shared out_*) the 1-norm of A and the number of squarings.  The result
// is in the returned pointer (inside S).  With c0, c1 >= 0 only columns c0
// and c1 of the result are valid: the last squaring then multiplies by those
// two columns alone, since the solver reads nothing else of the exponential
// (the saving the paper points out for the last column in Sect. 3.1).
__device__ __forceinline__ double* wg_expm(int N, double* S, double* L, double* out_norm1,
                                           int* out_s, int c0 = -1, int c1 = -1) {
  __shared__ double s_norm;
  __shared__ double s_c[14];
  const int tid = threadIdx.x;
  const size_t NN = (size_t)N * N;
  double* X = S;
  double* X2 = S + NN;
  double* X4 = S + 2 * NN;
  double* X6 = S + 3 * NN;
  double* T = S + 4 * NN;
  double* U1 = S + 5 * NN;
  double* U = S + 6 * NN;
  double* Vv = S + 7 * NN;

  if (tid == 0) {
    // Pade-13 coefficients c_j = (26-j)! 13! / (26! j! (13-j)!) by their ratio
    double c = 1.0;
    s_c[0] = c;
    for (int j = 0; j < 13; ++j) {
      c = c * (double)(13 - j) / ((double)(j + 1) * (double)(26 - j));
      s_c[j + 1] = c;
    }
  }
  // 1-norm: the largest absolute column sum
  {
    double v[1] = {0.0};
    for (int j = tid; j < N; j += BLOCK) {
      double s = 0.0;
      for (int i = 0; i < N; ++i) s += fabs(X[i * N + j]);
      v[0] = nanmax(v[0], s);
    }
    block_reduce<1>(v, RED_MAX, &s_norm);
  }
  const double nrm = s_norm;
  int s = 0;
  if (nrm > 5.37 && nrm <= 1e300) s = (int)ceil(log2(nrm / 5.37));  // non-finite: caller rejects
  const double scale = ldexp(1.0, -s);
  for (size_t e = tid; e < NN; e += BLOCK) X[e] *= scale;
  __syncthreads();
  const double* c = s_c;

  wg_matmul(N, X, X, X2, L);
  wg_matmul(N, X2, X2, X4, L);
  wg_matmul(N, X4, X2, X6, L);
  for (size_t e = tid; e < NN; e += BLOCK) T[e] = c[13] * X6[e] + c[11] * X4[e] + c[9] * X2[e];
  __syncthreads();
  wg_matmul(N, X6, T, U1, L);
  for (size_t e = tid; e < NN; e += BLOCK) {
    const int i = (int)(e / N), j = (int)(e - (size_t)i * N);
    U1[e] += c[7] * X6[e] + c[5] * X4[e] + c[3] * X2[e] + (i == j ? c[1] : 0.0);
    T[e] = c[12] * X6[e] + c[10] * X4[e] + c[8] * X2[e];
  }
  __syncthreads();
  wg_matmul(N, X, U1, U, L);    // odd part
  wg_matmul(N, X6, T, Vv, L);   // even part (before the low-order terms)
  double* P = T;
  double* Q = U1;
  for (size_t e = tid; e < NN; e += BLOCK) {
    const int i = (int)(e / N), j = (int)(e - (size_t)i * N);
    const double ev = Vv[e] + c[6] * X6[e] + c[4] * X4[e] + c[2] * X2[e] + (i == j ? c[0] : 0.0);
    P[e] = ev - U[e];
    Q[e] = ev + U[e];
  }
  __syncthreads();
  wg_gauss_jordan(N, P, Q, L);
  double* cur = Q;
  double* nxt = U;
  const bool cols = c0 >= 0 && c1 >= 0;
  for (int k = 0; k < s; ++k) {
    if (cols && k == s - 1) wg_matcols(N, cur, cur, nxt, c0, c1, L);
    else wg_matmul(N, cur, cur, nxt, L);
    double* t = cur; cur = nxt; nxt = t;
  }
  if (tid == 0) { *out_norm1 = nrm; *out_s = s; }
  __syncthreads();
  return cur;
}

}  // namespace pkr
