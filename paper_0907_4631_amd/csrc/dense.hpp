// Exponential of a small dense matrix by one workgroup, in float64: scaling
// and squaring as the paper takes from Higham for the augmented matrix
// (Sect. 3.1), with a degree-18 Taylor polynomial of the same accuracy in
// place of the degree-13 Pade approximant (no linear solve).  Matrices are
// row-major N x N in device memory (a per-team scratch region that stays in
// L2); products stage their operands in LDS.
#pragma once
#include "team.hpp"

namespace pkr {

constexpr int DENSE_LDS = 17408;  // doubles of LDS available to the dense routines

// Largest padded order (a multiple of 16) whose product runs on the matrix
// cores with both operands in LDS.
constexpr int MFMA_NMAX = 80;
static_assert(2 * MFMA_NMAX * MFMA_NMAX <= DENSE_LDS, "MFMA operands fit the dense LDS");
typedef double dbl4 __attribute__((ext_vector_type(4)));

// C = A B for N x N row-major matrices in device memory (an L2-resident
// scratch).  Up to N = MFMA_NMAX the matrix cores form 16 x 16 blocks of C
// from operands staged in LDS.  Above that, while both operands fit, A is
// staged transposed and B as is in LDS, zero-padded to a multiple of 4, and
// every thread accumulates a 4 x 4 block of C in registers from 16-byte LDS
// reads.  Up to N = 128 (at most one 4 x 4 block per thread) the same runs
// over panels of MM_KC values of k staged in turn; beyond that, one output
// entry per thread straight from memory.
__device__ __forceinline__ void wg_matmul(int N, const double* __restrict__ A,
                                          const double* __restrict__ B, double* __restrict__ C,
                                          double* L) {
  const int NN = N * N;
  const int N4 = (N + 3) & ~3;
  const int N16 = (N + 15) & ~15;
  if (N16 <= MFMA_NMAX) {
    // matrix cores: both operands in LDS as At[k][i] = A[i][k] and Bs[k][j],
    // zero-padded to a multiple of 16; each wavefront forms 16 x 16 blocks
    // of C with v_mfma_f64_16x16x4f64, four values of k per instruction.
    // Lane l supplies A[i0 + l%16][k + l/16] and B[k + l/16][j0 + l%16] and
    // receives C[i0 + l/16 + 4r][j0 + l%16] in element r of the result.
    double* At = L;
    double* Bs = L + N16 * N16;
    for (int e = threadIdx.x; e < N16 * N16; e += BLOCK) {
      const int r = e / N16, c = e - r * N16;
      const bool in = r < N && c < N;
      At[c * N16 + r] = in ? A[r * N + c] : 0.0;
      Bs[e] = in ? B[r * N + c] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int nb = N16 >> 4;
    const int lr = lane & 15, lk = lane >> 4;
    for (int blk = wv; blk < nb * nb; blk += NWAVES) {  // uniform per wavefront
      const int i0 = (blk / nb) * 16, j0 = (blk - (blk / nb) * nb) * 16;
      dbl4 acc = {0.0, 0.0, 0.0, 0.0};
      const double* pa = At + lk * N16 + i0 + lr;
      const double* pb = Bs + lk * N16 + j0 + lr;
#pragma unroll 4
      for (int k = 0; k < N16; k += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[k * N16], pb[k * N16], acc, 0, 0, 0);
      const int j = j0 + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + lk + 4 * r;
        if (i < N && j < N) C[i * N + j] = acc[r];
      }
    }
    __syncthreads();
    return;
  }
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

// Largest 1-norm of X for which the degree-18 Taylor polynomial T(X) of
// exp has a relative backward error of at most 2^-53: T(X) = exp(X + dX)
// with ||dX|| <= 2^-53 ||X||, from the power series of log(exp(-x) T(x))
// (computed exactly by taylor_theta.py beside these sources).
constexpr double TAYLOR18_THETA = 1.0908637192900361;

// Largest order whose whole exponential stays in LDS: two padded matrices,
// and at most two 16 x 16 blocks of each product per wavefront.
constexpr int EXPM_LDS_N = 80;
static_assert(2 * EXPM_LDS_N * EXPM_LDS_N <= DENSE_LDS, "two padded matrices fit the dense LDS");
static_assert((EXPM_LDS_N / 16) * (EXPM_LDS_N / 16) <= 2 * NWAVES, "two blocks per wavefront");

// One 16 x 16 block of At^T Bs on the matrix cores: At[k][i] and Bs[k][j] in
// LDS with row stride N16; lane l receives rows i0 + l/16 + 4r, column
// j0 + l%16 in element r.
__device__ __forceinline__ dbl4 mfma_block(const double* At, const double* Bs, int N16, int i0,
                                           int j0, int lr, int lk) {
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  const double* pa = At + lk * N16 + i0 + lr;
  const double* pb = Bs + lk * N16 + j0 + lr;
#pragma unroll 4
  for (int k = 0; k < N16; k += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[k * N16], pb[k * N16], acc, 0, 0, 0);
  return acc;
}

// exp(X) for N <= EXPM_LDS_N entirely in LDS: the same scaling, Taylor
// polynomial and Paterson-Stockmeyer scheme as wg_expm below, in two padded
// buffers, B0 the left operand transposed and B1 the right operand as is.
// The powers are formed as X^2 = X X, X^3 = X X^2, X^4 = X X^3 with X
// transposed in B0 throughout.  Each wavefront owns BPW 16 x 16 blocks of
// every product (blocks wv and wv + NWAVES) and keeps its entries of X, X^2
// and X^3 in registers for the Horner steps, so a product is its
// matrix-core instructions between two barriers, with no trip through
// memory.  The result is written to S + 4 N^2 (row-major).
template <int BPW>
__device__ __forceinline__ double* wg_expm_lds(int N, double* S, double* L, const double* a,
                                               double* out_norm1, int* out_s) {
  __shared__ double s_norm;
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
  const int N16 = (N + 15) & ~15, NB = N16 * N16;
  double* B0 = L;
  double* B1 = L + NB;
  constexpr int EPT = (EXPM_LDS_N * EXPM_LDS_N + BLOCK - 1) / BLOCK;
  // stage X (zero-padded), all of a thread's loads issued together
  double xv[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = tid + q * BLOCK, r = e / N16, c = e - r * N16;
    xv[q] = (e < NB && r < N && c < N) ? S[r * N + c] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = tid + q * BLOCK;
    if (e < NB) B1[e] = xv[q];
  }
  __syncthreads();
  // 1-norm: the largest absolute column sum
  {
    double v[1] = {0.0};
    for (int j = tid; j < N; j += BLOCK) {
      double s = 0.0;
      for (int i = 0; i < N; ++i) s += fabs(B1[i * N16 + j]);
      v[0] = nanmax(v[0], s);
    }
    block_reduce<1>(v, RED_MAX, &s_norm);
  }
  const double nrm = s_norm;
  int s = 0;
  if (nrm > TAYLOR18_THETA && nrm <= 1e300)  // non-finite: caller rejects
    s = (int)ceil(log2(nrm / TAYLOR18_THETA));
  const double scale = ldexp(1.0, -s);
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = tid + q * BLOCK, r = e / N16, c = e - r * N16;
    if (e < NB) {
      B0[c * N16 + r] = xv[q] * scale;
      B1[e] = xv[q] * scale;
    }
  }
  __syncthreads();
  const int nb = N16 >> 4;
  const int lr = lane & 15, lk = lane >> 4;
  bool act[BPW];
  int i0[BPW], j0[BPW];
  double x[BPW][4], x2[BPW][4], x3[BPW][4];
  bool diag[BPW][4];
  dbl4 c[BPW];
#pragma unroll
  for (int b = 0; b < BPW; ++b) {
    const int blk = wv + b * NWAVES;
    act[b] = blk < nb * nb;  // uniform per wavefront
    i0[b] = act[b] ? (blk / nb) * 16 : 0;
    j0[b] = act[b] ? (blk - (blk / nb) * nb) * 16 : 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0[b] + lk + 4 * r, j = j0[b] + lr;
      x[b][r] = act[b] ? B1[i * N16 + j] : 0.0;
      diag[b][r] = i == j && i < N;
    }
  }
  // C = B0^T B1 for this wavefront's blocks
  auto product = [&]() {
#pragma unroll
    for (int b = 0; b < BPW; ++b)
      if (act[b]) c[b] = mfma_block(B0, B1, N16, i0[b], j0[b], lr, lk);
  };
  // X^2, then X^3 (B1 <- X^2), then X^4 (B1 <- X^3)
  product();
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPW; ++b) {
    if (act[b]) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        x2[b][r] = c[b][r];
        B1[(i0[b] + lk + 4 * r) * N16 + j0[b] + lr] = c[b][r];
      }
    }
  }
  __syncthreads();
  product();
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPW; ++b) {
    if (act[b]) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        x3[b][r] = c[b][r];
        B1[(i0[b] + lk + 4 * r) * N16 + j0[b] + lr] = c[b][r];
      }
    }
  }
  __syncthreads();
  product();
  __syncthreads();
  // B0 <- X^4 (transposed), B1 <- Y = a16 I + a17 X + a18 X^2
#pragma unroll
  for (int b = 0; b < BPW; ++b) {
    if (act[b]) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0[b] + lk + 4 * r, j = j0[b] + lr;
        B0[j * N16 + i] = c[b][r];
        B1[i * N16 + j] = (diag[b][r] ? a[16] : 0.0) + a[17] * x[b][r] + a[18] * x2[b][r];
      }
    }
  }
  __syncthreads();
  // Horner in X^4: Y = B_h + X^4 Y for h = 3..0; the last Y also goes to B0
  // (transposed) as the left operand of the squarings
  for (int h = 3; h >= 0; --h) {
    product();
    __syncthreads();
    const double a0 = a[4 * h], a1 = a[4 * h + 1], a2 = a[4 * h + 2], a3 = a[4 * h + 3];
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
      if (act[b]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0[b] + lk + 4 * r, j = j0[b] + lr;
          const double y = c[b][r] + (diag[b][r] ? a0 : 0.0) + a1 * x[b][r] + a2 * x2[b][r] +
                           a3 * x3[b][r];
          B1[i * N16 + j] = y;
          if (h == 0) B0[j * N16 + i] = y;
        }
      }
    }
    __syncthreads();
  }
  for (int k = 0; k < s; ++k) {
    product();
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
      if (act[b]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0[b] + lk + 4 * r, j = j0[b] + lr;
          B0[j * N16 + i] = c[b][r];
          B1[i * N16 + j] = c[b][r];
        }
      }
    }
    __syncthreads();
  }
  double* E = S + 4 * (size_t)N * N;
  for (int e = tid; e < N * N; e += BLOCK) {
    const int r = e / N, cc = e - r * N;
    E[e] = B1[r * N16 + cc];
  }
  if (tid == 0) { *out_norm1 = nrm; *out_s = s; }
  __syncthreads();
  return E;
}

// E = exp(A) for the N x N matrix in S[0] (overwritten).  S must hold 8
// matrices of N*N doubles (6 are used); L is DENSE_LDS doubles of shared
// memory.  Returns (in shared out_*) the 1-norm of A and the number of
// squarings.  The result is in the returned pointer (inside S).
//
// Scaling and squaring as the paper takes from Higham, with the degree-18
// Taylor polynomial in place of the degree-13 Pade approximant: both reach
// double-precision backward error, and the polynomial needs no linear solve
// (the Pade solve, at one barrier per column, costs about as much as twelve
// products at order 58), at the price of about two more squarings (theta 1.09
// against 5.37).  T is evaluated by the Paterson-Stockmeyer scheme: X^2, X^3,
// X^4, then Horner in X^4 over blocks of four coefficients, seven products.
//
// With c0, c1 >= 0 only columns c0 and c1 of the result are valid: the last
// squaring then multiplies by those two columns alone, since the solver reads
// nothing else of the exponential (the saving the paper points out for the
// last column in Sect. 3.1).
__device__ __forceinline__ double* wg_expm(int N, double* S, double* L, double* out_norm1,
                                           int* out_s, int c0 = -1, int c1 = -1) {
  __shared__ double s_norm;
  __shared__ double s_a[20];  // Taylor coefficients 1/k!, k = 0..18, and a zero
  const int tid = threadIdx.x;
  const size_t NN = (size_t)N * N;
  double* X = S;
  double* X2 = S + NN;
  double* X3 = S + 2 * NN;
  double* X4 = S + 3 * NN;
  double* Y = S + 4 * NN;
  double* Z = S + 5 * NN;

  if (tid == 0) {
    double a = 1.0;
    s_a[0] = a;
    for (int k = 1; k <= 18; ++k) {
      a /= (double)k;
      s_a[k] = a;
    }
    s_a[19] = 0.0;
  }
  if (N <= 64) return wg_expm_lds<1>(N, S, L, s_a, out_norm1, out_s);
  if (N <= EXPM_LDS_N) return wg_expm_lds<2>(N, S, L, s_a, out_norm1, out_s);
  // 1-norm: the largest absolute column sum (the reduction's barriers also
  // publish s_a)
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
  if (nrm > TAYLOR18_THETA && nrm <= 1e300)  // non-finite: caller rejects
    s = (int)ceil(log2(nrm / TAYLOR18_THETA));
  const double scale = ldexp(1.0, -s);
  for (size_t e = tid; e < NN; e += BLOCK) X[e] *= scale;
  __syncthreads();
  const double* a = s_a;

  wg_matmul(N, X, X, X2, L);
  wg_matmul(N, X2, X, X3, L);
  wg_matmul(N, X2, X2, X4, L);
  // Y = B_4 = a16 I + a17 X + a18 X^2, then Y = B_j + X^4 Y for j = 3..0
  // with B_j = a_{4j} I + a_{4j+1} X + a_{4j+2} X^2 + a_{4j+3} X^3
  for (size_t e = tid; e < NN; e += BLOCK) {
    const int i = (int)(e / N), j = (int)(e - (size_t)i * N);
    Y[e] = (i == j ? a[16] : 0.0) + a[17] * X[e] + a[18] * X2[e];
  }
  __syncthreads();
  for (int b = 3; b >= 0; --b) {
    wg_matmul(N, X4, Y, Z, L);
    const double a0 = a[4 * b], a1 = a[4 * b + 1], a2 = a[4 * b + 2], a3 = a[4 * b + 3];
    for (size_t e = tid; e < NN; e += BLOCK) {
      const int i = (int)(e / N), j = (int)(e - (size_t)i * N);
      Y[e] = Z[e] + (i == j ? a0 : 0.0) + a1 * X[e] + a2 * X2[e] + a3 * X3[e];
    }
    __syncthreads();
  }
  double* cur = Y;
  double* nxt = Z;
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
