// Exponential of a small dense matrix by one workgroup, in float64: the
// degree-13 diagonal Pade approximant with scaling and squaring that the
// paper prescribes for the augmented matrix (Sect. 3.1, following Higham).
// Matrices are row-major N x N in device memory (a per-team scratch region
// that stays in L2); the linear system of the Pade step is solved by
// Gauss-Jordan elimination with partial pivoting.
#pragma once
#include "team.hpp"

namespace pkr {

// C = A B for N x N row-major matrices; one output entry per thread.
__device__ __forceinline__ void wg_matmul(int N, const double* __restrict__ A,
                                          const double* __restrict__ B, double* __restrict__ C) {
  const int NN = N * N;
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

// Solve P X = Q in place (X overwrites Q) by Gauss-Jordan with row pivoting.
__device__ __forceinline__ void wg_gauss_jordan(int N, double* P, double* Q) {
  __shared__ double s_fac[NMAX_EXPM];
  __shared__ int s_piv;
  const int tid = threadIdx.x;
  for (int k = 0; k < N; ++k) {
    if (tid < WAVE) {  // one wave finds the pivot row
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
      if (tid == 0) s_piv = bi;
    }
    __syncthreads();
    const int piv = s_piv;
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
    // factors of column k (the pivot entry becomes the reciprocal)
    for (int i = tid; i < N; i += BLOCK) s_fac[i] = P[i * N + k];
    __syncthreads();
    const double inv = 1.0 / s_fac[k];
    // scale the pivot row
    for (int j = tid; j < 2 * N; j += BLOCK) {
      if (j < N) { if (j > k) P[k * N + j] *= inv; }
      else Q[k * N + (j - N)] *= inv;
    }
    __syncthreads();
    // eliminate column k from every other row
    const int W = (N - k - 1) + N;  // columns k+1..N-1 of P, all of Q
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

// E = exp(A) for the N x N matrix in S[0] (overwritten).  S must hold 8
// matrices of N*N doubles.  Returns (in shared out_*) the 1-norm of A and the
// number of squarings.  The result is in the returned pointer (inside S).
__device__ __forceinline__ double* wg_expm(int N, double* S, double* out_norm1, int* out_s) {
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

  wg_matmul(N, X, X, X2);
  wg_matmul(N, X2, X2, X4);
  wg_matmul(N, X4, X2, X6);
  for (size_t e = tid; e < NN; e += BLOCK) T[e] = c[13] * X6[e] + c[11] * X4[e] + c[9] * X2[e];
  __syncthreads();
  wg_matmul(N, X6, T, U1);
  for (size_t e = tid; e < NN; e += BLOCK) {
    const int i = (int)(e / N), j = (int)(e - (size_t)i * N);
    U1[e] += c[7] * X6[e] + c[5] * X4[e] + c[3] * X2[e] + (i == j ? c[1] : 0.0);
    T[e] = c[12] * X6[e] + c[10] * X4[e] + c[8] * X2[e];
  }
  __syncthreads();
  wg_matmul(N, X, U1, U);       // odd part
  wg_matmul(N, X6, T, Vv);      // even part (before the low-order terms)
  double* P = T;
  double* Q = U1;
  for (size_t e = tid; e < NN; e += BLOCK) {
    const int i = (int)(e / N), j = (int)(e - (size_t)i * N);
    const double ev = Vv[e] + c[6] * X6[e] + c[4] * X4[e] + c[2] * X2[e] + (i == j ? c[0] : 0.0);
    P[e] = ev - U[e];
    Q[e] = ev + U[e];
  }
  __syncthreads();
  wg_gauss_jordan(N, P, Q);
  double* cur = Q;
  double* nxt = U;
  for (int k = 0; k < s; ++k) {
    wg_matmul(N, cur, cur, nxt);
    double* t = cur; cur = nxt; nxt = t;
  }
  if (tid == 0) { *out_norm1 = nrm; *out_s = s; }
  __syncthreads();
  return cur;
}

}  // namespace pkr
