// The adaptive solver of Niesen & Wright (Algorithm 3 with Algorithm 4) run
// by a team of workgroups of one persistent grid.
//
// Every workgroup owns a contiguous block of rows.  All vector work is
// row-local except the sparse products, which gather from vectors completed
// before the last team synchronisation (a team_sync, or in the Krylov steps
// a neighbour synchronisation with the workgroups owning the rows that the
// product reads).  Dot products are reduced with
// team_sync's fused deterministic reduction.  Scalar decisions (small matrix
// exponential, error estimate, step-size and dimension control) are made by
// workgroup 0 and published through the State block in device memory; every
// workgroup reads them after the next team_sync, so control flow is uniform
// across the team.
//
// Data layout in HBM (all column-major, leading dimensions padded to 64):
//   u            n          float64   output; also w_0
//   W            n x p      float64   w_1..w_p of eq. wrecurrence
//   V            n x (m+1)  T         Krylov basis
//   y0, y1       n          T         the candidate u and the product w of a Krylov step
//   H            (M_CAP+1) x M_CAP float64, row-major, one copy per workgroup
//                                     (workgroup 0's feeds the exponential)
//   ex           8 (m+p+1)^2 float64, the small exponential's scratch
#pragma once
#include "controller.hpp"
#include "dense.hpp"
#include "proposer.hpp"
#include "spmv.hpp"
#include "team.hpp"

namespace pkr {

enum {
  ST_OK = 0,
  ST_EINVAL = -1,
  ST_ENONFINITE = -4,
  ST_EMAXSTEPS = -5,
  ST_EABORT = -7,
};

struct Problem {
  int n, nnz, p;
  const int* rp;
  const int* ci;
  const void* val;          // CSR values, of the kernel's value type VT (float64 or float32)
  const double* b;          // n x (p+1), leading dimension ldb
  long long ldb;
  double* u;
  double t;                 // signed end time
  double tol;
  double tau_fixed;
  long long max_attempts;
  int symm, m_init, m_max, adapt_m, corrector, validate;
  int full_reorth;          // Lanczos: orthogonalise against every basis vector
  int fp32_flags;           // PHIPM_FP32_* bits (FP32 basis only)
  int fp32mode;             // the solve runs in FP32-basis mode
  int segment;              // SEG_*: which part of a chained FP32-basis solve this launch runs
  const float* proposer;    // MLP parameters, or null
  double* history;          // {tau, m, omega, valid} carried across calls, or null
  struct TraceStep* trace;  // per accepted step records, or null
  int trace_cap, pad;
};

// One accepted step as recorded for training the proposer (mirrors
// phipm_trace_step): the features seen at the start of the step, the step's
// outcome and the Krylov data that hindsight labelling needs (the leading
// (m_have+1) x m_have block of H, row-major with stride M_CAP).
struct TraceStep {
  float feat[MLP_IN];
  int m_use, m_have, p, lanczos;
  int n, nnz, attempts, pad;
  double t, tau, omega, beta, anorm, t_end, tol, pad_d;
  double H[(M_CAP + 1) * M_CAP];
};

struct Stats {              // mirrors phipm_stats
  long long steps, rejected, matvecs, expms;
  double t_reached, tau_last;
  int m_last, status, lanczos, workgroups;
  double anorm;
  int setup_flags, pad;
  double bytes;
  double rho_max;
  long long prec_rejects;
  double fp32_err;          // accumulated FP32 rounding estimate (absolute)
  int fp64_steps, trace_len;
  long long proposals;      // steps seeded by the proposer
  double bytes_ref;         // the same passes priced by the plain CGS2 byte model
  double krylov_bytes_ref;  // the Krylov builds' part of bytes_ref
  double krylov_ticks;      // wall-clock ticks workgroup 0 spent in Krylov builds
};

struct State {
  double t_end, sgn, anorm, bnorm, bd_tol;
  double t, tau, beta;
  double bytes;             // algorithmic HBM bytes so far
  double bytes_ref;         // bytes of the plain CGS2 model (reference byte count)
  double krylov_bytes_ref;  // the Krylov builds' part of bytes_ref
  unsigned long long krylov_ticks;  // wall-clock ticks workgroup 0 spent in Krylov builds
  unsigned long long krylov_t0;     // wall clock at the start of the current build
  double unorm;             // ||u_k||_2 of the current state
  double rho_max;           // largest ||beta y|| / ||u_k|| seen (FP32 basis)
  long long prec_rejects;   // FP32 attempts repeated with the FP64 basis
  double fp32_err;          // sum over accepted FP32 steps of the rounding estimate
  int redo64;               // the last attempt is to be repeated with the FP64 basis
  // the decision of attempt a in slot a % 2: {accept, done, redo64, m}.  A
  // workgroup reads its slot after the decision's barrier; workgroup 0
  // rewrites that slot only two attempts later, after a barrier that every
  // workgroup reaches after reading it.
  int dec[2][4];
  int steps64;              // accepted steps built with the FP64 basis (FP32 mode)
  double tau_step0;         // tau and m at the start of the current step (before a
  int m_step0, pad5;        // proposal), restored when a chained launch hands it on
  // step history (proposer features, warm start, trace)
  float feat[MLP_IN];       // features at the start of the current step
  double tau_prev, omega_prev, tau_prop;
  int m_prev, m_prop, step_rejects, prev_rejects;
  long long proposals;
  int trace_len, pad4;
  int setup_flags, pad0;
  double eps, omega, knorm;
  int m, m_cap, lanczos, zero_path;
  int accept, done, status, m_use;
  double coef[P_MAX + 1];
  double yb[M_CAP + 2];     // beta*y (0..m_use-1), corrector coefficient at [m_use]
  Alg4Mem mem;
  long long steps, rejected, matvecs, expms, attempts;
  double tau_last;
  int m_last, pad;
};

template <typename T>
struct Work {
  double* W;
  long long ldw;
  T* V;
  long long ldv;
  T* y0;
  T* y1;
  double* H;    // Hessenberg matrix, row stride M_CAP: workgroup 0's copy
  double* ex;
  State* st;
  Stats* stats;
  double* Hm;   // this workgroup's copy of H (== H in workgroup 0)
};

// Doubles of one copy of H.
constexpr size_t H_WORDS = (size_t)(M_CAP + 1) * M_CAP;

struct Shared {
  union {
    SpmvSmem<double> sm64;
    SpmvSmem<float> sm32;
    SpmvPipe<double> pipe64;
    SpmvPipe<float> pipe32;
    double dense[DENSE_LDS];  // workgroup 0's small-matrix work
    struct {
      double wpart[NWAVES][KMAX];  // per-wave partial dot products (phase_dots2)
      double stage[2][BLOCK];      // u and w rows staged by phase_dots2
    };
  };
  double blk[KMAX];
  double red[KMAX];
  double h1[KMAX];
  double qv[KMAX];
  double coef[P_MAX + 1];
  double yb[M_CAP + 2];
  double hcol[M_CAP + 1];  // first-pass entries of the newest column of H
  int dep_lo, dep_hi;  // row-block slots whose rows this workgroup's products read
};

// Statistics updates from the Krylov steps (workgroup 0, one thread): no-return
// atomics, so the thread does not wait for the old values.
__device__ __forceinline__ void add_matvec(State* st, double bytes) {
  atomicAdd(reinterpret_cast<unsigned long long*>(&st->matvecs), 1ull);
  atomicAdd(&st->bytes, bytes);
}
__device__ __forceinline__ void add_bytes(State* st, double bytes) { atomicAdd(&st->bytes, bytes); }

// Algorithmic HBM bytes of one CSR product y = A x with values of sv bytes
// and vectors of s bytes.
__device__ __forceinline__ double spmv_bytes(const Problem& P, double sv, double s) {
  return (sv + 4.0) * P.nnz + 4.0 * (P.n + 1.0) + 2.0 * s * P.n;
}

// Reference byte model of one Krylov step that builds basis vector j + 1
// (0-based j) with plain CGS2, whatever this solver's fused passes stream:
// the product plus two Gram-Schmidt passes that each read the j + 1 basis
// vectors twice, plus the traffic of w and the normalisation, (4 (j + 1) + 8)
// vectors (Arnoldi); a Lanczos step streams 16 vectors.
// For the `cnt` products j = j0 .. j0 + cnt - 1 of one build:
__device__ __forceinline__ double krylov_ref_bytes(const Problem& P, double sv, double s, int j0,
                                                   int cnt, bool lanczos) {
  // sum over j of 4 (j + 1) + 8 = 4 (cnt (j0 + 1) + cnt (cnt - 1) / 2) + 8 cnt
  const double c = cnt;
  const double vecs = lanczos ? 16.0 * c : 4.0 * (c * (j0 + 1.0) + 0.5 * c * (c - 1.0)) + 8.0 * c;
  return c * spmv_bytes(P, sv, s) + vecs * s * P.n;
}

// Rows owned by this workgroup.  When the team size is a multiple of 8 the
// blocks are dealt so that the workgroups of one XCD (hardware block ids
// congruent mod 8) hold neighbouring rows: the stencil gathers then stay in
// that XCD's L2.
// Rows per slot: an equal share padded to 64.
__device__ __forceinline__ long long row_chunk(int n, int size) {
  const long long chunk = ((long long)n + size - 1) / size;
  return (chunk + 63) / 64 * 64;
}

__device__ __forceinline__ void own_rows(const Team& tm, int n, int& rb, int& re) {
  const int slot = team_slot(tm.rank, tm.size);
  const long long chunk = row_chunk(n, tm.size);
  long long b = (long long)slot * chunk;
  rb = (int)(b < n ? b : n);
  long long e = b + chunk;
  re = (int)(e < n ? e : n);
}

template <typename T>
__device__ __forceinline__ SpmvSmem<T>& smem_for(Shared& sh);
template <>
__device__ __forceinline__ SpmvSmem<double>& smem_for<double>(Shared& sh) { return sh.sm64; }
template <>
__device__ __forceinline__ SpmvSmem<float>& smem_for<float>(Shared& sh) { return sh.sm32; }
template <typename T>
__device__ __forceinline__ SpmvPipe<T>& pipe_for(Shared& sh);
template <>
__device__ __forceinline__ SpmvPipe<double>& pipe_for<double>(Shared& sh) { return sh.pipe64; }
template <>
__device__ __forceinline__ SpmvPipe<float>& pipe_for<float>(Shared& sh) { return sh.pipe32; }

// Block sums over own rows (float64): blk[k] = V[:, i0+k] . w for k < K,
// and when with_u also blk[K+k] = V[:, i0+k] . u, blk[2K] = u . u,
// blk[2K+1] = u . w.  Jobs are the K basis columns and one (u.u, u.w) job.
// Each job gets the largest power-of-two share of the 16 wavefronts (at
// least one; with more jobs than wavefronts they go round robin), and a
// wavefront streams its share of the workgroup's rows of that column in
// 64-row chunks, so many independent loads are in flight; u and w are
// re-read from L1.  With more jobs than half the wavefronts and at most one
// row per thread, u and w are staged in LDS instead and each wavefront
// streams its columns with up to sixteen loads in flight per lane (the same
// per-job row order).  Partial sums are reduced with DPP and then across a
// job's wavefronts in a fixed order.
template <typename T>
__device__ __forceinline__ void phase_dots2(const T* V, long long ldv, int i0, int K, const T* U,
                                            const T* Wv, bool with_u, int rb, int re,
                                            Shared& sh) {
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int jobs = K + 1;
  int wpj = 1;
  while (2 * wpj * jobs <= NWAVES) wpj *= 2;
  const int seg = wv % wpj;
  // the rows of u and w were written by other threads of the workgroup
  __syncthreads();
  if (wpj == 1 && re - rb <= BLOCK) {
    // more jobs than half the wavefronts and one row per thread: u and w
    // are staged in LDS, and wavefront wv takes jobs wv, wv+16, ..., one per
    // pass over the rows with all rows of a lane loaded together, so its
    // global loads are basis columns only (per job the same row order as the
    // path below)
    constexpr int JC = 1;  // jobs per pass over the rows
    {
      const int r = rb + threadIdx.x;
      if (r < re) {
        sh.stage[0][threadIdx.x] = (double)U[r];
        sh.stage[1][threadIdx.x] = (double)Wv[r];
      }
    }
    __syncthreads();
    const int nj = wv < jobs ? (jobs - wv + NWAVES - 1) / NWAVES : 0;
    constexpr int RR = 16;  // rows per lane and iteration (all of them: rows <= BLOCK)
    for (int t0 = 0; t0 < nj; t0 += JC) {
      // a_t = sum v.w and b_t = sum v.u over the rows; the (u.u, u.w) job
      // reads u as its column, so a = u.w and b = u.u there.  Slots past
      // the wavefront's jobs read u too and are not stored.  No branches in
      // the loop: JC x RR loads in flight per lane.
      const T* src[JC];
#pragma unroll
      for (int t = 0; t < JC; ++t) {
        const int job = wv + (t0 + t) * NWAVES;
        src[t] = (t0 + t < nj && job < K) ? V + (long long)(i0 + job) * ldv : U;
      }
      double a[JC], b[JC];
#pragma unroll
      for (int t = 0; t < JC; ++t) a[t] = b[t] = 0.0;
      for (int r = rb + lane; r < re; r += RR * WAVE) {
        double v[RR][JC];
#pragma unroll
        for (int q = 0; q < RR; ++q) {
          const int rq = r + q * WAVE < re ? r + q * WAVE : r;
#pragma unroll
          for (int t = 0; t < JC; ++t) v[q][t] = (double)src[t][rq];
        }
#pragma unroll
        for (int q = 0; q < RR; ++q) {
          if (r + q * WAVE < re) {
            const double ur = sh.stage[0][r + q * WAVE - rb], wr = sh.stage[1][r + q * WAVE - rb];
#pragma unroll
            for (int t = 0; t < JC; ++t) {
              a[t] += v[q][t] * wr;
              b[t] += v[q][t] * ur;
            }
          }
        }
      }
#pragma unroll
      for (int t = 0; t < JC; ++t) {
        if (t0 + t < nj) {
          const int job = wv + (t0 + t) * NWAVES;
          const double x = wave_sum(a[t]), y = wave_sum(b[t]);
          if (lane == 0) {
            sh.wpart[0][2 * job] = job < K ? x : y;
            sh.wpart[0][2 * job + 1] = job < K ? (with_u ? y : 0.0) : x;
          }
        }
      }
    }
  } else {
    for (int job = wv / wpj; job < jobs; job += NWAVES / wpj) {
      double s0 = 0.0, s1 = 0.0;
      if (job < K) {
        const T* col = V + (long long)(i0 + job) * ldv;
#pragma unroll 4
        for (int r = rb + seg * WAVE + lane; r < re; r += WAVE * wpj) {
          const double v = (double)col[r];
          s0 += v * (double)Wv[r];
          if (with_u) s1 += v * (double)U[r];
        }
      } else {
#pragma unroll 4
        for (int r = rb + seg * WAVE + lane; r < re; r += WAVE * wpj) {
          const double ur = (double)U[r];
          s0 += ur * ur;
          s1 += ur * (double)Wv[r];
        }
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      if (lane == 0) {
        sh.wpart[seg][2 * job] = s0;
        sh.wpart[seg][2 * job + 1] = s1;
      }
    }
  }
  __syncthreads();
  for (int job = threadIdx.x; job < jobs; job += BLOCK) {
    double s0 = sh.wpart[0][2 * job], s1 = sh.wpart[0][2 * job + 1];
    for (int q = 1; q < wpj; ++q) {
      s0 += sh.wpart[q][2 * job];
      s1 += sh.wpart[q][2 * job + 1];
    }
    if (job < K) {
      sh.blk[job] = s0;
      sh.blk[K + job] = s1;
    } else {
      sh.blk[2 * K] = s0;
      sh.blk[2 * K + 1] = s1;
    }
  }
  __syncthreads();
}

// The same sums for a window of at most two columns (windowed Lanczos): one
// pass in which each thread reads its own rows of the columns, u and w once
// and forms all 2K + 2 terms (every wavefront busy, u and w read once), then
// one block reduction in a fixed order.  Layout of blk as phase_dots2's.
template <typename T>
__device__ __forceinline__ void phase_dots_window(const T* V, long long ldv, int i0, int K,
                                                  const T* U, const T* Wv, bool with_u, int rb,
                                                  int re, Shared& sh) {
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // v0.w, v1.w, v0.u, v1.u, u.u, u.w
  const T* va = V + (long long)i0 * ldv;
  const T* vb = va + ldv;
  for (int r = rb + (int)threadIdx.x; r < re; r += BLOCK) {
    const double u = (double)U[r], w = (double)Wv[r];
    const double a = K > 0 ? (double)va[r] : 0.0;
    const double b = K > 1 ? (double)vb[r] : 0.0;
    acc[0] += a * w;
    acc[1] += b * w;
    acc[2] += a * u;
    acc[3] += b * u;
    acc[4] += u * u;
    acc[5] += u * w;
  }
  block_reduce<6>(acc, RED_SUM, sh.qv);
  for (int k = threadIdx.x; k < K; k += BLOCK) {
    sh.blk[k] = sh.qv[k];
    sh.blk[K + k] = with_u ? sh.qv[2 + k] : 0.0;
  }
  if (threadIdx.x == 0) {
    sh.blk[2 * K] = sh.qv[4];
    sh.blk[2 * K + 1] = sh.qv[5];
  }
  __syncthreads();
}

// Team-uniform state of an incremental Krylov build.  Columns 0..have-1 of
// V are final; U holds the candidate for column `have` (orthogonalised once,
// not normalised) unless u_final, when it holds v_have itself.  Columns
// 0..have-2 of H are final, column have-1 holds its first-pass
// coefficients until finalised.
struct KrylovCtl {
  int have, u_final, broke, final_col;  // final_col: H column have-1 is final
  int products;                         // products with A made by this build
};

// Store written through to the level shared by all XCDs (an agent-scope
// relaxed atomic store): the vectors a step streams out are then not left
// dirty in this XCD's L2 for the next synchronisation's release to write
// back.
template <typename T>
__device__ __forceinline__ void st_wt(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// y = A x over the workgroup's rows [rb, re): ld(c) gives x_c in float64,
// st(r, y_r) takes each row's sum.  Double-buffered DMA staging (the next
// tile's indices and float32 values load while this tile gathers); float64
// values of long rows (more than six entries on average) use staged tiles
// instead, since the pipelined path reads float64 values row by row.
template <typename VT, typename Load, typename Store>
__device__ __forceinline__ void csr_product(const Problem& P, const VT* val, int rb, int re,
                                            Shared& sh, Load ld, Store st) {
  if (sizeof(VT) == 8 && (long long)P.nnz > 6ll * P.n) {
    for (int r0 = rb; r0 < re; r0 += BLOCK) {
      const int r1 = r0 + BLOCK < re ? r0 + BLOCK : re;
      const double acc = spmv_tile<VT, double, 8>(P.rp, P.ci, val, r0, r1, smem_for<VT>(sh), ld);
      const int r = r0 + threadIdx.x;
      if (r < r1) st(r, acc);
    }
  } else {
    spmv_pipelined<VT, double, 8>(P.rp, P.ci, val, rb, re, pipe_for<VT>(sh), ld, st);
  }
}

// Second pass of the candidate in U against columns [zb, j) of V and its
// norm.  The coefficients s go to sh.h1[0..K) (the caller adds them to
// column j-1 of H, with H[j][j-1] = beta).  beta comes from Pythagoras,
// beta^2 = u.u - |s|^2, unless the first pass left more than a quarter of
// ||u||^2 in span(V) (cancellation), when U is reorthogonalised in place
// and its norm reduced directly (one more team barrier; then sh.h1 is the
// applied correction and *applied is set).  Returns beta, or -1 on abort.
template <typename T>
__device__ __forceinline__ double second_pass(const Team& tm, const Work<T>& w, int zb, int j,
                                              double a, T* U, int rb, int re, bool* applied,
                                              Shared& sh) {
  const int K = j - zb;
  double ss = 0.0;
  {
    // every wavefront forms the same sum (lanes over k, fixed DPP order)
    double a = 0.0;
    for (int k = threadIdx.x % WAVE; k < K; k += WAVE) a += sh.h1[k] * sh.h1[k];
    ss = wave_sum(a);
  }
  double b2 = a - ss;
  *applied = false;
  if (!(ss <= 0.25 * a) || !(b2 > 0.0)) {
    double acc[1] = {0.0};
    for (int r = rb + threadIdx.x; r < re; r += BLOCK) {
      double ur = (double)U[r];
      for (int k = 0; k < K; ++k) ur -= sh.h1[k] * (double)w.V[(long long)(zb + k) * w.ldv + r];
      const T ut = T(ur);
      U[r] = ut;
      acc[0] += (double)ut * (double)ut;
    }
    block_reduce<1>(acc, RED_SUM, sh.blk);
    if (!team_sync<true>(tm, sh.blk, 1, RED_SUM, sh.qv)) return -1.0;
    b2 = sh.qv[0];
    *applied = true;
    __syncthreads();  // sh.qv is reused by the caller
  }
  return sqrt(b2 > 0.0 ? b2 : 0.0);
}

// One iteration j of the Krylov process, classical Gram-Schmidt applied
// twice with the second pass delayed by one iteration: the product w = A u_j
// of the candidate u_j, then ONE team reduction of V^T w, V^T u_j, u_j.u_j
// and u_j.w over the projection window, from which every workgroup derives
// (identically) the second-pass coefficients s and norm beta of u_j, hence
// v_j = (u_j - V s) / beta, column j-1 of H (first-pass + s, beta), and the
// first-pass coefficients of A v_j = (w - A V s) / beta through the Arnoldi
// relation A V s = V (H s) + beta s_{j-1} v_j.  A row-local pass then writes
// v_j and the next candidate; a plain team barrier publishes it for the
// next product.  In exact arithmetic V and H equal those of CGS2.
// Arnoldi projects against all previous columns; Lanczos against the two
// most recent ones (second pass of u_j over {j-2, j-1}, first pass of A v_j
// over {j-1, j}).  With seed != null (j = 0) v_0 = seed * seed_scale is
// gathered directly and stored.  Returns false if the team was aborted.
template <typename T, typename VT, typename S>
__device__ __forceinline__ bool krylov_iter(const Team& tm, const Problem& P, const Work<T>& w,
                                            const VT* valT, double sgn, bool lanczos, double bd_tol,
                                            KrylovCtl& kc, const S* seed, double seed_scale,
                                            int rb, int re, Shared& sh) {
  const int j = kc.have;
  T* U = w.y0;
  T* Wv = w.y1;
  const bool uf = kc.u_final != 0;
  // P1: w = A u_j
  if (seed) {
    T* v0 = w.V;
    for (int r0 = rb; r0 < re; r0 += BLOCK) {
      const int r1 = r0 + BLOCK < re ? r0 + BLOCK : re;
      auto ld = [&](int c) -> double { return (double)T(seed[c] * seed_scale); };
      const double acc = spmv_tile<VT, double>(P.rp, P.ci, valT, r0, r1, smem_for<VT>(sh), ld);
      const int r = r0 + threadIdx.x;
      if (r < r1) {
        Wv[r] = T(sgn * acc);
        const T v = T(seed[r] * seed_scale);
        v0[r] = v;
        U[r] = v;
      }
    }
  } else {
    auto ld = [&](int c) -> double { return (double)U[c]; };
    auto st = [&](int r, double acc) { st_wt(Wv + r, T(sgn * acc)); };
    csr_product<VT>(P, valT, rb, re, sh, ld, st);
  }
  // P2: one reduction over the window [zb, j)
  const int zb = lanczos ? (j > 2 ? j - 2 : 0) : 0;
  const int K = j - zb;
  // (the own rows of u and w were written by these same threads)
  if (lanczos) phase_dots_window<T>(w.V, w.ldv, zb, K, U, Wv, !uf, rb, re, sh);
  else phase_dots2<T>(w.V, w.ldv, zb, K, U, Wv, !uf, rb, re, sh);
  if (!team_sync<true>(tm, sh.blk, 2 * K + 2, RED_SUM, sh.red)) return false;
  const double a = sh.red[2 * K], c = sh.red[2 * K + 1];
  // z -> sh.red[0..K), s -> sh.h1[0..K)
  for (int k = threadIdx.x; k < K; k += BLOCK) sh.h1[k] = uf ? 0.0 : sh.red[K + k];
  __syncthreads();
  double beta = 1.0;
  bool applied = false;
  if (!uf) {
    beta = second_pass<T>(tm, w, zb, j, a, U, rb, re, &applied, sh);
    if (beta < 0.0) return false;
  }
  const double sj1 = (!uf && j > 0) ? sh.h1[K - 1] : 0.0;   // s_{j-1}
  if (!uf && beta <= bd_tol) {
    // invariant subspace: finalise column j-1 (every workgroup in its own
    // copy of H); there is no v_j
    for (int i = threadIdx.x; i < j; i += BLOCK)
      if (i >= zb) w.Hm[(long long)i * M_CAP + (j - 1)] = sh.hcol[i] + sh.h1[i - zb];
    if (threadIdx.x == 0) {
      w.Hm[(long long)j * M_CAP + (j - 1)] = beta;
      if (tm.rank == 0) {
        add_matvec(w.st, spmv_bytes(P, sizeof(VT), sizeof(T)) + (K + 2.0) * sizeof(T) * (double)P.n);
      }
    }
    __syncthreads();
    kc.broke = 1;
    kc.final_col = 1;
    kc.products += 1;
    return true;
  }
  // g = H s over rows [ub, j) from the stored H (its column j-1 still holds
  // the first pass: add s_i s_{j-1}); the coefficients of the row-local pass
  //   v_j = (u - V s) / beta
  //   u_{j+1} = w / beta - V q - (s_{j-1} + h_jj) v_j,  q = g / beta + h1
  // with h1 the first-pass coefficients of A v_j on the window.
  const int ub = lanczos ? (j > 3 ? j - 3 : 0) : 0;
  const int KU = j - ub;
  double sdz = 0.0;
  {
    double a = 0.0;
    for (int k = threadIdx.x % WAVE; k < K; k += WAVE) a += sh.h1[k] * sh.red[k];
    sdz = wave_sum(a);
  }
  const double ib = 1.0 / beta;
  const double hjj = uf ? c : (c - sdz) * ib * ib - sj1;   // first pass, row j of column j
  {
    // one wavefront per row of g, lanes across the columns of H (a row of H
    // is contiguous), so the reads of H are issued together
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    for (int i = wv; i < KU; i += NWAVES) {
      const int row = ub + i;
      double g = 0.0;
      if (!uf) {
        for (int k = lane; k < K; k += WAVE) {
          const int col = zb + k;
          if (row <= col + 1) g += w.Hm[(long long)row * M_CAP + col] * sh.h1[k];
        }
        g = wave_sum(g);
        if (row >= zb) g += sh.h1[row - zb] * sj1;
      }
      if (lane == 0) {
        const bool inwin = !lanczos || row == j - 1;
        const double z = row >= zb ? sh.red[row - zb] : 0.0;
        const double h1 = inwin ? (z - g) * ib : 0.0;
        sh.qv[i] = g * ib + h1;
        sh.blk[i] = h1;                                                     // column j of H
        sh.wpart[0][i] = (!applied && row >= zb) ? sh.h1[row - zb] : 0.0;  // s on [ub, j)
      }
    }
  }
  __syncthreads();
  // this workgroup's copy of H (g above has read it): column j-1 final,
  // column j first pass in rows [ub, j]; its other rows stay zero from the
  // solve's setup (a column never has entries outside its window and the
  // subdiagonal)
  // (sh.hcol holds column j-1's first pass and takes column j's)
  for (int i = threadIdx.x; i <= j; i += BLOCK) {
    if (!uf && j > 0 && i < j && i >= zb)
      w.Hm[(long long)i * M_CAP + (j - 1)] = sh.hcol[i] + sh.h1[i - zb];
    const double hv = i < ub ? 0.0 : (i < j ? sh.blk[i - ub] : hjj);
    if (i >= ub) w.Hm[(long long)i * M_CAP + j] = hv;
    sh.hcol[i] = hv;
  }
  if (threadIdx.x == 0) {
    if (!uf && j > 0) w.Hm[(long long)j * M_CAP + (j - 1)] = beta;
    if (tm.rank == 0) {
      // product (+ the v_0 store), the fused dots (K columns, u, w), the
      // row-local pass (KU columns, u, w read; v_j, u written)
      add_matvec(w.st, spmv_bytes(P, sizeof(VT), sizeof(T)) + (seed ? 2.0 : 0.0) * sizeof(T) * (double)P.n +
                           (K + 2.0 + KU + 2.0 + (uf ? 1.0 : 2.0)) * sizeof(T) * (double)P.n);
    }
  }
  // P3: row-local pass, then publish u_{j+1}
  const double tj = sj1 + hjj;
  T* vj = w.V + (long long)j * w.ldv;
  for (int r = rb + threadIdx.x; r < re; r += BLOCK) {
    double vs = 0.0, vq = 0.0;
    // two columns per iteration: their loads are issued together, the sums
    // stay in column order
    const T* vp = w.V + (long long)ub * w.ldv + r;
    for (int i = 0; i < KU; i += 2) {
      const double v0 = (double)vp[(long long)i * w.ldv];
      const double v1 = i + 1 < KU ? (double)vp[(long long)(i + 1) * w.ldv] : 0.0;
      vs += sh.wpart[0][i] * v0;
      vq += sh.qv[i] * v0;
      if (i + 1 < KU) {
        vs += sh.wpart[0][i + 1] * v1;
        vq += sh.qv[i + 1] * v1;
      }
    }
    const double ur = (double)U[r];
    const T vjt = uf ? T(ur) : T((ur - vs) * ib);
    if (!uf) st_wt(vj + r, vjt);
    st_wt(U + r, T((double)Wv[r] * ib - vq - tj * (double)vjt));
  }
  // the next product reads u_{j+1} only in the rows of the slots this
  // workgroup depends on
  if (!team_neighbor_sync(tm, sh.dep_lo, sh.dep_hi)) return false;
  kc.have = j + 1;
  kc.u_final = 0;
  kc.final_col = 0;
  kc.products += 1;
  return true;
}

// Finalise column have-1: second pass and norm of the candidate in U, then
// v_have into V[:, have] and U (the corrector's vector, and the start of
// any later extension).  Returns false if the team was aborted.
template <typename T>
__device__ __forceinline__ bool krylov_finalize(const Team& tm, const Problem& P,
                                                const Work<T>& w, bool lanczos, double bd_tol,
                                                KrylovCtl& kc, int rb, int re, Shared& sh) {
  if (kc.broke || kc.u_final || kc.have == 0) return true;
  const int j = kc.have;
  T* U = w.y0;
  const int zb = lanczos ? (j > 2 ? j - 2 : 0) : 0;
  const int K = j - zb;
  phase_dots2<T>(w.V, w.ldv, zb, K, U, U, true, rb, re, sh);
  if (!team_sync<true>(tm, sh.blk + K, K + 1, RED_SUM, sh.red)) return false;
  // sh.red[0..K) = V^T u, sh.red[K] = u.u
  const double a = sh.red[K];
  for (int k = threadIdx.x; k < K; k += BLOCK) sh.h1[k] = sh.red[k];
  __syncthreads();
  bool applied = false;
  const double beta = second_pass<T>(tm, w, zb, j, a, U, rb, re, &applied, sh);
  if (beta < 0.0) return false;
  for (int i = threadIdx.x; i < j; i += BLOCK)
    if (i >= zb) w.Hm[(long long)i * M_CAP + (j - 1)] = sh.hcol[i] + sh.h1[i - zb];
  if (threadIdx.x == 0) {
    w.Hm[(long long)j * M_CAP + (j - 1)] = beta;
    if (tm.rank == 0) add_bytes(w.st, (K + 1.0) * sizeof(T) * (double)P.n);
  }
  kc.final_col = 1;
  if (beta <= bd_tol) {
    __syncthreads();
    kc.broke = 1;
    return true;
  }
  const double ib = 1.0 / beta;
  T* vh = w.V + (long long)j * w.ldv;
  for (int r = rb + threadIdx.x; r < re; r += BLOCK) {
    double ur = (double)U[r];
    if (!applied)
      for (int k = 0; k < K; ++k) ur -= sh.h1[k] * (double)w.V[(long long)(zb + k) * w.ldv + r];
    const T v = T(ur * ib);
    vh[r] = v;
    U[r] = v;
  }
  if (tm.rank == 0 && threadIdx.x == 0) add_bytes(w.st, (K + 3.0) * sizeof(T) * (double)P.n);
  __syncthreads();
  kc.u_final = 1;
  return true;
}

enum { SOLVE_DONE = 0, SOLVE_ABORTED = -1 };

// Share of the tolerance the FP32 rounding estimates of a solve may take
// together (absolute, against max(1, ||u_k||)).
constexpr double FP32_BUDGET = 1.0;

// Scalars the decision step needs (passed by value so that the out-of-line
// call does not force the kernel arguments into private memory).
struct DecideArgs {
  double tol, tau_fixed, nnz, n;
  long long max_attempts;
  int p, adapt_m, corrector, have, broke;
  int fp32;        // this attempt's basis is FP32
  int fp32mode;    // the solve runs in FP32-basis mode (some steps may use FP64)
  TraceStep* trace;
  int trace_cap;
  int fp32_flags;  // PHIPM_FP32_* bits
  int window;      // windowed Lanczos: the eq. 4 cost of Lanczos (else Arnoldi's)
};

// FP32-basis option bits (phipm_opts.fp32_flags).
enum { FP32_ONLY = 1 };

// An FP32-basis solve runs as three chained launches on one stream: the
// FP64 solver from the setup while its steps need FP64 (SEG_LEAD), the FP32
// solver while they fit FP32 (SEG_FP32), the FP64 solver to the end
// (SEG_TAIL).  Each kernel then holds only its own basis type's code.  A
// launch that is not needed returns at once.  SEG_WHOLE: one launch does
// everything (FP64 mode; the batched kernel).
enum { SEG_WHOLE = 0, SEG_LEAD = 1, SEG_FP32 = 2, SEG_TAIL = 3 };

// Unit roundoff of the FP32 basis.
constexpr double EPS32 = 5.9604644775390625e-08;

// Workgroup 0: exponential of the augmented matrix, error estimate and the
// decisions of Algorithms 3 and 4 for one attempt.  Kept out of line: it is
// cold code with high register pressure.
__device__ __noinline__ void decide(DecideArgs a, State* st, const double* H, double* ex,
                                   double* L) {
  __shared__ double s_c, s_norm;
  __shared__ int s_sq;
  const int p = a.p;
  const int have = a.have;
  const bool broke = a.broke != 0;
  const double beta = st->beta;
  const int m = st->m;
  const int m_use = beta > 0.0 ? (have < m ? have : m) : m;
  double tau = st->tau;
  if (beta > 0.0 && broke && !(a.tau_fixed > 0.0)) tau = st->t_end - st->t;  // exact for any tau
  double eps = 0.0, hnext = 0.0, knorm = 0.0, c = 0.0;
  if (beta > 0.0) {
    hnext = broke ? 0.0 : H[(long long)m_use * M_CAP + (m_use - 1)];
    const int N = m_use + p + 1;
    double* K = ex;
    for (int e = threadIdx.x; e < N * N; e += BLOCK) {
      const int i = e / N, jj = e - i * N;
      double v = 0.0;
      if (i < m_use && jj < m_use) v = tau * H[(long long)i * M_CAP + jj];
      else if (i == 0 && jj == m_use) v = tau;
      else if (i >= m_use && i < m_use + p && jj == i + 1) v = tau;
      K[e] = v;
    }
    __syncthreads();
    const int col = p == 0 ? 0 : m_use + p - 1;
    const double* E = wg_expm(N, ex, L, &s_norm, &s_sq, col, m_use + p);
    for (int k = threadIdx.x; k < m_use; k += BLOCK) st->yb[k] = beta * E[(long long)k * N + col];
    if (threadIdx.x == 0) s_c = E[(long long)(m_use - 1) * N + m_use + p];
    __syncthreads();
    c = s_c;
    knorm = s_norm;
    eps = beta * fabs(hnext) * fabs(c);
  }
  if (threadIdx.x == 0) {
    const Alg4Mem mem0 = st->mem;  // restored when the attempt is repeated in FP64
    if (beta > 0.0) st->expms += 1;
    st->attempts += 1;
    const double t = st->t, t_end = st->t_end;
    const double omega = t_end * eps / (tau * a.tol);
    int accept;
    double tau_next = tau;
    int m_next = m_use;
    Alg4Mem& mem = st->mem;
    if (a.tau_fixed > 0.0) {
      accept = 1;
    } else if (!isfinite(omega)) {
      accept = 0;
      tau_next = tau / 5.0;
      mem.rejected = 0;
    } else {
      double tau_new, m_new;
      ctrl_alg4(mem, tau, m_use, eps, omega, &tau_new, &m_new);
      const double M = ctrl_M(knorm);
      const double rem = t_end - t;
      const double m_cost = m_new < 1.0 ? 1.0 : m_new;
      const bool lz = a.window != 0;
      const double c_tau = ctrl_C(rem, tau_new, ctrl_C1(lz, m_use, p, a.nnz, a.n, M));
      const double c_m = ctrl_C(rem, tau, ctrl_C1(lz, m_cost, p, a.nnz, a.n, M));
      accept = omega <= CTRL_DELTA;
      int m_cand = m_use;
      if (a.adapt_m && !broke) {
        double mm = m_new;
        const double lo = floor(0.75 * m_use), hi = ceil(4.0 * m_use / 3.0);
        if (mm < lo) mm = lo;
        if (mm < 1.0) mm = 1.0;
        if (mm > hi) mm = hi;
        if (mm > st->m_cap) mm = st->m_cap;
        m_cand = (int)mm;
      }
      const bool tau_branch =
          c_tau < c_m || !a.adapt_m || broke || (!accept && m_cand <= m_use);
      if (tau_branch) {
        double tn = tau_new;
        if (tn < tau / 5.0) tn = tau / 5.0;
        if (tn > 2.0 * tau) tn = 2.0 * tau;
        if (tn > rem) tn = rem;
        tau_next = tn;
      } else {
        m_next = m_cand;
      }
      mem.branch = tau_branch ? 1 : 2;
      mem.eps = eps;
      mem.tau = tau;
      mem.m = m_use;
      mem.rejected = !accept;
    }
    // FP32 basis.  The phi-part beta V y of eq. step carries the rounding of
    // the FP32 basis: to first order the basis is the exact Krylov basis of a
    // matrix within relative EPS32 of A, which perturbs the phi-part by about
    // EPS32 ||beta y|| (on the benchmark operators the error of a whole FP32
    // solve against the oracle is 0.1 to 1 times the sum of these estimates).
    // The estimates of the FP32 steps are summed; an attempt whose estimate
    // would take the sum past FP32_BUDGET tol max(1, ||u_k||) is repeated with
    // the FP64 basis at the same tau and m (the error estimate accepted it, so
    // this is not a rejection of Algorithm 3).
    double fp32_est = 0.0;
    if (a.fp32mode && beta > 0.0) {
      double ys = 0.0;
      for (int k = 0; k < m_use; ++k) ys += st->yb[k] * st->yb[k];
      const double rho = sqrt(ys) / (st->unorm > 0.0 ? st->unorm : 1.0);
      if (rho > st->rho_max) st->rho_max = rho;
      if (a.fp32) fp32_est = EPS32 * sqrt(ys);
    }
    st->redo64 = 0;
    if (a.fp32 && accept && !(a.fp32_flags & FP32_ONLY) && !(a.tau_fixed > 0.0) &&
        st->fp32_err + fp32_est > FP32_BUDGET * a.tol * fmax(1.0, st->unorm)) {
      accept = 0;
      st->redo64 = 1;
      st->prec_rejects += 1;
      tau_next = tau;
      m_next = m_use;
      mem = mem0;
    }
    st->eps = eps;
    st->omega = omega;
    st->knorm = knorm;
    st->accept = accept;
    st->m_use = m_use;
    if (accept && a.trace && beta > 0.0 && have > 0 && st->trace_len < a.trace_cap) {
      TraceStep* r = a.trace + st->trace_len;
      for (int i = 0; i < MLP_IN; ++i) r->feat[i] = st->feat[i];
      r->m_use = m_use;
      r->m_have = have;
      r->p = p;
      r->lanczos = st->lanczos;
      r->n = (int)a.n;
      r->nnz = (int)a.nnz;
      r->attempts = st->step_rejects + 1;
      r->pad = 0;
      r->t = t;
      r->tau = tau;
      r->omega = omega;
      r->beta = beta;
      r->anorm = st->anorm;
      r->t_end = t_end;
      r->tol = a.tol;
      r->pad_d = 0.0;
    }
    if (accept) {
      st->tau_prev = tau;
      st->m_prev = m_use;
      st->omega_prev = omega;
      st->prev_rejects = st->step_rejects;
      st->step_rejects = 0;
      st->tau_prop = tau_next;
      st->m_prop = m_next;
      double f = 1.0;
      for (int j = 0; j < p; ++j) {
        st->coef[j] = f;
        f *= tau / (double)(j + 1);
      }
      st->yb[m_use] = (beta > 0.0 && a.corrector && hnext != 0.0) ? beta * hnext * c : 0.0;
      double tn = t + tau;
      if (t_end - tn <= 4.0 * 2.220446049250313e-16 * t_end) tn = t_end;
      st->t = tn;
      st->steps += 1;
      st->fp32_err += fp32_est;
      if (a.fp32mode && !a.fp32) st->steps64 += 1;
      st->tau_last = tau;
      st->m_last = m_use;
      st->mem = Alg4Mem{};
      st->done = tn >= t_end;
      st->m = m_next;
      st->tau = tau_next < t_end - tn ? tau_next : t_end - tn;
    } else if (st->redo64) {
      st->tau = tau_next;
      st->m = m_next;
    } else {
      st->rejected += 1;
      st->step_rejects += 1;
      st->tau = tau_next;
      st->m = m_next;
    }
    if (!st->done && st->attempts >= a.max_attempts) {
      st->status = ST_EMAXSTEPS;
      st->done = 1;
      st->accept = 0;
    }
    int* dec = st->dec[st->attempts & 1];
    dec[0] = st->accept;
    dec[1] = st->done;
    dec[2] = st->redo64;
    dec[3] = st->m;
  }
  __syncthreads();
}

// Fraction of the proposer's predicted boundary substep that is attempted.
constexpr double PROPOSER_TAU_MARGIN = 0.7;

// Start of a step (workgroup 0 only): the features of eq. step's next
// substep and, with a proposer, its proposal for (tau, m).  The proposal is
// kept within [tau_plain, 8 tau_plain] and [floor(3 m_plain / 4), m_cap];
// the error estimate still decides every attempt.
__device__ __noinline__ void step_start(const float* proposer, double tol, int p, int adapt_m,
                                       double tau_fixed, State* st, double beta) {
  __shared__ float s_x[MLP_IN];
  __shared__ float s_h[MLP_H];
  __shared__ float s_y[MLP_OUT];
  if (threadIdx.x == 0) {
    const double an = st->anorm, te = st->t_end;
    float x[MLP_IN];
    x[F_STIFF] = log10c(an * te, -6.f, 12.f);
    x[F_RTOL] = log10c(tol / (st->bnorm > 0.0 ? st->bnorm : 1.0), -20.f, 4.f);
    x[F_P] = 0.25f * (float)p;
    x[F_SEED] = log10c(beta / (st->unorm > 0.0 ? st->unorm : 1.0), -20.f, 20.f);
    x[F_PROGRESS] = clampf((float)(st->t / te), 0.f, 1.f);
    x[F_TAU_PREV] = log10c(st->tau_prev * an, -12.f, 12.f);
    x[F_M_PREV] = (float)st->m_prev / 32.f;
    x[F_OMEGA_PREV] = log10c(st->omega_prev, -12.f, 6.f);
    x[F_REJ_PREV] = clampf(0.25f * (float)st->prev_rejects, 0.f, 4.f);
    x[F_TAU_PLAIN] = log10c(st->tau * an, -12.f, 12.f);
    x[F_M_PLAIN] = (float)st->m / 32.f;
    x[F_LANCZOS] = st->lanczos ? 1.f : 0.f;
    for (int i = 0; i < MLP_IN; ++i) {
      st->feat[i] = x[i];
      s_x[i] = x[i];
    }
  }
  __syncthreads();
  if (proposer) {
    if (threadIdx.x < WAVE) mlp_forward_wave(proposer, s_x, s_h, s_y);
    __syncthreads();
    if (threadIdx.x == 0) {
      const double an = st->anorm;
      const double rem = st->t_end - st->t;
      const double tp = st->tau;
      // the network predicts the largest admissible tau (omega = gamma); the
      // error estimate is steep in tau at large m, so aim a little below it
      double tau =
          (an > 0.0 && isfinite(s_y[0])) ? PROPOSER_TAU_MARGIN * pow(10.0, (double)s_y[0]) / an : tp;
      if (!(tau > 0.0) || !isfinite(tau)) tau = tp;
      // trust region: tau only upwards (up to 8x the plain controller's
      // choice), m down to Algorithm 3's own lower clamp floor(3 m / 4).  A
      // tau that is too large costs a rejection, after which Algorithm 4
      // reduces it; a tau below the plain choice would feed back through the
      // next step's features and could shrink the steps geometrically.
      tau = fmin(fmax(tau, tp), 8.0 * tp);
      if (tau > rem) tau = rem;
      double mm = isfinite(s_y[1]) ? rint(32.0 * (double)s_y[1]) : (double)st->m;
      mm = fmin(fmax(mm, fmax(1.0, floor(0.75 * (double)st->m))), (double)st->m_cap);
      if (tau_fixed <= 0.0) {
        st->tau = tau;
        if (adapt_m) st->m = (int)mm;
      }
      st->proposals += 1;
    }
  }
  __syncthreads();
}

// Build (or extend) the Krylov basis of w_p with basis type TB to `target`
// columns and finalise the last one.  Returns false if the team was aborted.
template <typename TB, typename VT>
__device__ __forceinline__ bool build_basis(const Team& tm, const Problem& P, const Work<TB>& w,
                                            const VT* val, double sgn, bool lanczos,
                                            double bd_tol, KrylovCtl& kc, int target,
                                            const double* wp, double beta, int rb, int re,
                                            Shared& sh) {
  kc.products = 0;
  // the start time goes to the state, not a register held across the loop
  if (tm.rank == 0 && threadIdx.x == 0) w.st->krylov_t0 = wall_clock64();
  while (!kc.broke && kc.have < target && kc.have < P.n) {
    const bool ok =
        kc.have == 0
            ? krylov_iter<TB, VT, double>(tm, P, w, val, sgn, lanczos, bd_tol, kc, wp, 1.0 / beta,
                                          rb, re, sh)
            : krylov_iter<TB, VT, double>(tm, P, w, val, sgn, lanczos, bd_tol, kc, nullptr, 0.0,
                                          rb, re, sh);
    if (!ok) return false;
  }
  if (!krylov_finalize<TB>(tm, P, w, lanczos, bd_tol, kc, rb, re, sh)) return false;
  if (kc.have >= P.n) kc.broke = 1;  // the whole space: exact for any tau
  if (tm.rank == 0 && threadIdx.x == 0 && kc.products > 0) {
    const double b =
        krylov_ref_bytes(P, sizeof(VT), sizeof(TB), kc.have - kc.products, kc.products, lanczos);
    w.st->bytes_ref += b;
    w.st->krylov_bytes_ref += b;
    w.st->krylov_ticks += wall_clock64() - w.st->krylov_t0;
  }
  return true;
}

// The FP64 build of a step inside the FP32-basis solver, out of line: the
// FP32 steps' inlined loop keeps its own register allocation.
template <typename VT>
__device__ __noinline__ bool build_basis64(const Team& tm, const Problem& P,
                                           const Work<double>& w, const VT* val, double sgn,
                                           bool lanczos, double bd_tol, KrylovCtl& kc, int target,
                                           const double* wp, double beta, int rb, int re,
                                           Shared& sh) {
  return build_basis<double, VT>(tm, P, w, val, sgn, lanczos, bd_tol, kc, target, wp, beta, rb,
                                 re, sh);
}

// eq. step with the corrected projection eq. phipapprox2 over the own rows:
// u = sum_{j<p} tau^j/j! w_j + sum_k (beta y)_k v_k (+ the corrector term).
// Coefficients in sh.coef / sh.yb.  Returns this thread's part of ||u||^2.
template <typename TB>
__device__ __forceinline__ double step_update(const Problem& P, const Work<TB>& w, int p, int mu,
                                              bool use_v, bool use_corr, int rb, int re,
                                              Shared& sh) {
  double un = 0.0;
  for (int r = rb + (int)threadIdx.x; r < re; r += BLOCK) {
    double s = p > 0 ? sh.coef[0] * P.u[r] : 0.0;
    for (int j = 1; j < p; ++j) s += sh.coef[j] * w.W[(long long)(j - 1) * w.ldw + r];
    if (use_v) {
      // four columns' loads issued together; the sum stays in column order
      const TB* vp = w.V + r;
      int k = 0;
      for (; k + 4 <= mu; k += 4) {
        const double v0 = (double)vp[(long long)k * w.ldv];
        const double v1 = (double)vp[(long long)(k + 1) * w.ldv];
        const double v2 = (double)vp[(long long)(k + 2) * w.ldv];
        const double v3 = (double)vp[(long long)(k + 3) * w.ldv];
        s += sh.yb[k] * v0;
        s += sh.yb[k + 1] * v1;
        s += sh.yb[k + 2] * v2;
        s += sh.yb[k + 3] * v3;
      }
      for (; k < mu; ++k) s += sh.yb[k] * (double)vp[(long long)k * w.ldv];
      if (use_corr) s += sh.yb[mu] * (double)vp[(long long)mu * w.ldv];
    }
    st_wt(P.u + r, s);
    un += s * s;
  }
  return un;
}

__device__ __noinline__ double step_update64(const Problem& P, const Work<double>& w, int p,
                                             int mu, bool use_v, bool use_corr, int rb, int re,
                                             Shared& sh) {
  return step_update<double>(P, w, p, mu, use_v, use_corr, rb, re, sh);
}

// Solve one problem.  Returns SOLVE_DONE, or SOLVE_ABORTED if a team wait ran
// out of time (the team must stop); the same in every workgroup of the team.
//
// With T = float (FP32-basis mode) each step chooses its basis type before
// its first attempt: FP32 unless the a-priori bound of its phi-part,
// ||tau^p phi_p(tau A) w_p|| <= beta tau^p / p! (A dissipative), could take
// the summed FP32 rounding estimates past their budget; then FP64 in the
// same buffers (sized for FP64).  decide() checks the actual estimate of
// every FP32 attempt and has it repeated in FP64 when it does not fit.
// kChain: T = float runs only FP32 steps and hands the others on to the
// chained FP64 launch (single solves); without it the FP32 solver builds
// those steps with the FP64 basis itself (the batched kernel, whose teams
// cannot relaunch).
template <typename T, typename VT, bool kChain>
__device__ __forceinline__ int solve(const Team& tm, const Problem& P, const Work<T>& w, Shared& sh) {
  State* st = w.st;
  const int tid = threadIdx.x;
  const int n = P.n, p = P.p;
  int rb, re;
  own_rows(tm, n, rb, re);
  constexpr bool fp32 = sizeof(T) == 4;
  const VT* val = static_cast<const VT*>(P.val);
  // the same buffers seen with an FP64 basis (steps that need it)
  const Work<double> w64{w.W, w.ldw, reinterpret_cast<double*>(w.V), w.ldv,
                         reinterpret_cast<double*>(w.y0), reinterpret_cast<double*>(w.y1), w.H,
                         w.ex, w.st, w.stats, w.Hm};
  const bool resume = P.segment == SEG_FP32 || P.segment == SEG_TAIL;

  // ---------------------------------------------------------------- setup
  if (resume) {
    // a chained launch: the state is in st; only the rows this workgroup's
    // products read (the setup scan's column extent) are found again
    int cmin = n, cmax = -1;
    for (int r = rb + tid; r < re; r += BLOCK) {
      const int k0 = P.rp[r], k1 = P.rp[r + 1];
      if (k1 > k0) {
        cmin = min(cmin, P.ci[k0]);
        cmax = max(cmax, P.ci[k1 - 1]);
      }
    }
    double cr[2] = {-(double)cmin, (double)cmax};
    block_reduce<2>(cr, RED_MAX, sh.h1);
    if (tid == 0) {
      const long long chunk = row_chunk(n, tm.size);
      const long long lo = (long long)(-sh.h1[0]), hi = (long long)sh.h1[1];
      if (hi < lo || hi < 0) {
        sh.dep_lo = 1;
        sh.dep_hi = 0;
      } else {
        const long long slo = (lo < 0 ? 0 : lo) / chunk, shi = (hi >= n ? n - 1 : hi) / chunk;
        sh.dep_lo = (int)slo;
        sh.dep_hi = (int)(shi < tm.size - 1 ? shi : tm.size - 1);
      }
    }
    __syncthreads();
  } else {
    // structure / finiteness / symmetry flags and the row sums of |A|
    double f[4] = {0.0, 0.0, 0.0, 0.0};  // bad, nonfinite, asym, max row sum
    int cmin = n, cmax = -1;             // columns the own rows reference
    const bool check_sym = P.symm < 0;
    // the right-hand sides in the same pass: max |b_k| for k < 4, u_0 = b_0
    // and ||b_0||^2
    double bmax[4] = {0.0, 0.0, 0.0, 0.0};
    double usq = 0.0;
    // entries above the diagonal minus entries below it (symmetry test)
    double cdiff = 0.0;
    for (int r = rb + tid; r < re; r += BLOCK) {
      {
        const double b0 = P.b[r];
        P.u[r] = b0;
        usq += b0 * b0;
        bmax[0] = nanmax(bmax[0], fabs(b0));
#pragma unroll
        for (int k = 1; k < 4; ++k)
          if (k <= p) bmax[k] = nanmax(bmax[k], fabs(P.b[(long long)k * P.ldb + r]));
      }
      const int k0 = P.rp[r], k1 = P.rp[r + 1];
      bool row_ok = true;
      if (P.validate) {
        if (k0 < 0 || k1 < k0 || k1 > P.nnz) { f[0] = 1.0; row_ok = false; }
        if (r == 0 && k0 != 0) f[0] = 1.0;
        if (r == n - 1 && k1 != P.nnz) f[0] = 1.0;
      }
      double s = 0.0;
      int prev = -1;
      int kup = k1;  // the row's first entry above the diagonal
      // (loops below avoid `break`: the compiler has dropped flag updates
      // after early exits from nested divergent loops)
      for (int k = k0; k < k1 && row_ok; ++k) {
        const int c = P.ci[k];
        const double a = (double)val[k];
        if (P.validate && (c < 0 || c >= n || c <= prev)) {
          f[0] = 1.0;
          row_ok = false;
        } else {
          prev = c;
          cmin = c < cmin ? c : cmin;
          cmax = c > cmax ? c : cmax;
          if (!isfinite(a)) f[1] = 1.0;
          s += fabs(a);
          if (check_sym) {
            cdiff += c > r ? 1.0 : (c < r ? -1.0 : 0.0);
            kup = (c > r && k < kup) ? k : kup;
            if (c == r && !(a == a)) f[2] = 1.0;  // a_rr == a_rr fails for NaN
          }
        }
      }
      if (check_sym && row_ok) {
        // a_rc == a_cr for every entry above the diagonal: binary searches of
        // rows c for column r, eight entries of the row at a time in lock
        // step, so that their loads are in flight together.  In a CSR matrix
        // with sorted, distinct columns in each row, mirroring maps the
        // entries above the diagonal one-to-one onto entries below it, so
        // with as many entries below as above (cdiff summed to zero over the
        // whole matrix) every entry below is covered as well.
        for (int kb = kup; kb < k1; kb += 8) {
          int lo[8], hi[8], pos[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            lo[q] = 0;
            hi[q] = -1;
            pos[q] = -1;
            if (kb + q < k1) {
              const int c = P.ci[kb + q];
              const int q0 = P.rp[c], q1 = P.rp[c + 1];
              if (q0 >= 0 && q1 <= P.nnz && q0 <= q1) {
                lo[q] = q0;
                hi[q] = q1 - 1;
              }
            }
          }
          bool more = true;
          while (more) {
            more = false;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              if (lo[q] <= hi[q]) {
                const int mid = (lo[q] + hi[q]) >> 1;
                const int cm = P.ci[mid];
                if (cm < r) lo[q] = mid + 1;
                else if (cm > r) hi[q] = mid - 1;
                else { pos[q] = mid; lo[q] = hi[q] + 1; }
                more = more || lo[q] <= hi[q];
              }
            }
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            if (kb + q < k1) {
              const bool mirrored = pos[q] >= 0 && (double)val[pos[q]] == (double)val[kb + q];
              f[2] = mirrored ? f[2] : 1.0;
            }
          }
        }
      }
      f[3] = nanmax(f[3], s);
    }
    {
      // sh.blk[0..8): the flags, the largest row sum and max |b_0..3|
      double f8[8] = {f[0], f[1], f[2], f[3], bmax[0], bmax[1], bmax[2], bmax[3]};
      block_reduce<8>(f8, RED_MAX, sh.blk);
    }
    // this workgroup's copy of H starts at zero: the Krylov steps write only
    // each column's window and subdiagonal
    for (size_t e = tid; e < H_WORDS; e += BLOCK) w.Hm[e] = 0.0;
    {
      // slots owning the referenced columns: the rows a product here reads
      double cr[2] = {-(double)cmin, (double)cmax};
      block_reduce<2>(cr, RED_MAX, sh.h1);
      if (tid == 0) {
        const long long chunk = row_chunk(n, tm.size);
        const long long lo = (long long)(-sh.h1[0]), hi = (long long)sh.h1[1];
        if (hi < lo || hi < 0) {
          sh.dep_lo = 1;
          sh.dep_hi = 0;
        } else {
          const long long slo = (lo < 0 ? 0 : lo) / chunk, shi = (hi >= n ? n - 1 : hi) / chunk;
          sh.dep_lo = (int)slo;
          sh.dep_hi = (int)(shi < tm.size - 1 ? shi : tm.size - 1);
        }
      }
      __syncthreads();
    }
    // max |b_k| for the columns past the first four (one pass each)
    for (int k = 4; k <= p; ++k) {
      double bm[1] = {0.0};
      const double* bk = P.b + (long long)k * P.ldb;
      for (int r = rb + tid; r < re; r += BLOCK) bm[0] = nanmax(bm[0], fabs(bk[r]));
      block_reduce<1>(bm, RED_MAX, sh.blk + 4 + k);
    }
    {
      double a2[2] = {usq, cdiff};
      block_reduce<2>(a2, RED_SUM, sh.blk + 5 + p);
    }
    // one team reduction: maxima for the first 5 + p values, ||b_0||^2 and
    // the count difference summed
    if (!team_sync(tm, sh.blk, 7 + p, RED_SUM, sh.red, 5 + p)) return SOLVE_ABORTED;
    if (tm.rank == 0 && tid == 0) {
      const double* o = sh.red;
      st->status = ST_OK;
      bool nonfinite = o[1] != 0.0 || !isfinite(o[3]) || !isfinite(P.t);
      for (int k = 0; k <= p; ++k) nonfinite = nonfinite || !isfinite(o[4 + k]);
      if (o[0] != 0.0) st->status = ST_EINVAL;
      else if (nonfinite) st->status = ST_ENONFINITE;
      st->sgn = P.t < 0.0 ? -1.0 : 1.0;
      st->t_end = fabs(P.t);
      st->anorm = o[3];
      double bn = o[4];
      for (int k = 1; k <= p && bn == 0.0; ++k) bn = o[4 + k];
      st->bnorm = bn;
      const bool asym = o[2] != 0.0 || o[6 + p] != 0.0;
      st->lanczos = P.symm < 0 ? !asym : (P.symm != 0);
      st->setup_flags = (o[0] != 0.0 ? 1 : 0) | (o[1] != 0.0 ? 2 : 0) | (asym ? 4 : 0);
      st->zero_path = (st->anorm == 0.0 || bn == 0.0 || st->t_end == 0.0);
      st->m_cap = P.m_max < n ? P.m_max : n;
      double tau;
      if (P.tau_fixed > 0.0) tau = P.tau_fixed;
      else tau = ctrl_tau0(P.tol, st->anorm, bn, 0.5 * (double)(P.m_init + P.m_max));
      if (!(tau > 0.0) || !isfinite(tau)) tau = st->t_end;
      if (tau > st->t_end) tau = st->t_end;
      int m0 = P.m_init < st->m_cap ? P.m_init : st->m_cap;
      // warm start: the previous call's proposal for the step after its last
      double om0 = 1.0;
      if (P.history && P.history[3] > 0.0 && P.tau_fixed <= 0.0) {
        const double ht = P.history[0];
        const double hm = P.history[1];
        if (ht > 0.0 && isfinite(ht)) tau = ht < st->t_end ? ht : st->t_end;
        if (hm >= 1.0 && isfinite(hm)) m0 = (int)fmin(hm, (double)st->m_cap);
        if (P.history[2] > 0.0 && isfinite(P.history[2])) om0 = P.history[2];
      }
      st->tau = tau;
      st->m = m0;
      st->tau_prev = tau;
      st->m_prev = m0;
      st->omega_prev = om0;
      st->tau_prop = tau;
      st->m_prop = m0;
      st->step_rejects = st->prev_rejects = 0;
      st->proposals = 0;
      st->trace_len = 0;
      st->t = 0.0;
      st->bd_tol = ldexp(st->anorm, -40);
      st->done = (st->status != ST_OK);
      st->steps = st->rejected = st->matvecs = st->expms = st->attempts = 0;
      st->tau_last = 0.0;
      st->m_last = 0;
      st->mem = Alg4Mem{};
      st->rho_max = 0.0;
      st->prec_rejects = 0;
      st->fp32_err = 0.0;
      st->redo64 = 0;
      st->steps64 = 0;
      st->unorm = sqrt(o[5 + p]);  // u_0 = b_0
      // (the mirror searches read about half the entries again)
      st->bytes = (check_sym ? 1.5 : 1.0) * (sizeof(VT) + 4.0) * P.nnz + 4.0 * (n + 1.0) +
                  8.0 * n * (p + 2.0);
      st->bytes_ref = 0.0;
      st->krylov_bytes_ref = 0.0;
      st->krylov_ticks = 0;
    }
    if (!team_sync(tm, nullptr, 0, RED_SUM, nullptr)) return SOLVE_ABORTED;
  }
  const double sgn = st->sgn;
  const double t_end = st->t_end;
  long long natt = st->attempts;  // attempts decided so far (the decision slots' index)
  if (st->status != ST_OK || st->done) goto finish;

  if (!resume && st->zero_path) {
    // A = 0, b = 0 or t = 0: u = sum_k t^k/k! b_k (phi_k(0) = 1/k!)
    for (int r = rb + tid; r < re; r += BLOCK) {
      double s = 0.0, f = 1.0;
      for (int k = 0; k <= p; ++k) {
        s += f * P.b[(long long)k * P.ldb + r];
        f *= sgn * t_end / (double)(k + 1);
      }
      P.u[r] = s;
    }
    if (tm.rank == 0 && tid == 0) {
      st->t = t_end;
      st->done = 1;
    }
    goto finish;
  }

  {
    // Lanczos orthogonalises against the two previous vectors, or (full
    // reorthogonalisation) against all of them like Arnoldi
    const bool lanczos = st->lanczos != 0 && !P.full_reorth;
    while (!st->done) {
      const double t = st->t;
      // ---- eq. wrecurrence: w_j = A w_{j-1} + sum_l t^l/l! b_{j+l} (A, b scaled by sgn)
      for (int j = 1; j <= p; ++j) {
        const double* wprev = j == 1 ? P.u : w.W + (long long)(j - 2) * w.ldw;
        double* wj = w.W + (long long)(j - 1) * w.ldw;
        double nrm = 0.0;
        auto ld = [&](int c) -> double { return wprev[c]; };
        auto stw = [&](int r, double acc) {
          double s = sgn * acc;
          double f = 1.0;  // t^l / l!, times the sign of b_{j+l}
          for (int l = 0; l <= p - j; ++l) {
            s += (((j + l) & 1) ? sgn * f : f) * P.b[(long long)(j + l) * P.ldb + r];
            f *= t / (double)(l + 1);
          }
          st_wt(wj + r, s);
          nrm += s * s;
        };
        csr_product<VT>(P, val, rb, re, sh, ld, stw);
        if (tm.rank == 0 && tid == 0) {
          st->bytes += spmv_bytes(P, sizeof(VT), 8.0) + 8.0 * n * (p - j + 1.0);
          st->bytes_ref += spmv_bytes(P, sizeof(VT), 8.0) + 3.0 * 8.0 * n;  // w-recurrence
        }
        if (j == p) {
          double a1[1] = {nrm};
          block_reduce<1>(a1, RED_SUM, sh.blk);
          if (!team_sync(tm, sh.blk, 1, RED_SUM, sh.red)) return SOLVE_ABORTED;
        } else {
          // the next product reads w_j only in the rows of the slots this
          // workgroup depends on
          if (!team_neighbor_sync(tm, sh.dep_lo, sh.dep_hi)) return SOLVE_ABORTED;
        }
      }
      if (p == 0) {
        double a = 0.0;
        if (tm.rank == 0 && tid == 0) st->bytes += 8.0 * n;
        for (int r = rb + tid; r < re; r += BLOCK) a += P.u[r] * P.u[r];
        double a1[1] = {a};
        block_reduce<1>(a1, RED_SUM, sh.blk);
        if (!team_sync(tm, sh.blk, 1, RED_SUM, sh.red)) return SOLVE_ABORTED;
      }
      const double beta = sqrt(sh.red[0]);
      if (tm.rank == 0 && tid == 0) {
        st->beta = beta;
        st->matvecs += p;
        if (!isfinite(beta)) { st->status = ST_ENONFINITE; }
      }
      if (!isfinite(beta)) goto finish;

      // ---- basis type of this step (FP32-basis mode), from the plain
      // controller's tau: FP32 unless the a-priori bound of the step's
      // phi-part, ||tau^p phi_p(tau A) w_p|| <= beta tau^p / p! (A
      // dissipative), could take the summed FP32 rounding estimates past
      // their budget.  Team-uniform: every workgroup derives it from the
      // same values.
      bool step64 = !fp32;
      if (P.fp32mode) {
        bool need64 = false;
        if (!(P.fp32_flags & FP32_ONLY) && !(P.tau_fixed > 0.0) && beta > 0.0) {
          double bnd = beta;
          const double tau0 = st->tau;
          for (int j = 1; j <= p; ++j) bnd *= tau0 / (double)j;
          need64 = st->fp32_err + EPS32 * bnd > FP32_BUDGET * P.tol * fmax(1.0, st->unorm);
        }
        // chained launches hand the step on at its start
        if ((P.segment == SEG_LEAD && !need64) || (P.segment == SEG_FP32 && need64)) goto finish;
        if constexpr (fp32 && !kChain) step64 = need64;
      }
      if (tm.rank == 0 && tid == 0) {
        st->tau_step0 = st->tau;
        st->m_step0 = st->m;
      }
      // features of this step; the proposer (if any) seeds tau and m
      if (P.proposer || P.trace) {
        if (tm.rank == 0) step_start(P.proposer, P.tol, p, P.adapt_m, P.tau_fixed, st, beta);
        if (P.proposer && !team_sync(tm, nullptr, 0, RED_SUM, nullptr)) return SOLVE_ABORTED;
      }
      const double* wp = p == 0 ? P.u : w.W + (long long)(p - 1) * w.ldw;

      // ---- attempts of this step (Algorithm 3 inner loop)
      KrylovCtl kc{0, 1, 0, 1, 0};  // v_0 = w_p / beta is final by construction
      const double bd_tol = st->bd_tol;
      auto build = [&](int target) -> bool {
        if constexpr (fp32 && !kChain) {
          if (step64)
            return build_basis64<VT>(tm, P, w64, val, sgn, lanczos, bd_tol, kc, target, wp, beta,
                                     rb, re, sh);
        }
        return build_basis<T, VT>(tm, P, w, val, sgn, lanczos, bd_tol, kc, target, wp, beta, rb,
                                  re, sh);
      };
      int m = st->m;
      for (;;) {
        if (beta > 0.0 && !build(m)) return SOLVE_ABORTED;
        const int have = kc.have;
        const bool broke = kc.broke != 0;
        if (tm.rank == 0) {
          DecideArgs da{P.tol, P.tau_fixed, (double)P.nnz, (double)n, P.max_attempts,
                        p, P.adapt_m, P.corrector, have, broke ? 1 : 0,
                        (fp32 && !step64) ? 1 : 0, P.fp32mode,
                        P.trace, P.trace_cap, P.fp32_flags, lanczos ? 1 : 0};
          decide(da, st, w.H, w.ex, sh.dense);
        }
        if (!team_sync(tm, nullptr, 0, RED_SUM, nullptr)) return SOLVE_ABORTED;
        // this attempt's slot: workgroup 0 may already be deciding the next
        // attempt (in the other slot) when a slow workgroup reads it
        const volatile int* dec = st->dec[++natt & 1];
        const bool accept = dec[0] != 0;
        const bool done = dec[1] != 0;
        const bool redo64 = dec[2] != 0;
        m = dec[3];
        if (!accept) {
          if (done) goto finish;  // attempt limit
          if (redo64) {
            // this FP32 attempt's rounding did not fit: the step again in FP64
            if constexpr (kChain) {
              // by the chained FP64 launch, from the step's start
              if (tm.rank == 0 && tid == 0) {
                st->tau = st->tau_step0;
                st->m = st->m_step0;
              }
              goto finish;
            } else {
              step64 = true;
              kc = KrylovCtl{0, 1, 0, 1, 0};
            }
          }
          continue;
        }
        // ---- eq. step with the corrected projection eq. phipapprox2
        const int mu = st->m_use;
        for (int k = tid; k < p; k += BLOCK) sh.coef[k] = st->coef[k];
        for (int k = tid; k <= mu; k += BLOCK) sh.yb[k] = st->yb[k];
        __syncthreads();
        const bool use_v = beta > 0.0;
        const bool use_corr = use_v && sh.yb[mu] != 0.0;
        double un[1];
        if constexpr (fp32 && !kChain) {
          un[0] = step64 ? step_update64(P, w64, p, mu, use_v, use_corr, rb, re, sh)
                         : step_update<T>(P, w, p, mu, use_v, use_corr, rb, re, sh);
        } else {
          un[0] = step_update<T>(P, w, p, mu, use_v, use_corr, rb, re, sh);
        }
        const double sv = step64 ? 8.0 : (double)sizeof(T);
        if (tm.rank == 0 && tid == 0) {
          st->bytes += 8.0 * n * (p > 0 ? p + 1.0 : 1.0) +
                       (use_v ? (mu + (use_corr ? 1.0 : 0.0)) * sv * (double)n : 0.0);
          st->bytes_ref += (p + mu + 2.0) * sv * (double)n;
        }
        block_reduce<1>(un, RED_SUM, sh.blk);
        if (!team_sync(tm, sh.blk, 1, RED_SUM, sh.red)) return SOLVE_ABORTED;
        if (tm.rank == 0 && tid == 0) st->unorm = sqrt(sh.red[0]);
        if (P.trace && use_v) {
          // training record: extend the basis (prefix-stable, tau-independent)
          // to m_cap columns so that hindsight labels can weigh every m,
          // then store H
          if (!kc.broke && !build(st->m_cap)) return SOLVE_ABORTED;
          const int mh = kc.have;
          if (tm.rank == 0) {
            const int slot = st->trace_len;
            if (slot < P.trace_cap) {
              double* dst = P.trace[slot].H;
              for (int e = tid; e < (mh + 1) * M_CAP; e += BLOCK) {
                const int jj = e % M_CAP;
                dst[e] = jj < mh ? w.H[e] : 0.0;
              }
              if (tid == 0) P.trace[slot].m_have = mh;
            }
            __syncthreads();
            if (tid == 0) st->trace_len = slot + 1;
          }
        }
        break;
      }
    }
  }

finish:
  if (tm.rank == 0 && tid == 0) {
    Stats* o = w.stats;
    o->steps = st->steps;
    o->rejected = st->rejected;
    o->matvecs = st->matvecs;
    o->expms = st->expms;
    o->t_reached = sgn * st->t;
    o->tau_last = st->tau_last;
    o->m_last = st->m_last;
    o->status = st->status;
    o->lanczos = st->lanczos;
    o->workgroups = tm.size;
    o->anorm = st->anorm;
    o->setup_flags = st->setup_flags;
    o->bytes = st->bytes;
    o->bytes_ref = st->bytes_ref;
    o->krylov_bytes_ref = st->krylov_bytes_ref;
    o->krylov_ticks = (double)st->krylov_ticks;
    o->rho_max = st->rho_max;
    o->prec_rejects = st->prec_rejects;
    o->fp32_err = st->fp32_err;
    o->fp64_steps = st->steps64;
    o->trace_len = st->trace_len;
    o->proposals = st->proposals;
    // the next call's warm start: the proposal for the step after the last
    if (P.history && st->status == ST_OK && st->steps > 0 && st->done) {
      P.history[0] = st->tau_prop;
      P.history[1] = (double)st->m_prop;
      P.history[2] = st->omega_prev;
      P.history[3] = 1.0;
    }
  }
  return SOLVE_DONE;
}

}  // namespace pkr
