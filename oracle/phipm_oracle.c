/*
 * CPU oracle for the adaptive Krylov phi-function solver of Niesen & Wright.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, obviously-correct double-precision
 * implementation that the GPU library is checked against.  Only tests/, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code with the GPU path: the two sides meet only through seeded inputs.
 *
 * Every function follows the paper's steps in the paper's order.  Readings of
 * passages that are ambiguous or misprinted are marked "Reading:".  Sparse
 * products and inner products are OpenMP-parallel over rows; everything else
 * is straight loops.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- defaults */

void oracle_default_opts(oracle_opts* o) {
  memset(o, 0, sizeof(*o));
  o->tol = 1e-7;          /* Sect. 3.5: default tolerance */
  o->symm = -1;           /* Sect. 3.5: detect symmetry when A is explicit */
  o->m_init = 10;         /* Algorithm 3: initial guess m = 10 */
  o->m_max = 100;         /* Reading: the paper never fixes the maximum */
  o->reorth = 1;
  o->adapt_m = 1;
  o->corrector = 1;
  o->tau_fixed = 0.0;
  o->max_attempts = 1000000;
}

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int k) {
#ifdef _OPENMP
  if (k >= 1) omp_set_num_threads(k);
#else
  (void)k;
#endif
}

/* ------------------------------------------------------- scalar phi_k(z) */

/* Eq. phifunctions.  Small |z|: the power series phi_k(z) = sum_i z^i/(i+k)!
 * that follows from the integral.  Otherwise the recurrence eq. phirelation
 * run upward from phi_0 = e^z: phi_{l+1} = (phi_l - 1/l!) / z. */
double oracle_phi(int k, double z) {
  if (fabs(z) < 1.0) {
    double term = 1.0, sum = 0.0;
    for (int i = 1; i <= k; ++i) term /= (double)i;       /* 1/k! */
    for (int i = 0; i < 80; ++i) {
      sum += term;
      term *= z / (double)(i + k + 1);
      if (fabs(term) < 1e-20 * fabs(sum)) break;
    }
    return sum;
  }
  double ph = exp(z), fact = 1.0;                           /* fact = l! */
  for (int l = 0; l < k; ++l) {
    ph = (ph - 1.0 / fact) / z;
    fact *= (double)(l + 1);
  }
  return ph;
}

/* ------------------------------------------------------ vector primitives */

void oracle_spmv(int n, const int32_t* rp, const int32_t* ci, const double* val,
                 const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) acc += val[k] * x[ci[k]];
    y[i] = acc;
  }
}

/* Inner product summed over a fixed split of the rows into DOT_BLOCKS
 * contiguous blocks, each summed in row order, then the block sums in block
 * order: the result does not depend on the number of threads or on the order
 * in which they finish. */
enum { DOT_BLOCKS = 256 };
static double dot(int n, const double* x, const double* y) {
  double part[DOT_BLOCKS];
#pragma omp parallel for schedule(static)
  for (int k = 0; k < DOT_BLOCKS; ++k) {
    const long lo = (long)n * k / DOT_BLOCKS, hi = (long)n * (k + 1) / DOT_BLOCKS;
    double s = 0.0;
    for (long i = lo; i < hi; ++i) s += x[i] * y[i];
    part[k] = s;
  }
  double s = 0.0;
  for (int k = 0; k < DOT_BLOCKS; ++k) s += part[k];
  return s;
}

static double norm2(int n, const double* x) { return sqrt(dot(n, x, x)); }

static double norm_inf(int n, const double* x) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s = fmax(s, fabs(x[i]));
  return s;
}

static void axpy(int n, double a, const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) y[i] += a * x[i];
}

int oracle_is_symmetric(int n, const int32_t* rp, const int32_t* ci, const double* val) {
  for (int i = 0; i < n; ++i) {
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      int j = ci[k];
      int found = 0;
      for (int32_t q = rp[j]; q < rp[j + 1]; ++q) {
        if (ci[q] == i) { found = (val[q] == val[k]); break; }
      }
      if (!found) return 0;
    }
  }
  return 1;
}

/* --------------------------------------------- dense exponential (Pade-13) */

static void matmul(int N, const double* A, const double* B, double* C) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int k = 0; k < N; ++k) s += A[i * N + k] * B[k * N + j];
      C[i * N + j] = s;
    }
}

static double norm1_dense(int N, const double* A) {
  double best = 0.0;
  for (int j = 0; j < N; ++j) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += fabs(A[i * N + j]);
    best = fmax(best, s);
  }
  return best;
}

/* Solve M X = R (both N x N) by LU with partial pivoting; X overwrites R. */
static void lu_solve(int N, double* M, double* R) {
  for (int k = 0; k < N; ++k) {
    int piv = k;
    for (int i = k + 1; i < N; ++i)
      if (fabs(M[i * N + k]) > fabs(M[piv * N + k])) piv = i;
    if (piv != k) {
      for (int j = 0; j < N; ++j) {
        double t = M[k * N + j]; M[k * N + j] = M[piv * N + j]; M[piv * N + j] = t;
        t = R[k * N + j]; R[k * N + j] = R[piv * N + j]; R[piv * N + j] = t;
      }
    }
    for (int i = k + 1; i < N; ++i) {
      double l = M[i * N + k] / M[k * N + k];
      M[i * N + k] = l;
      for (int j = k + 1; j < N; ++j) M[i * N + j] -= l * M[k * N + j];
      for (int j = 0; j < N; ++j) R[i * N + j] -= l * R[k * N + j];
    }
  }
  for (int k = N - 1; k >= 0; --k) {
    for (int j = 0; j < N; ++j) {
      double s = R[k * N + j];
      for (int i = k + 1; i < N; ++i) s -= M[k * N + i] * R[i * N + j];
      R[k * N + j] = s / M[k * N + k];
    }
  }
}

/* Higham's scaling-and-squaring with the degree-13 diagonal Pade approximant,
 * as the paper prescribes for exp of the augmented matrix.  Reading: degree
 * 13 is always used (the paper's cost model eq. 8 assumes it) and the scaling
 * threshold is the paper's 5.37.  Pade coefficients from their closed form
 * c_j = (26-j)! 13! / (26! j! (13-j)!). */
int oracle_expm(int N, const double* A, double* E) {
  if (N <= 0) return 0;
  const size_t sz = (size_t)N * N;
  double* X = (double*)malloc(sz * sizeof(double));
  double* X2 = (double*)malloc(sz * sizeof(double));
  double* X4 = (double*)malloc(sz * sizeof(double));
  double* X6 = (double*)malloc(sz * sizeof(double));
  double* T = (double*)malloc(sz * sizeof(double));
  double* U = (double*)malloc(sz * sizeof(double));
  double* V = (double*)malloc(sz * sizeof(double));

  double c[14];
  c[0] = 1.0;
  for (int j = 0; j < 13; ++j) c[j + 1] = c[j] * (double)(13 - j) / ((double)(j + 1) * (double)(26 - j));

  double nrm = norm1_dense(N, A);
  int s = 0;
  if (nrm > 5.37) s = (int)ceil(log2(nrm / 5.37));
  if (s < 0) s = 0;
  double scale = ldexp(1.0, -s);
  for (size_t i = 0; i < sz; ++i) X[i] = A[i] * scale;

  matmul(N, X, X, X2);
  matmul(N, X2, X2, X4);
  matmul(N, X4, X2, X6);

  /* U = X [ X6 (c13 X6 + c11 X4 + c9 X2) + c7 X6 + c5 X4 + c3 X2 + c1 I ] */
  for (size_t i = 0; i < sz; ++i) T[i] = c[13] * X6[i] + c[11] * X4[i] + c[9] * X2[i];
  matmul(N, X6, T, U);
  for (size_t i = 0; i < sz; ++i) U[i] += c[7] * X6[i] + c[5] * X4[i] + c[3] * X2[i];
  for (int i = 0; i < N; ++i) U[i * N + i] += c[1];
  matmul(N, X, U, T);
  memcpy(U, T, sz * sizeof(double));

  /* V = X6 (c12 X6 + c10 X4 + c8 X2) + c6 X6 + c4 X4 + c2 X2 + c0 I */
  for (size_t i = 0; i < sz; ++i) T[i] = c[12] * X6[i] + c[10] * X4[i] + c[8] * X2[i];
  matmul(N, X6, T, V);
  for (size_t i = 0; i < sz; ++i) V[i] += c[6] * X6[i] + c[4] * X4[i] + c[2] * X2[i];
  for (int i = 0; i < N; ++i) V[i * N + i] += c[0];

  /* (V - U) R = (V + U) */
  for (size_t i = 0; i < sz; ++i) { T[i] = V[i] - U[i]; E[i] = V[i] + U[i]; }
  lu_solve(N, T, E);

  for (int k = 0; k < s; ++k) {
    matmul(N, E, E, T);
    memcpy(E, T, sz * sizeof(double));
  }
  free(X); free(X2); free(X4); free(X6); free(T); free(U); free(V);
  return s;
}

/* --------------------------------------------------------- Krylov bases */

/* One step j (0-based) of the chosen flavour: given v_0..v_j in V (columns of
 * length n), fills column j of H (row-major, ldh columns) and v_{j+1}.
 * Returns h_{j+1,j}.  w is scratch of length n. */
static double krylov_step(int n, const int32_t* rp, const int32_t* ci, const double* val,
                          double* V, double* H, int ldh, int j, int lanczos, int reorth,
                          double* w) {
  const double* vj = V + (size_t)j * n;
  oracle_spmv(n, rp, ci, val, vj, w);
  if (!lanczos && !reorth) {
    /* Algorithm 1 as printed: modified Gram-Schmidt */
    for (int i = 0; i <= j; ++i) {
      double h = dot(n, V + (size_t)i * n, w);
      H[i * ldh + j] = h;
      axpy(n, -h, V + (size_t)i * n, w);
    }
  } else if (lanczos && !reorth) {
    /* Algorithm 2.  Reading: the standard three-term recurrence; the printed
     * indices of the off-diagonal entries are garbled. */
    double a = dot(n, vj, w);
    H[j * ldh + j] = a;
    if (j > 0) {
      double bprev = H[j * ldh + (j - 1)];
      H[(j - 1) * ldh + j] = bprev;
      axpy(n, -bprev, V + (size_t)(j - 1) * n, w);
    }
    axpy(n, -a, vj, w);
  } else {
    /* CGS2: classical Gram-Schmidt twice.  Lanczos restricts the projection
     * to the two most recent basis vectors (reorth = 1) or projects against
     * all of them like Arnoldi (reorth = 2, full reorthogonalisation). */
    int i0 = (lanczos && reorth == 1) ? (j > 0 ? j - 1 : 0) : 0;
    double c[1024];
    for (int i = i0; i <= j; ++i) H[i * ldh + j] = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = i0; i <= j; ++i) c[i - i0] = dot(n, V + (size_t)i * n, w);
      for (int i = i0; i <= j; ++i) {
        axpy(n, -c[i - i0], V + (size_t)i * n, w);
        H[i * ldh + j] += c[i - i0];
      }
    }
  }
  double h = norm2(n, w);
  H[(j + 1) * ldh + j] = h;
  double* vn = V + (size_t)(j + 1) * n;
  if (h > 0.0)
    for (int i = 0; i < n; ++i) vn[i] = w[i] / h;
  else
    for (int i = 0; i < n; ++i) vn[i] = 0.0;
  return h;
}

int oracle_krylov(int n, const int32_t* rp, const int32_t* ci, const double* val,
                  const double* v, int m, int lanczos, int reorth,
                  double* V, double* H, double* beta_out) {
  double beta = norm2(n, v);
  *beta_out = beta;
  memset(H, 0, sizeof(double) * (size_t)(m + 1) * m);
  for (int i = 0; i < n; ++i) V[i] = v[i] / beta;
  double* w = (double*)malloc(sizeof(double) * n);
  int j = 0;
  for (; j < m; ++j) {
    double h = krylov_step(n, rp, ci, val, V, H, m, j, lanczos, reorth, w);
    if (h == 0.0) { ++j; break; }
  }
  free(w);
  return j;
}

/* ----------------------------------------------------- controller pieces */

/* Eq. tau_0: the Expokit initial step, enlarged by a factor 10. */
double oracle_tau0(double tol, double anorm, double bnorm, double m_ave) {
  const double mp1 = m_ave + 1.0;
  double inner = tol * pow(mp1 / exp(1.0), mp1) * sqrt(2.0 * M_PI * mp1) / (4.0 * anorm * bnorm);
  return 10.0 / anorm * pow(inner, 1.0 / m_ave);
}

/* Eq. 8: M(A) = 44/3 + 2 ceil_+(log2(||A||_1 / 5.37)).  Reading: ceil_+ is
 * max(0, ceil(.)), the number of squarings of the Pade method. */
double oracle_cost_M(double norm1) {
  double s = 0.0;
  if (norm1 > 5.37) s = ceil(log2(norm1 / 5.37));
  if (s < 0.0) s = 0.0;
  return 44.0 / 3.0 + 2.0 * s;
}

/* Eq. 4: cost of one step with Krylov dimension m. */
double oracle_cost_C1(int lanczos, double m, int p, double nnz, double n, double M) {
  double mp = m + (double)p;
  double e = M * pow(mp + 1.0, 3.0);
  if (lanczos) return mp * nnz + 3.0 * mp * n + e;
  return mp * nnz + (m * m + 3.0 * p + 2.0) * n + e;
}

/* Eq. 5: C(tau, m) = ceil((t_end - t_k)/tau) C_1(m).  Reading: at least one
 * step is always needed, so the count is at least 1. */
double oracle_cost_C(double remaining, double tau, double C1) {
  double k = ceil(remaining / tau);
  if (!(k >= 1.0)) k = 1.0;
  return k * C1;
}

/* Algorithm 4.  Readings: "previous step" is the previous attempt within the
 * same time step; eq. 6 is used with its ratio the right way up
 * (q = log(eps/eps_old)/log(tau/tau_old) - 1, matching error ~ tau^(q+1));
 * "m was reduced" is read as "m was changed" (after a rejection m can only
 * grow).  Non-finite or non-positive estimates fall back to the defaults. */
void oracle_alg4(oracle_alg4_state* s, double tau, int m, double eps, double omega,
                 double* tau_new, double* m_new, double* q_used, double* k_used) {
  const double gamma = 0.8;
  double q;
  if (s->prev_rejected && s->prev_branch == 1) {
    q = log(eps / s->eps_old) / log(tau / s->tau_old) - 1.0;
    if (isfinite(q) && q > 0.0) s->q_valid = 1; else { q = 0.25 * m; s->q_valid = 0; }
    s->q_hat = q;
  } else if (s->prev_rejected && s->q_valid) {
    q = s->q_hat;
  } else {
    q = 0.25 * m;
    s->q_valid = 0;
    s->q_hat = q;
  }
  *tau_new = tau * pow(gamma / omega, 1.0 / (q + 1.0));

  double kap;
  if (s->prev_rejected && s->prev_branch == 2) {
    kap = pow(eps / s->eps_old, 1.0 / (double)(s->m_old - m));
    if (isfinite(kap) && kap > 1.0) s->k_valid = 1; else { kap = 2.0; s->k_valid = 0; }
    s->k_hat = kap;
  } else if (s->prev_rejected && s->k_valid) {
    kap = s->k_hat;
  } else {
    kap = 2.0;
    s->k_valid = 0;
    s->k_hat = kap;
  }
  /* Eq. 3, rounded up to the smallest integer dimension that meets it. */
  *m_new = ceil((double)m + log(omega / gamma) / log(kap));
  if (q_used) *q_used = q;
  if (k_used) *k_used = kap;
}

/* ------------------------------------------------------------ the solver */

static double fact(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= (double)i;
  return f;
}

typedef struct {
  int n, nnz;
  const int32_t* rp;
  const int32_t* ci;
  const double* val;
} csr_t;

/* Eq. wrecurrence: w_0 = u_k, w_j = A w_{j-1} + sum_{l=0}^{p-j} t_k^l/l! b_{j+l}. */
static void w_recurrence(const csr_t* A, int p, const double* b, double tk,
                         const double* uk, double* W) {
  const int n = A->n;
  memcpy(W, uk, sizeof(double) * n);
  for (int j = 1; j <= p; ++j) {
    double* wj = W + (size_t)j * n;
    oracle_spmv(n, A->rp, A->ci, A->val, W + (size_t)(j - 1) * n, wj);
    for (int l = 0; l <= p - j; ++l)
      axpy(n, pow(tk, l) / fact(l), b + (size_t)(j + l) * n, wj);
  }
}

/* exp of the augmented matrix tau*K, K = [[H_m, e_1, 0], [0, 0, I_p], [0, 0, 0]]
 * of size m+p+1 (eq. hathm with one extra row/column so that phi_{p+1} needed
 * by the corrector eq. phipapprox2 appears too).  Column m+k-1 (0-based) of
 * exp(tau K) holds tau^k phi_k(tau H_m) e_1 in its top m rows; column 0
 * holds exp(tau H_m) e_1.  Outputs y = tau^p phi_p(tau H) e_1 (m entries) and
 * c = [tau^{p+1} phi_{p+1}(tau H)]_{m,1}.  Returns norm_1(tau K). */
static double augmented_expm(const double* H, int ldh, int m, int p, double tau,
                             double* y, double* c) {
  const int N = m + p + 1;
  double* K = (double*)calloc((size_t)N * N, sizeof(double));
  double* E = (double*)malloc(sizeof(double) * (size_t)N * N);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) K[i * N + j] = tau * H[i * ldh + j];
  K[0 * N + m] = tau;
  for (int i = 0; i < p; ++i) K[(m + i) * N + (m + i + 1)] = tau;
  double nrm = norm1_dense(N, K);
  oracle_expm(N, K, E);
  int col = (p == 0) ? 0 : (m + p - 1);
  for (int i = 0; i < m; ++i) y[i] = E[i * N + col];
  *c = E[(m - 1) * N + (m + p)];
  free(K);
  free(E);
  return nrm;
}

int oracle_step(int n, const int32_t* rp, const int32_t* ci, const double* val,
                int p, const double* b, double t_k, const double* u_k,
                double tau, int m, int lanczos, int reorth, int corrector,
                double* u_next, double* eps) {
  csr_t A = {n, rp[n], rp, ci, val};
  double* W = (double*)malloc(sizeof(double) * (size_t)n * (p + 1));
  w_recurrence(&A, p, b, t_k, u_k, W);
  const double* wp = W + (size_t)p * n;
  double beta = norm2(n, wp);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < p; ++j) s += pow(tau, j) / fact(j) * W[(size_t)j * n + i];
    u_next[i] = s;
  }
  *eps = 0.0;
  if (beta > 0.0) {
    double* V = (double*)malloc(sizeof(double) * (size_t)n * (m + 1));
    double* H = (double*)malloc(sizeof(double) * (size_t)(m + 1) * m);
    double bdummy;
    int mm = oracle_krylov(n, rp, ci, val, wp, m, lanczos, reorth, V, H, &bdummy);
    double hnext = H[mm * m + (mm - 1)];
    double* y = (double*)malloc(sizeof(double) * mm);
    double c;
    /* H_mm sits in the leading block of the (m+1) x m array */
    augmented_expm(H, m, mm, p, tau, y, &c);
    for (int k = 0; k < mm; ++k) axpy(n, beta * y[k], V + (size_t)k * n, u_next);
    if (corrector) axpy(n, beta * hnext * c, V + (size_t)mm * n, u_next);
    *eps = beta * fabs(hnext) * fabs(c);
    free(y); free(V); free(H);
  }
  free(W);
  return 0;
}

static double csr_norm_inf(const csr_t* A) {
  double best = 0.0;
  for (int i = 0; i < A->n; ++i) {
    double s = 0.0;
    for (int32_t k = A->rp[i]; k < A->rp[i + 1]; ++k) s += fabs(A->val[k]);
    best = fmax(best, s);
  }
  return best;
}

/* One decision of Algorithm 3 after an attempt: accept or reject (omega <=
 * delta = 1.2), then which of tau and m to change for the next attempt (or the
 * next step, on acceptance).  Algorithm 4 supplies the proposals tau_new
 * (eq. 2) and m_new (eq. 3); the cheaper of C(tau_new, m) and C(tau, m_new)
 * (eq. 4, eq. 5, with M of eq. 8 from ||tau K||_1 of this attempt) picks the
 * branch.  Readings: ties choose the m-branch; the m-branch clamps m_new to
 * [floor(3m/4), ceil(4m/3)], to at least 1 and to m_cap; tau is clamped to
 * [tau/5, 2 tau] and to t_end - t; the tau-branch is taken when m is fixed,
 * after a happy breakdown, or when rejecting and m cannot grow; a non-finite
 * omega rejects and divides tau by 5; a fixed substep accepts everything. */
void oracle_decide(oracle_alg4_state* s, const oracle_attempt* a, oracle_decision* d) {
  const double delta = 1.2;
  const double tau = a->tau;
  memset(d, 0, sizeof(*d));
  d->tau_next = tau;
  d->m_next = a->m_req;
  d->tau_new = tau;
  d->m_new = a->m_use;
  if (a->tau_fixed) {
    d->accept = 1;
    return;
  }
  if (!isfinite(a->omega)) {
    d->accept = 0;
    d->tau_next = tau / 5.0;
    s->prev_rejected = 0;
    return;
  }
  double tau_new, m_new;
  oracle_alg4(s, tau, a->m_use, a->eps, a->omega, &tau_new, &m_new, NULL, NULL);
  d->tau_new = tau_new;
  d->m_new = m_new;
  const double M = oracle_cost_M(a->knorm);
  const double m_cost = m_new < 1.0 ? 1.0 : m_new;  /* Reading: dimension >= 1 */
  const double c_tau =
      oracle_cost_C(a->rem, tau_new, oracle_cost_C1(a->lanczos, a->m_use, a->p, a->nnz, a->n, M));
  const double c_m =
      oracle_cost_C(a->rem, tau, oracle_cost_C1(a->lanczos, m_cost, a->p, a->nnz, a->n, M));
  const int accept = a->omega <= delta;
  int m_cand = a->m_req;
  if (a->adapt_m && !a->broke) {
    double mm = m_new;
    const double lo = floor(0.75 * a->m_use);
    if (mm < lo) mm = lo;
    if (mm < 1.0) mm = 1.0;
    const double hi = ceil(4.0 * a->m_use / 3.0);
    if (mm > hi) mm = hi;
    if (mm > a->m_cap) mm = a->m_cap;
    m_cand = (int)mm;
  }
  int branch;
  if (c_tau < c_m || !a->adapt_m || a->broke || (!accept && m_cand <= a->m_use)) branch = 1;
  else branch = 2;
  if (branch == 1) {
    double tn = tau_new;
    if (tn < tau / 5.0) tn = tau / 5.0;
    if (tn > 2.0 * tau) tn = 2.0 * tau;
    if (tn > a->rem) tn = a->rem;
    d->tau_next = tn;
    d->m_next = a->m_use;
  } else {
    d->m_next = m_cand;
  }
  d->accept = accept;
  d->branch = branch;
  s->prev_branch = branch;
  s->eps_old = a->eps;
  s->tau_old = tau;
  s->m_old = a->m_use;
  s->prev_rejected = !accept;
}

/* Algorithm 3 with Algorithm 4. */
int oracle_phipm(double t_end, int n, const int32_t* rp, const int32_t* ci, const double* val_in,
                 int p, const double* b_in, const oracle_opts* o, double* u,
                 oracle_stats* st, oracle_trace_rec* trace, int trace_cap, int* trace_len) {
  oracle_stats stats;
  memset(&stats, 0, sizeof(stats));
  if (trace_len) *trace_len = 0;
  if (n <= 0 || p < 0 || !(o->tol > 0.0) || !isfinite(t_end) || o->m_init < 1 ||
      o->m_max < o->m_init || o->m_max > 1000) {
    stats.status = ORACLE_EINVAL;
    if (st) *st = stats;
    return ORACLE_EINVAL;
  }
  const int nnz = rp[n];

  /* t_end = 0: u = b_0. */
  if (t_end == 0.0) {
    memcpy(u, b_in, sizeof(double) * n);
    if (st) *st = stats;
    return ORACLE_OK;
  }

  /* Reading: a negative end time integrates the ODE with -A and b_k scaled by
   * (-1)^k over |t_end|, which gives the same linear combination. */
  const double sgn = t_end < 0.0 ? -1.0 : 1.0;
  t_end = fabs(t_end);
  double* val = (double*)malloc(sizeof(double) * (nnz > 0 ? nnz : 1));
  for (int k = 0; k < nnz; ++k) val[k] = sgn * val_in[k];
  double* b = (double*)malloc(sizeof(double) * (size_t)n * (p + 1));
  for (int k = 0; k <= p; ++k) {
    double f = (sgn < 0.0 && (k & 1)) ? -1.0 : 1.0;
    for (int i = 0; i < n; ++i) b[(size_t)k * n + i] = f * b_in[(size_t)k * n + i];
  }
  csr_t A = {n, nnz, rp, ci, val};

  const double anorm = csr_norm_inf(&A);
  double bnorm = norm_inf(n, b);
  for (int k = 1; k <= p && bnorm == 0.0; ++k) bnorm = fmax(bnorm, norm_inf(n, b + (size_t)k * n));

  int status = ORACLE_OK;
  if (anorm == 0.0 || bnorm == 0.0) {
    /* A = 0: phi_k(0) = 1/k!, so u = sum_k t^k/k! b_k (also covers b = 0). */
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = 0; k <= p; ++k) s += pow(t_end, k) / fact(k) * b[(size_t)k * n + i];
      u[i] = s;
    }
    stats.t_reached = t_end;
    goto done;
  }

  {
    int lanczos;
    if (o->symm < 0) lanczos = oracle_is_symmetric(n, rp, ci, val);
    else lanczos = o->symm ? 1 : 0;
    const int m_cap = o->m_max < n ? o->m_max : n;

    double tau;
    if (o->tau_fixed > 0.0) tau = o->tau_fixed;
    else tau = oracle_tau0(o->tol, anorm, bnorm, 0.5 * (double)(o->m_init + o->m_max));
    if (!(tau > 0.0) || !isfinite(tau)) tau = t_end;  /* Reading: degenerate tau_0 */
    if (tau > t_end) tau = t_end;
    int m = o->m_init < m_cap ? o->m_init : m_cap;

    double* W = (double*)malloc(sizeof(double) * (size_t)n * (p + 1));
    double* V = (double*)malloc(sizeof(double) * (size_t)n * (m_cap + 1));
    double* H = (double*)malloc(sizeof(double) * (size_t)(m_cap + 1) * m_cap);
    double* wtmp = (double*)malloc(sizeof(double) * n);
    double* y = (double*)malloc(sizeof(double) * (m_cap + 1));
    const double bd_tol = ldexp(anorm, -40);  /* Reading: happy-breakdown level */

    double t = 0.0;
    memcpy(u, b, sizeof(double) * n);
    int64_t attempts = 0;

    while (t < t_end) {
      if (tau > t_end - t) tau = t_end - t;
      w_recurrence(&A, p, b, t, u, W);
      stats.matvecs += p;
      const double* wp = W + (size_t)p * n;
      const double beta = norm2(n, wp);
      if (!isfinite(beta)) { status = ORACLE_ENONFINITE; break; }

      int have = 0;          /* basis vectors v_0..v_have built: H has `have` columns */
      int broke = 0;         /* happy breakdown after `have` columns */
      if (beta > 0.0)
        for (int i = 0; i < n; ++i) V[i] = wp[i] / beta;
      memset(H, 0, sizeof(double) * (size_t)(m_cap + 1) * m_cap);

      oracle_alg4_state as;
      memset(&as, 0, sizeof(as));
      for (;;) {
        if (++attempts > o->max_attempts) { status = ORACLE_EMAXSTEPS; break; }
        double eps = 0.0, hnext = 0.0, c = 0.0, knorm = 0.0;
        int m_use = m;
        if (beta > 0.0) {
          while (!broke && have < m) {
            double h = krylov_step(n, rp, ci, val, V, H, m_cap, have, lanczos, o->reorth, wtmp);
            stats.matvecs += 1;
            ++have;
            if (h <= bd_tol || have == n) broke = 1;
          }
          if (broke && have < m_use) m_use = have;
          if (broke) {
            /* Invariant subspace: the projection is exact for any tau. */
            hnext = 0.0;
            if (o->tau_fixed <= 0.0) tau = t_end - t;
          } else {
            hnext = H[m_use * m_cap + (m_use - 1)];
          }
          knorm = augmented_expm(H, m_cap, m_use, p, tau, y, &c);
          stats.expms += 1;
          eps = beta * fabs(hnext) * fabs(c);   /* eq. errest */
        }
        const double omega = t_end * eps / (tau * o->tol);   /* eq. taunew */

        oracle_attempt at;
        memset(&at, 0, sizeof(at));
        at.tau = tau; at.eps = eps; at.omega = omega; at.knorm = knorm; at.rem = t_end - t;
        at.nnz = (double)nnz; at.n = (double)n;
        /* eq. 4 prices the work done: full reorthogonalisation is Arnoldi's */
        at.m_use = m_use; at.m_req = m; at.m_cap = m_cap; at.p = p;
        at.lanczos = lanczos && o->reorth != 2;
        at.adapt_m = o->adapt_m; at.broke = broke; at.tau_fixed = o->tau_fixed > 0.0;
        oracle_decision dc;
        oracle_decide(&as, &at, &dc);
        const int accept = dc.accept;
        const double tau_next = dc.tau_next;
        const int m_next = dc.m_next;

        if (trace && trace_len && *trace_len < trace_cap) {
          oracle_trace_rec* r = &trace[(*trace_len)++];
          r->t = t; r->tau = tau; r->eps = eps; r->omega = omega; r->beta = beta;
          r->hnext = hnext; r->anorm = anorm; r->tau_next = tau_next;
          r->m = m_use; r->accepted = accept; r->step = (int)stats.steps; r->m_next = m_next;
          r->branch = dc.branch; r->have = have;
        }

        if (accept) {
          /* eq. step with the corrected approximation eq. phipapprox2 */
          for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int j = 0; j < p; ++j) s += pow(tau, j) / fact(j) * W[(size_t)j * n + i];
            u[i] = s;
          }
          if (beta > 0.0) {
            for (int k = 0; k < m_use; ++k) axpy(n, beta * y[k], V + (size_t)k * n, u);
            if (o->corrector && hnext != 0.0)
              axpy(n, beta * hnext * c, V + (size_t)m_use * n, u);
          }
          t += tau;
          if (t_end - t <= 4.0 * DBL_EPSILON * t_end) t = t_end;
          stats.steps += 1;
          stats.tau_last = tau;
          stats.m_last = m_use;
          tau = tau_next;
          m = m_next;
          break;
        }
        stats.rejected += 1;
        tau = tau_next;
        m = m_next;
      }
      if (status != ORACLE_OK) break;
    }
    stats.t_reached = sgn * t;
    free(W); free(V); free(H); free(wtmp); free(y);
  }

done:
  stats.status = status;
  if (st) *st = stats;
  free(val);
  free(b);
  return status;
}

/* ------------------------------------------------------------------------
 * Learned (tau, m) proposer: plain FP64 references of the network, its loss
 * gradient, one Adam update (Kingma & Ba) and the hindsight label of a
 * recorded step.  Parameter order: W1[64][12] b1[64] W2[64][64] b2[64]
 * W3[2][64] b3[2].
 * ---------------------------------------------------------------------- */

enum { MI = 12, MH = 64, MO = 2 };
enum { PW1 = 0, PB1 = PW1 + MH * MI, PW2 = PB1 + MH, PB2 = PW2 + MH * MH, PW3 = PB2 + MH,
       PB3 = PW3 + MO * MH, PN = PB3 + MO };

/* GELU in its tanh form (Hendrycks & Gimpel): 0.5 z (1 + tanh(c (z + a z^3))). */
double oracle_gelu(double z) {
  const double c = sqrt(2.0 / M_PI), a = 0.044715;
  return 0.5 * z * (1.0 + tanh(c * (z + a * z * z * z)));
}

double oracle_gelu_grad(double z) {
  const double c = sqrt(2.0 / M_PI), a = 0.044715;
  const double th = tanh(c * (z + a * z * z * z));
  return 0.5 * (1.0 + th) + 0.5 * z * (1.0 - th * th) * c * (1.0 + 3.0 * a * z * z);
}

int oracle_mlp_params(void) { return PN; }

/* Forward pass of one row; z1, a1, z2, a2 (64 each) may be NULL. */
static void mlp_row(const double* P, const double* x, double* y, double* z1, double* a1,
                    double* z2, double* a2) {
  double Z1[MH], A1[MH], Z2[MH], A2[MH];
  for (int j = 0; j < MH; ++j) {
    double s = P[PB1 + j];
    for (int i = 0; i < MI; ++i) s += P[PW1 + j * MI + i] * x[i];
    Z1[j] = s;
    A1[j] = oracle_gelu(s);
  }
  for (int j = 0; j < MH; ++j) {
    double s = P[PB2 + j];
    for (int k = 0; k < MH; ++k) s += P[PW2 + j * MH + k] * A1[k];
    Z2[j] = s;
    A2[j] = oracle_gelu(s);
  }
  for (int o = 0; o < MO; ++o) {
    double s = P[PB3 + o];
    for (int j = 0; j < MH; ++j) s += P[PW3 + o * MH + j] * A2[j];
    y[o] = s;
  }
  if (z1) memcpy(z1, Z1, sizeof Z1);
  if (a1) memcpy(a1, A1, sizeof A1);
  if (z2) memcpy(z2, Z2, sizeof Z2);
  if (a2) memcpy(a2, A2, sizeof A2);
}

void oracle_mlp_forward(const double* P, const double* X, int rows, double* Y) {
  for (int r = 0; r < rows; ++r) mlp_row(P, X + (size_t)r * MI, Y + (size_t)r * MO, 0, 0, 0, 0);
}

/* L = 1/(2 rows) sum_r sum_o (y_ro - t_ro)^2 and dL/dP by backpropagation
 * (chain rule layer by layer).  Returns L. */
double oracle_mlp_loss_grad(const double* P, const double* X, const double* T, int rows,
                            double* grad) {
  double L = 0.0;
  if (grad) memset(grad, 0, sizeof(double) * PN);
  for (int r = 0; r < rows; ++r) {
    double y[MO], z1[MH], a1[MH], z2[MH], a2[MH];
    const double* x = X + (size_t)r * MI;
    mlp_row(P, x, y, z1, a1, z2, a2);
    double dy[MO];
    for (int o = 0; o < MO; ++o) {
      const double e = y[o] - T[(size_t)r * MO + o];
      L += e * e;
      dy[o] = e / rows;
    }
    if (!grad) continue;
    double dz2[MH], dz1[MH];
    for (int o = 0; o < MO; ++o) {
      grad[PB3 + o] += dy[o];
      for (int j = 0; j < MH; ++j) grad[PW3 + o * MH + j] += dy[o] * a2[j];
    }
    for (int j = 0; j < MH; ++j) {
      double d = 0.0;
      for (int o = 0; o < MO; ++o) d += dy[o] * P[PW3 + o * MH + j];
      dz2[j] = d * oracle_gelu_grad(z2[j]);
    }
    for (int j = 0; j < MH; ++j) {
      grad[PB2 + j] += dz2[j];
      for (int k = 0; k < MH; ++k) grad[PW2 + j * MH + k] += dz2[j] * a1[k];
    }
    for (int k = 0; k < MH; ++k) {
      double d = 0.0;
      for (int j = 0; j < MH; ++j) d += dz2[j] * P[PW2 + j * MH + k];
      dz1[k] = d * oracle_gelu_grad(z1[k]);
    }
    for (int j = 0; j < MH; ++j) {
      grad[PB1 + j] += dz1[j];
      for (int i = 0; i < MI; ++i) grad[PW1 + j * MI + i] += dz1[j] * x[i];
    }
  }
  return L / (2.0 * rows);
}

/* One Adam update with step number t (1-based): beta1 0.9, beta2 0.999, eps 1e-8. */
void oracle_adam_step(double* P, double* m, double* v, const double* g, int n, double lr,
                      long long t) {
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  for (int i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    const double mh = m[i] / (1.0 - pow(b1, (double)t));
    const double vh = v[i] / (1.0 - pow(b2, (double)t));
    P[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* omega(tau) of eq. taunew for the first mm columns of a step's H (row-major,
 * row stride ldh), with beta = ||w_p||; *knorm = ||tau K||_1. */
double oracle_step_omega(const double* H, int ldh, int mm, int p, double beta, double tau,
                         double t_end, double tol, double* knorm) {
  double* y = (double*)malloc(sizeof(double) * (size_t)mm);
  double c;
  double nrm = augmented_expm(H, ldh, mm, p, tau, y, &c);
  free(y);
  if (knorm) *knorm = nrm;
  const double eps = beta * fabs(H[(size_t)mm * ldh + (mm - 1)]) * fabs(c);
  return t_end * eps / (tau * tol);
}

/* Time of a step of Krylov dimension mm under the device time model of the
 * library (barriers, streamed algorithmic bytes, small exponential). */
double oracle_step_time(int mm, int p, int lanczos, double n, double nnz,
                        const oracle_label_costs* c) {
  const double s = 8.0;
  const double S = (s + 4.0) * nnz + 4.0 * (n + 1.0) + 2.0 * s * n;
  double bytes = p * S;
  for (int j = 1; j <= p; ++j) bytes += s * n * (p - j + 1);
  for (int j = 0; j < mm; ++j) {
    const double K = lanczos ? fmin(j + 1.0, 2.0) : j + 1.0;
    bytes += S + (4.0 * K + 8.0) * s * n;
  }
  bytes += 2.0 * s * n + s * n * fmax(p + 1.0, 1.0) + (mm + 1.0) * s * n;
  double G = fmin(fmax(ceil(n / 1024.0), 1.0), (double)c->workgroups);
  const double bw = fmin(c->bw_bytes_per_s, G * c->wg_bytes_per_s);
  const double sync = G > 1.0 ? c->sync_s : c->sync1_s;
  const double syncs = 3.0 * mm + fmax((double)p, 1.0) + 2.0;
  return syncs * sync + bytes / bw + c->expm_s[mm + p + 1];
}

/* Hindsight label of an accepted step (reading of the training target): over
 * the candidate dimensions m' in {1, ..., 16, 20, 24, ...} up to m_have (and
 * m_have itself), take tau*(m') = sup{tau in [tau_used/4096, t_end - t] :
 * omega(tau, m') <= gamma} (bisection on log tau to full double precision;
 * the whole interval if omega <= gamma at its top, its bottom if omega >
 * gamma there; t_end - t if h_{m'+1,m'} = 0), and return the pair of least
 * cost per unit time: C1(m') / tau*(m') (eq. 4 with M from ||tau* K||_1)
 * without a time model, the modelled step time / tau*(m') with one. */
void oracle_label_step(const double* H, int ldh, int m_use, int m_have, int p, int lanczos,
                       double n, double nnz, double t, double tau, double beta, double t_end,
                       double tol, const oracle_label_costs* costs, double* tau_star,
                       int* m_star) {
  const double gamma = 0.8;
  const double rem = t_end - t;
  double best = INFINITY;
  *tau_star = tau;
  *m_star = m_use;
  for (int mm = 1; mm <= m_have;) {
    double ts, kn;
    if (H[(size_t)mm * ldh + (mm - 1)] == 0.0) {
      ts = rem;
      oracle_step_omega(H, ldh, mm, p, beta, ts, t_end, tol, &kn);
    } else {
      double a = tau / 4096.0, b = rem;
      if (a > b) a = b;
      if (oracle_step_omega(H, ldh, mm, p, beta, b, t_end, tol, &kn) <= gamma) {
        ts = b;
      } else if (oracle_step_omega(H, ldh, mm, p, beta, a, t_end, tol, &kn) > gamma) {
        ts = a;
      } else {
        for (int it = 0; it < 200 && b > a * (1.0 + 4.0 * DBL_EPSILON); ++it) {
          const double mid = sqrt(a * b);
          if (mid <= a || mid >= b) break;
          if (oracle_step_omega(H, ldh, mm, p, beta, mid, t_end, tol, &kn) <= gamma) a = mid;
          else b = mid;
        }
        ts = a;
        oracle_step_omega(H, ldh, mm, p, beta, ts, t_end, tol, &kn);
      }
    }
    const double work = costs ? oracle_step_time(mm, p, lanczos, n, nnz, costs)
                              : oracle_cost_C1(lanczos, mm, p, nnz, n, oracle_cost_M(kn));
    const double cost = work / ts;
    if (cost < best) {
      best = cost;
      *tau_star = ts;
      *m_star = mm;
    }
    int nx = mm < 16 ? mm + 1 : (mm / 4 + 1) * 4;
    if (nx > m_have && mm < m_have) nx = m_have;
    mm = nx;
  }
}
