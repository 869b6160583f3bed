/*
 * CPU oracle for the adaptive Krylov phi-function solver of Niesen & Wright,
 * "A Krylov subspace algorithm for evaluating the phi-functions appearing in
 * exponential integrators" (Algorithms 3 and 4 with eqs. tau_0 ... 8).
 *
 * TEST INFRASTRUCTURE ONLY.  This header and its C file are a plain, slow,
 * double-precision reference used by tests/, the smoke check and the CPU
 * baseline leg of the benchmark.  The GPU library never includes, links or
 * calls anything from here, and nothing here includes GPU headers.
 *
 * Parity status of each exported function (see the pins under tests/):
 *   oracle_phi           pinned: closed forms of phi_1..phi_3, phi_k(0)=1/k!,
 *                        the recurrence (eq. phirelation) and quadrature of
 *                        the integral definition (eq. phifunctions).
 *   oracle_expm          pinned: diagonal, nilpotent, rotation closed forms,
 *                        a library matrix exponential, the augmented-matrix
 *                        identity of eq. hathm.
 *   oracle_krylov        pinned: orthonormality, the Arnoldi relation,
 *                        tridiagonal H for symmetric A, MGS vs CGS2 agreement.
 *   oracle_phipm         pinned: brute-force exponential of the augmented
 *                        block matrix (Lemma 2.1 / eq. phide), diagonal A,
 *                        A = 0, eigenvector decay, stepping and resume
 *                        identities (eq. steppre), linearity, forward-back.
 *   oracle_gelu, oracle_mlp_*, oracle_adam_step, oracle_label_step
 *                        pinned: GELU closed forms, finite differences,
 *                        Adam's first step, brute-force omega scans.
 *   oracle_tau0, oracle_cost_*, oracle_alg4
 *                        pinned by properties (fixed points at omega=gamma,
 *                        recovery of a known order / decay rate).
 *   oracle_decide        pinned: hand-computed cases of acceptance at
 *                        delta = 1.2, each clamp and both branches, and
 *                        properties of every attempt of traced solves.  The
 *                        step-by-step trajectory of the controller has no
 *                        printed worked example: parity unpinned.
 */
#ifndef PHIPM_ORACLE_H
#define PHIPM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Krylov flavours.  Arnoldi: 0 = modified Gram-Schmidt exactly as Algorithm 1,
 * 1 or 2 = classical Gram-Schmidt applied twice (CGS2).  Lanczos: 0 = three-term
 * recurrence of Algorithm 2 (indices read as the standard recurrence), 1 = CGS2
 * against the two previous basis vectors only, 2 = CGS2 against all previous
 * basis vectors (full reorthogonalisation; the step is then priced by eq. 4 as
 * Arnoldi's). */
typedef struct {
  double  tol;        /* absolute tolerance Tol of eq. taunew (default 1e-7) */
  int32_t symm;       /* -1 detect exactly, 0 Arnoldi, 1 Lanczos */
  int32_t m_init;     /* initial Krylov dimension (Algorithm 3: 10) */
  int32_t m_max;      /* largest Krylov dimension (default 100) */
  int32_t reorth;     /* 1 = CGS2 flavour (default), 0 = as printed, 2 = full CGS2 */
  int32_t adapt_m;    /* 1 = adapt m (phipm), 0 = keep m fixed (phip) */
  int32_t corrector;  /* 1 = use eq. phipapprox2 (default), 0 = eq. phipapprox */
  int32_t pad_;
  double  tau_fixed;  /* > 0: fixed substep, every attempt accepted */
  int64_t max_attempts;
} oracle_opts;

typedef struct {
  int64_t steps, rejected, matvecs, expms;  /* the four counters of stats */
  double  t_reached, tau_last;
  int32_t m_last, status;
} oracle_stats;

/* One record per attempt (accepted or rejected). */
typedef struct {
  double  t, tau, eps, omega, beta, hnext, anorm, tau_next;
  int32_t m, accepted, step, m_next;
  int32_t branch;     /* 1 = tau changed, 2 = m changed, 0 = no decision */
  int32_t have;       /* basis vectors built in this step so far */
} oracle_trace_rec;

enum { ORACLE_OK = 0, ORACLE_EINVAL = -1, ORACLE_EMAXSTEPS = -5, ORACLE_ENONFINITE = -4 };

void   oracle_default_opts(oracle_opts* o);

/* threads the OpenMP loops use; set_threads changes it (k >= 1) */
int    oracle_threads(void);
void   oracle_set_threads(int k);

/* scalar phi_k(z), k >= 0 */
double oracle_phi(int k, double z);

/* E = exp(A) for a dense row-major N x N matrix: degree-13 diagonal Pade with
 * scaling and squaring.  Returns the number of squarings s. */
int    oracle_expm(int N, const double* A, double* E);

/* y = A x for CSR A */
void   oracle_spmv(int n, const int32_t* rp, const int32_t* ci, const double* val,
                   const double* x, double* y);

/* 1 if the CSR matrix equals its transpose entry by entry (bitwise values). */
int    oracle_is_symmetric(int n, const int32_t* rp, const int32_t* ci, const double* val);

/* Build an m-step Krylov basis of v.  V: n x (m+1) column-major, H: (m+1) x m
 * row-major.  lanczos/reorth select the flavour.  Returns the number of
 * columns of H actually produced (< m on breakdown). */
int    oracle_krylov(int n, const int32_t* rp, const int32_t* ci, const double* val,
                     const double* v, int m, int lanczos, int reorth,
                     double* V, double* H, double* beta_out);

/* Controller pieces. */
double oracle_tau0(double tol, double anorm, double bnorm, double m_ave);
double oracle_cost_M(double norm1);
double oracle_cost_C1(int lanczos, double m, int p, double nnz, double n, double M);
double oracle_cost_C(double remaining, double tau, double C1);

typedef struct {
  int32_t prev_rejected, prev_branch;   /* branch: 1 = tau changed, 2 = m changed */
  int32_t q_valid, k_valid;
  double  q_hat, k_hat, eps_old, tau_old;
  int32_t m_old, pad_;
} oracle_alg4_state;

/* Algorithm 4: given the current attempt (tau, m, eps, omega) returns the
 * proposals tau_new and m_new (eq. 2, eq. 3; m_new rounded up). */
void   oracle_alg4(oracle_alg4_state* s, double tau, int m, double eps, double omega,
                   double* tau_new, double* m_new, double* q_used, double* k_used);

/* One attempt as Algorithm 3 sees it when it decides. */
typedef struct {
  double  tau, eps, omega;  /* substep, estimate eq. errest, ratio eq. taunew */
  double  knorm;            /* ||tau K||_1 of the attempt (M of eq. 8) */
  double  rem;              /* t_end - t_k */
  double  nnz, n;           /* N_A and n of eq. 4 */
  int32_t m_use;            /* dimension the attempt used */
  int32_t m_req;            /* dimension that was requested (> m_use after breakdown) */
  int32_t m_cap, lanczos, p, adapt_m, broke, tau_fixed;
} oracle_attempt;

typedef struct {
  double  tau_next, tau_new, m_new;  /* clamped tau, and the raw Algorithm 4 proposals */
  int32_t accept, branch, m_next, pad_;
} oracle_decision;

/* Algorithm 3's decision after one attempt: acceptance (omega <= 1.2), the
 * branch (1 = tau, 2 = m) by the cost comparison of eqs. 4-5, and the clamped
 * tau / m of the next attempt.  Updates the Algorithm 4 memory in s. */
void   oracle_decide(oracle_alg4_state* s, const oracle_attempt* a, oracle_decision* d);

/* Full solver: u = phi_0(tA)b_0 + t phi_1(tA)b_1 + ... + t^p phi_p(tA) b_p.
 * b is n x (p+1) column-major.  trace may be NULL. */
int    oracle_phipm(double t, int n, const int32_t* rp, const int32_t* ci, const double* val,
                    int p, const double* b, const oracle_opts* o, double* u,
                    oracle_stats* st, oracle_trace_rec* trace, int trace_cap, int* trace_len);

/* One step of eq. step with a fixed (tau, m) from state (t_k, u_k).  Returns
 * the error estimate in *eps. */
int    oracle_step(int n, const int32_t* rp, const int32_t* ci, const double* val,
                   int p, const double* b, double t_k, const double* u_k,
                   double tau, int m, int lanczos, int reorth, int corrector,
                   double* u_next, double* eps);

/* Learned (tau, m) proposer references (FP64).  Parameters: 5122 doubles,
 * W1[64][12] b1[64] W2[64][64] b2[64] W3[2][64] b3[2]; X rows x 12, T/Y
 * rows x 2, row-major.  Pinned: GELU closed forms and limits, the gradient
 * against central finite differences of the loss, Adam's first-step closed
 * form, the label against a brute-force scan of omega. */
double oracle_gelu(double z);
double oracle_gelu_grad(double z);
int    oracle_mlp_params(void);
void   oracle_mlp_forward(const double* P, const double* X, int rows, double* Y);
double oracle_mlp_loss_grad(const double* P, const double* X, const double* T, int rows,
                            double* grad);
void   oracle_adam_step(double* P, double* m, double* v, const double* g, int n, double lr,
                        long long t);
double oracle_step_omega(const double* H, int ldh, int mm, int p, double beta, double tau,
                         double t_end, double tol, double* knorm);
typedef struct {
  double  sync_s, sync1_s, bw_bytes_per_s, wg_bytes_per_s;
  int32_t workgroups, pad_;
  double  expm_s[128 + 8 + 2];
} oracle_label_costs;
double oracle_step_time(int mm, int p, int lanczos, double n, double nnz,
                        const oracle_label_costs* c);
void   oracle_label_step(const double* H, int ldh, int m_use, int m_have, int p, int lanczos,
                         double n, double nnz, double t, double tau, double beta, double t_end,
                         double tol, const oracle_label_costs* costs, double* tau_star,
                         int* m_star);

#ifdef __cplusplus
}
#endif
#endif
