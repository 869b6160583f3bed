/*
 * phipm for MI355X (gfx950): adaptive Krylov evaluation of
 *
 *     u(t) = phi_0(tA) b_0 + t phi_1(tA) b_1 + ... + t^p phi_p(tA) b_p
 *
 * for a large sparse matrix A in CSR form (Niesen & Wright, eq. lincomb2 /
 * eq. phide), by time stepping (eq. step, eq. wrecurrence), Arnoldi or Lanczos
 * projection with classical Gram-Schmidt applied twice, the exponential of the
 * augmented Hessenberg matrix (eq. hathm, by scaling and squaring; the paper's
 * degree-13 Pade approximant is replaced by a degree-18 Taylor polynomial of
 * the same double-precision backward error), the corrector eq. phipapprox2
 * and the error estimate eq. errest that adapts the substep tau and the Krylov
 * dimension m (Algorithms 3 and 4).
 *
 * Plain C ABI.  All array arguments marked "device" are HIP device pointers;
 * the caller owns every buffer (matrix, vectors, workspace).  The library
 * never allocates on the solve path.  Work is enqueued on `stream`; results
 * are valid after the stream has been synchronised.  Calls that share a
 * workspace must not overlap.
 *
 * Status codes: 0 = success, negative = error (see PHIPM_E*).  When a `stats`
 * pointer is passed the call synchronises the stream and the return value
 * also reflects errors found on the device (invalid CSR structure, non-finite
 * data, attempt limit).  Without it, device-side errors are reported only by
 * phipm_last_status().
 */
#ifndef PHIPM_H
#define PHIPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* phipm_stream_t; /* a hipStream_t; NULL = default stream */

enum {
  PHIPM_OK = 0,
  PHIPM_EINVAL = -1,     /* bad argument or malformed CSR */
  PHIPM_ENOMEM = -2,     /* workspace smaller than phipm_workspace_bytes() */
  PHIPM_EHIP = -3,       /* a HIP runtime call failed */
  PHIPM_ENONFINITE = -4, /* NaN/Inf in A, b or t */
  PHIPM_EMAXSTEPS = -5,  /* attempt limit reached before t_end */
  PHIPM_EUNSUPPORTED = -6,
  PHIPM_EABORT = -7,     /* a device-side wait exceeded its time budget; results invalid */
  PHIPM_ESCRATCH = -8    /* phipm_noalloc: the problem needs more than its fixed scratch */
};

enum { PHIPM_F64 = 0, PHIPM_F32 = 1 };
enum { PHIPM_FP64 = 0, PHIPM_FP32_BASIS = 1 };

/* Square n x n CSR matrix, 0-based, columns strictly increasing within each
 * row.  All three arrays are device pointers owned by the caller; val holds
 * float64 (val_dtype = PHIPM_F64) or float32 (PHIPM_F32) entries, and the
 * matrix is exactly those values: the solver reads them in that type and
 * accumulates every product in float64.  Read-only for the library. */
typedef struct {
  int32_t n;
  int32_t nnz;
  const int32_t* row_ptr; /* device, n+1 entries, row_ptr[0] = 0, row_ptr[n] = nnz */
  const int32_t* col_idx; /* device, nnz entries */
  const void* val;        /* device, nnz entries of type val_dtype */
  int32_t val_dtype;      /* PHIPM_F64 (0) or PHIPM_F32 (1) */
  int32_t pad_;
} phipm_csr;

/* Options.  Defaults from phipm_default_opts(). */
typedef struct {
  double tol;            /* absolute tolerance Tol of eq. taunew; default 1e-7 (Sect. 3.5) */
  int32_t symm;          /* -1: detect exact symmetry (Sect. 3.5), 0: Arnoldi, 1: Lanczos */
  int32_t m_init;        /* initial Krylov dimension; default 10 (Algorithm 3) */
  int32_t m_max;         /* largest Krylov dimension; default 100, at most PHIPM_M_CAP */
  int32_t precision;     /* PHIPM_FP64, or PHIPM_FP32_BASIS: Krylov basis stored in FP32
                            (products and sums accumulated in FP64; the CSR values in
                            their own type; W, u, the small exponential and the control
                            in FP64).  Each step picks its basis type: FP32 while the
                            summed FP32 rounding estimates eps32 ||beta y|| of the
                            steps fit tol max(1, ||u||), FP64 for a step that would not
                            fit (see phipm_stats.fp64_steps and fp32_flags) */
  int32_t adapt_m;       /* 1: adapt m (phipm); 0: keep m fixed (the phip variant) */
  int32_t corrector;     /* 1: eq. phipapprox2 (default); 0: eq. phipapprox */
  double tau_fixed;      /* > 0: fixed substep, every attempt accepted (diagnostics) */
  int64_t max_attempts;  /* limit on attempts (accepted + rejected); default 1e6 */
  int32_t workgroups;    /* 0: library choice (1 up to 2048 rows, else one per 320 rows,
                            at most one per CU); else workgroups cooperating on the solve */
  int32_t validate;      /* 1 (default): check CSR structure and finiteness on the device */
  const float* proposer; /* device, PHIPM_MLP_PARAMS floats: learned (tau, m) proposer that
                            seeds every step (see phipm_mlp_*); NULL (default): plain
                            step control.  The error estimate still accepts or rejects
                            every attempt and Algorithm 4 handles rejections. */
  double* history;       /* device, 4 doubles {tau, m, omega, valid}, in/out, or NULL: when
                            valid, the first step starts from the stored (tau, m) instead of
                            eq. tau_0 and m_init (warm start across calls); on success the
                            call stores the proposal for the step after its last one */
  void* trace;           /* device, trace_cap phipm_trace_step records, or NULL: one record
                            per accepted step (training data of the proposer) */
  int32_t trace_cap;
  int32_t reorth;        /* Lanczos (Algorithm 2): PHIPM_REORTH_LOCAL (default) applies
                            classical Gram-Schmidt twice against the two previous basis
                            vectors; PHIPM_REORTH_FULL against all of them (the Arnoldi
                            process on a symmetric matrix; eq. 4 then prices the step as
                            Arnoldi).  No effect on Arnoldi. */
  int32_t fp32_flags;    /* FP32 basis only: PHIPM_FP32_ONLY builds every step in FP32
                            whatever its rounding estimate (diagnostics: the true error
                            of the FP32 basis).  Default 0. */
  int32_t pad_;
} phipm_opts;

enum { PHIPM_REORTH_LOCAL = 0, PHIPM_REORTH_FULL = 1 };
enum { PHIPM_FP32_ONLY = 1 };

#define PHIPM_M_CAP 128
#define PHIPM_P_MAX 8
#define PHIPM_MLP_IN 12
#define PHIPM_MLP_HIDDEN 64
#define PHIPM_MLP_OUT 2
#define PHIPM_MLP_PARAMS 5122

/* The four counters of the paper's stats output (Sect. 3.5) and extras. */
typedef struct {
  int64_t steps;     /* accepted steps */
  int64_t rejected;  /* rejected attempts */
  int64_t matvecs;   /* products with A */
  int64_t expms;     /* small matrix exponentials */
  double t_reached;  /* end time actually reached */
  double tau_last;   /* last accepted substep */
  int32_t m_last;    /* Krylov dimension of the last accepted step */
  int32_t status;    /* PHIPM_OK or an error code */
  int32_t lanczos;   /* 1 if the Lanczos (symmetric) path was used */
  int32_t workgroups;/* workgroups that cooperated on the solve */
  double anorm;      /* ||A||_inf as used by eq. tau_0 */
  int32_t setup_flags; /* bit 0: malformed CSR, bit 1: non-finite data, bit 2: A != A^T */
  int32_t pad_;
  double bytes;      /* algorithmic HBM bytes of the streaming phases: every CSR array,
                        basis column and vector counted once per pass that touches it */
  double phi_ratio_max;        /* FP32 basis: largest ||beta y||_2 / ||u_k||_2 of a step */
  int64_t precision_rejects;   /* FP32 basis: FP32 attempts accepted by the error estimate
                                  but repeated with the FP64 basis (rounding over budget) */
  double fp32_error_estimate;  /* FP32 basis: summed absolute rounding estimates
                                  eps32 ||beta y||_2 of the FP32 steps */
  int32_t fp64_steps;          /* FP32 basis: accepted steps built with the FP64 basis */
  int32_t trace_len;           /* accepted steps offered to the trace (records beyond
                                  trace_cap are dropped) */
  int64_t proposals;           /* steps seeded by the proposer */
  double bytes_ref;            /* the same work priced by the reference byte model of a
                                  plain CGS2 Krylov step: per basis vector j+1 (0-based j)
                                  the CSR product plus (4(j+1) + 8) vectors (Arnoldi) or
                                  16 vectors (Lanczos); per step p products and 3p vectors
                                  for eq. wrecurrence and (p + m + 2) vectors for eq. step */
  double krylov_bytes_ref;     /* the part of bytes_ref spent building Krylov bases (the
                                  CSR products and the orthogonalisation, Algorithms 1-2) */
  double krylov_seconds;       /* device time spent building Krylov bases, from the
                                  constant-rate wall clock of the solve's first workgroup
                                  (every workgroup of a solve builds in lock step) */
} phipm_stats;

void phipm_default_opts(phipm_opts* opts);

/* Bytes of device workspace phipm() needs for this matrix, p and options.
 * Returns PHIPM_OK or PHIPM_EINVAL. */
int phipm_workspace_bytes(const phipm_csr* A, int p, const phipm_opts* opts, size_t* bytes);

/* u = sum_{k=0}^{p} t^k phi_k(tA) b_k  (eq. lincomb2 at t = t_end).
 *   t          end time; any finite value (t < 0 integrates with -A).
 *   b          device, n x (p+1) column-major (column k = b_k, leading dim n).
 *   u          device, n entries, output; must not alias b or the workspace.
 *   workspace  device, ws_bytes >= phipm_workspace_bytes(); 256-byte aligned.
 *   stats      host, may be NULL (then the call does not synchronise).
 * 0 <= p <= PHIPM_P_MAX. */
int phipm(double t, const phipm_csr* A, int p, const double* b, const phipm_opts* opts,
          double* u, void* workspace, size_t ws_bytes, phipm_stats* stats,
          phipm_stream_t stream);

/* phipm() without a caller workspace and without any device allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  The workspace is a fixed array of
 * phipm_noalloc_scratch_bytes() (64 MiB) in the library's device code, one
 * per GPU, held until the process ends; the call allocates nothing (no
 * hipMalloc, no allocating library routine).  Arguments, results, status
 * codes and synchronisation as for phipm(), plus PHIPM_ESCRATCH (checked on
 * the host before any device work) when phipm_workspace_bytes() for this
 * problem exceeds the fixed size: roughly n (m_max + 4) 8 bytes plus 132 KB
 * per workgroup must fit, e.g. n = 65536 with the default options.  Every
 * call on a GPU uses that GPU's one array: calls that overlap on one GPU
 * (other host threads, other streams) race and must be serialised by the
 * caller; a call leaves its data in the array, and the solver writes every
 * word it reads before reading it. */
int phipm_noalloc(double t, const phipm_csr* A, int p, const double* b, const phipm_opts* opts,
                  double* u, phipm_stats* stats, phipm_stream_t stream);

/* Size of phipm_noalloc()'s fixed device scratch, in bytes. */
size_t phipm_noalloc_scratch_bytes(void);

/* Status of the last phipm() on this host thread as seen on the device
 * (synchronises the stream the call used). */
int phipm_last_status(void);

/* y = A x with the solver's CSR product: the products with A that the Krylov
 * processes of Sect. 3.1 (Algorithms 1 and 2) and eq. wrecurrence are built
 * from.  x, y: device, n float64 entries (y must not overlap x); A's values in
 * either val_dtype, accumulated in float64.  Same validity rules as phipm()
 * (an invalid CSR structure is not detected here: pass a valid matrix);
 * asynchronous.  Returns PHIPM_OK, PHIPM_EINVAL for a null pointer or a bad
 * descriptor, PHIPM_EHIP. */
int phipm_spmv(const phipm_csr* A, const double* x, double* y, phipm_stream_t stream);

/* Pointwise data of one exponential Rosenbrock-Euler step for the Allen-Cahn
 * equation u_t = L u + u - u^3, the integrator that drives the solver the
 * way Sect. 1 describes (one phi_1 evaluation per step, with the Jacobian
 * J = L + diag(1 - 3 u^2) as the operator).  In order, on `stream`:
 *   if du:    u += du                              (the previous step's increment)
 *   if F:     F = L u + (u - u^3)                  (the right-hand side, b_1)
 *   if J_val: J_val[diag_pos[i]] = lap_diag[i] + (1 - 3 u_i^2)   for i < n
 * L: CSR of the linear part (device arrays, as for phipm()); u, du, F: device,
 * n = L->n doubles (F must not alias u); diag_pos: device, n int32 positions of
 * the diagonal in J's value array J_val (J shares L's pattern); lap_diag:
 * device, the n diagonal values of L.  Any of du, F and J_val may be NULL;
 * diag_pos and lap_diag are required with J_val.  Asynchronous.  Returns
 * PHIPM_OK, PHIPM_EINVAL for a bad argument, PHIPM_EHIP. */
int phipm_allen_cahn_update(const phipm_csr* L, double* u, const double* du,
                            const int32_t* diag_pos, const double* lap_diag, double* J_val,
                            double* F, phipm_stream_t stream);

/* E = exp(H) for a dense row-major N x N float64 matrix on the device with the
 * solver's small-matrix exponential (Sect. 3.1: scaling and squaring; here with
 * a degree-18 Taylor polynomial of double-precision backward error instead of
 * the degree-13 Pade approximant, so no linear solve).
 * N <= PHIPM_M_CAP + PHIPM_P_MAX + 1.  scratch: device, >= 8*N*N doubles. */
int phipm_expm(int N, const double* H, double* E, double* scratch, phipm_stream_t stream);

/* m steps of the solver's Krylov process started from v (device, n entries):
 * the Arnoldi process of Algorithm 1 (lanczos = 0) or the Lanczos process of
 * Algorithm 2 (lanczos = 1), Sect. 3.1, each with classical Gram-Schmidt
 * applied twice (Lanczos against the two previous vectors).  Outputs, in
 * float64: V (device, n x (m+1) column-major, leading dimension n: the
 * orthonormal basis v_1..v_{m+1} with v_1 = v / ||v||) and H (device,
 * (m+1) x m row-major: the Hessenberg matrix with A V_m = V_{m+1} H).  The
 * number of steps done (< m after a happy breakdown) goes to *m_done (host).
 * A: float64 values only (PHIPM_EINVAL otherwise); 1 <= m <= PHIPM_M_CAP.
 * workspace: device, 256-byte aligned, at least phipm_workspace_bytes() for
 * p = 0 and m_max = max(m, 10).  Synchronises the stream.  Returns PHIPM_OK,
 * PHIPM_EINVAL, PHIPM_ENOMEM (workspace too small), PHIPM_EHIP. */
int phipm_krylov(const phipm_csr* A, const double* v, int m, int lanczos, double* V, double* H,
                 void* workspace, size_t ws_bytes, int* m_done, phipm_stream_t stream);

/* ------------------------------------------------------------------------
 * Many independent solves in one persistent launch.
 *
 * A plan binds `count` instances u_i = sum_k t_i^k phi_k(t_i A_i) b_{i,k},
 * each exactly the problem of phipm() with the shared options, to one
 * persistent kernel.  The grid (one workgroup per compute unit) is split into
 * teams of power-of-two sizes; instances are grouped into team-size classes
 * by cost and queued in descending cost; a team takes the next instance of
 * its class's queue, then of the smaller classes' queues, until all are
 * solved.  The team layout is chosen by an autotuner that times candidate
 * layouts on the device with the plan's own instances (costs predicted from
 * n_i, t_i, p_i and ||A_i||_inf, then measured).  The tuned launch is
 * captured in a hipGraph that phipm_plan_execute() replays.
 *
 * Ownership: the plan allocates and owns its device memory (descriptors,
 * one work buffer per team, per-instance statistics), released by
 * phipm_plan_destroy().  It stores the caller's pointers: every A_i, b_i and
 * u_i must stay allocated, with unchanged shapes, while the plan lives; the
 * contents of b_i (and of A_i's values) may change between executions.
 * Creating a plan with autotuning runs the whole batch several times (it
 * writes u_i).  Executions of one plan must not overlap.
 * ---------------------------------------------------------------------- */
typedef struct phipm_plan phipm_plan;

typedef struct {
  int32_t autotune;  /* 1 (default): time candidate layouts at creation; 0: model layout */
  int32_t graph;     /* 1 (default): capture the launch in a hipGraph */
  int32_t max_team;  /* 0: library default (16); else largest team of the untuned layout,
                        a power of two */
  int32_t pad_;
} phipm_plan_opts;

typedef struct {
  int32_t count;          /* instances */
  int32_t workgroups;     /* grid size of the persistent kernel */
  int32_t teams;          /* teams of the chosen layout */
  int32_t classes;        /* team-size classes (at most 8 reported) */
  int32_t class_size[8];  /* workgroups per team of each class, largest first */
  int32_t class_teams[8]; /* teams of each class */
  int32_t graph;          /* 1 if executions replay a captured hipGraph */
  int32_t cooperative;    /* 1 if the persistent kernel is launched cooperatively */
  int32_t candidates;     /* distinct layouts timed by the autotuner (0: not tuned) */
  int32_t max_team;       /* largest team size allowed by the chosen layout */
  double alpha;           /* cost threshold factor of the chosen layout */
  double tuned_ms;        /* time of the chosen layout while tuning */
  double default_ms;      /* time of the untuned layout while tuning */
  uint64_t device_bytes;  /* device memory held by the plan */
} phipm_plan_info;

void phipm_default_plan_opts(phipm_plan_opts* popts);

/* Create a plan for `count` >= 1 instances.  Host arrays of length count:
 *   A   CSR descriptors (device pointers inside, as for phipm())
 *   p   0 <= p_i <= PHIPM_P_MAX
 *   t   finite end times
 *   b   device pointers, n_i x (p_i+1) column-major float64
 *   u   device pointers, n_i float64 outputs; no u_i may overlap another u_j
 *       or its b_i
 * opts applies to every instance (opts->workgroups > 0 caps the grid size;
 * opts->proposer is shared by all instances; opts->history and opts->trace
 * are ignored).
 * Work during creation (norms, tuning runs) is enqueued on `stream` and
 * synchronised.  Returns PHIPM_OK and *plan, or an error (PHIPM_EINVAL,
 * PHIPM_ENONFINITE for a non-finite t_i, PHIPM_ENOMEM, PHIPM_EHIP,
 * PHIPM_EABORT). */
int phipm_plan_create(int count, const phipm_csr* A, const int32_t* p, const double* t,
                      const double* const* b, double* const* u, const phipm_opts* opts,
                      const phipm_plan_opts* popts, phipm_stream_t stream, phipm_plan** plan);

/* Solve all instances once (asynchronous on `stream`; must be called on the
 * device the plan was created on). */
int phipm_plan_execute(phipm_plan* plan, phipm_stream_t stream);

/* Per-instance statistics of the last execution (host array of count
 * entries; synchronises the stream of that execution).  Returns PHIPM_OK or
 * the first instance's error. */
int phipm_plan_stats(phipm_plan* plan, phipm_stats* stats);

int phipm_plan_get_info(const phipm_plan* plan, phipm_plan_info* info);

/* Synchronises the last execution's stream and frees the plan. */
int phipm_plan_destroy(phipm_plan* plan);

/* One-off convenience: create an untuned, uncaptured plan, execute it, fill
 * stats (host, count entries, may be NULL), destroy it.  Synchronous; it
 * allocates and frees the plan's device memory. */
int phipm_batched(int count, const phipm_csr* A, const int32_t* p, const double* t,
                  const double* const* b, double* const* u, const phipm_opts* opts,
                  phipm_stats* stats, phipm_stream_t stream);

/* Host-only, no device work: the team layout the planner derives from
 * per-instance costs (cost[i] >= 0, any unit) for a grid of `workgroups`
 * workgroups, teams of at most max_team (a power of two) and the threshold
 * factor alpha > 0.  Outputs (host arrays): team_size[t], team_class[t] for
 * t < *nteams (capacity workgroups); order (capacity count): instance ids,
 * queue after queue; qbeg (capacity workgroups + 1): queue c is
 * order[qbeg[c] .. qbeg[c+1]) for c < *nclasses.  Teams are listed in
 * grid order (team t starts at the sum of the sizes before it). */
int phipm_batch_layout(int count, const double* cost, int workgroups, int max_team,
                       double alpha, int32_t* team_size, int32_t* team_class, int32_t* nteams,
                       int32_t* order, int32_t* qbeg, int32_t* nclasses);

/* ------------------------------------------------------------------------
 * Learned (tau, m) proposer (an addition to the paper's method, which it does
 * not change: it only replaces the starting point of each step).
 *
 * Network: FP32 multilayer perceptron 12 -> 64 -> 64 -> 2, GELU (tanh form)
 * after both hidden layers.  Parameters (PHIPM_MLP_PARAMS floats, in order):
 * W1[64][12] b1[64] W2[64][64] b2[64] W3[2][64] b3[2].  Inputs (computed by
 * the solver at the start of a step; all clipped to a few decades):
 *   0 log10(||A||_inf t_end)       1 log10(tol / max_k ||b_k||_inf)   2 p / 4
 *   3 log10(||w_p||_2 / ||u_k||_2)  4 t_k / t_end
 *   5 log10(tau_prev ||A||_inf)    6 m_prev / 32   7 log10(omega_prev)
 *   8 rejections of the previous step / 4
 *   9 log10(tau_plain ||A||_inf)   10 m_plain / 32  11 1 if Lanczos
 * where "prev" is the last accepted step (or the warm-start history) and
 * "plain" the plain controller's choice for this step.  Outputs:
 * (log10(tau* ||A||_inf), m / 32) with tau* the predicted largest admissible
 * substep; the solver attempts 0.7 tau*, kept within
 * [tau_plain, 8 tau_plain] (and below t_end - t_k) and m within
 * [max(1, floor(3 m_plain / 4)), min(m_max, n)]: the proposer can make a
 * step longer than the plain controller's, never shorter, and a rejection
 * hands the step back to Algorithm 4.
 * ---------------------------------------------------------------------- */

/* One accepted step as recorded by phipm() with opts.trace set. */
typedef struct {
  float features[PHIPM_MLP_IN];  /* inputs seen at the start of the step */
  int32_t m_use;                  /* Krylov dimension of the accepted attempt */
  int32_t m_have;                 /* basis columns available (>= m_use): with a trace the
                                     solver extends the step's basis to m_cap = min(m_max,
                                     n) columns after the step (extra products, counted
                                     in the stats) */
  int32_t p, lanczos, n, nnz, attempts, pad_;
  double t, tau, omega, beta, anorm, t_end, tol, pad2_;
  double H[(PHIPM_M_CAP + 1) * PHIPM_M_CAP]; /* leading (m_have+1) x m_have block of the
                                                step's Hessenberg matrix, row-major,
                                                row stride PHIPM_M_CAP */
} phipm_trace_step;

/* Y = MLP(X) for `rows` rows (device: X rows x 12, Y rows x 2, row-major)
 * with the solver's inference routine (one wavefront per row). */
int phipm_mlp_forward(const float* params, const float* X, int rows, float* Y,
                      phipm_stream_t stream);

/* Gradient of the loss L = 1/(2 rows) sum_r sum_o (MLP(X)_ro - T_ro)^2 with
 * respect to the parameters (device: grad PHIPM_MLP_PARAMS floats, loss 1
 * float).  One workgroup, deterministic order. */
int phipm_mlp_grad(const float* params, const float* X, const float* T, int rows, float* grad,
                   float* loss, phipm_stream_t stream);

/* Train in place with Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning rate
 * lr) on minibatches of `batch` (1..64) consecutive rows, `epochs` passes in
 * row order; adam_m / adam_v (device, PHIPM_MLP_PARAMS floats) are the moment
 * estimates and step0 the number of updates already made with them.
 * loss (device, epochs floats) receives each epoch's mean loss. */
int phipm_mlp_train(float* params, float* adam_m, float* adam_v, const float* X, const float* T,
                    int rows, int batch, int epochs, float lr, int step0, float* loss,
                    phipm_stream_t stream);

/* Time model of one step on the device, used by hindsight labels in place
 * of the flop count of eq. 4: a step with Krylov dimension m costs
 *   (3m + max(p, 1) + 2) sync_s                          team barriers
 * + bytes(m) / min(bw_bytes_per_s, G wg_bytes_per_s)    streaming phases
 * + expm_s[m + p + 1]                                   small exponential
 * with G = min(workgroups, ceil(n / 1024)), sync_s replaced by sync1_s when
 * G = 1, and bytes(m) the solver's algorithmic bytes in float64 (s = 8,
 * S = (s + 4) nnz + 4 (n + 1) + 2 s n per CSR product):
 *   p S + sum_{j=1..p} s n (p - j + 1)              w-recurrence
 * + sum_{j=0..m-1} [S + (4 K_j + 8) s n]            Krylov steps, K_j = j + 1
 *                                                   (Arnoldi), min(j + 1, 2)
 *                                                   (Lanczos)
 * + 2 s n + s n max(p + 1, 1) + (m + 1) s n         corrector vector, update */
typedef struct {
  double sync_s;          /* one team barrier with G > 1 workgroups */
  double sync1_s;         /* one barrier of a single workgroup */
  double bw_bytes_per_s;  /* streaming bandwidth of the whole grid */
  double wg_bytes_per_s;  /* streaming bandwidth of one workgroup */
  int32_t workgroups;     /* grid size of the solver */
  int32_t pad_;
  double expm_s[PHIPM_M_CAP + PHIPM_P_MAX + 2]; /* time of the exponential of order N */
} phipm_label_costs;

/* Hindsight labels of recorded steps: for m' in {1..16, 20, 24, ...,
 * m_have} (and m_have) the largest tau in [tau/4096, t_end - t] with
 * omega(tau, m') <= 0.8 (bisection on log tau with the solver's small
 * exponential), and the (tau*, m') of least cost per unit time: C1(m') / tau*
 * (eq. 4, eq. 8) when costs is NULL, else the time model above divided by
 * tau*.  Device outputs: X (count x 12, the recorded features) and T
 * (count x 2: log10(tau* ||A||_inf), m'/32).  workspace: device,
 * >= phipm_label_workspace_bytes(count); costs: host, may be NULL. */
size_t phipm_label_workspace_bytes(int count);
int phipm_label_steps(const phipm_trace_step* records, int count, float* X, float* T,
                      void* workspace, size_t ws_bytes, const phipm_label_costs* costs,
                      phipm_stream_t stream);

const char* phipm_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif
