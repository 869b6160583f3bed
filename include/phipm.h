/*
 * phipm for MI355X (gfx950): adaptive Krylov evaluation of
 *
 *     u(t) = phi_0(tA) b_0 + t phi_1(tA) b_1 + ... + t^p phi_p(tA) b_p
 *
 * for a large sparse matrix A in CSR form (Niesen & Wright, eq. lincomb2 /
 * eq. phide), by time stepping (eq. step, eq. wrecurrence), Arnoldi or Lanczos
 * projection with classical Gram-Schmidt applied twice, the exponential of the
 * augmented Hessenberg matrix (eq. hathm, degree-13 Pade with scaling and
 * squaring), the corrector eq. phipapprox2 and the error estimate eq. errest
 * that adapts the substep tau and the Krylov dimension m (Algorithms 3 and 4).
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
  PHIPM_EABORT = -7      /* a device-side wait exceeded its time budget; results invalid */
};

enum { PHIPM_F64 = 0, PHIPM_F32 = 1 };
enum { PHIPM_FP64 = 0, PHIPM_FP32_BASIS = 1 };

/* Square n x n CSR matrix, 0-based, columns strictly increasing within each
 * row.  All three arrays are device pointers owned by the caller; val holds
 * float64 entries.  Read-only for the library. */
typedef struct {
  int32_t n;
  int32_t nnz;
  const int32_t* row_ptr; /* device, n+1 entries, row_ptr[0] = 0, row_ptr[n] = nnz */
  const int32_t* col_idx; /* device, nnz entries */
  const double* val;      /* device, nnz entries */
} phipm_csr;

/* Options.  Defaults from phipm_default_opts(). */
typedef struct {
  double tol;            /* absolute tolerance Tol of eq. taunew; default 1e-7 (Sect. 3.5) */
  int32_t symm;          /* -1: detect exact symmetry (Sect. 3.5), 0: Arnoldi, 1: Lanczos */
  int32_t m_init;        /* initial Krylov dimension; default 10 (Algorithm 3) */
  int32_t m_max;         /* largest Krylov dimension; default 100, at most PHIPM_M_CAP */
  int32_t precision;     /* PHIPM_FP64 or PHIPM_FP32_BASIS */
  int32_t adapt_m;       /* 1: adapt m (phipm); 0: keep m fixed (the phip variant) */
  int32_t corrector;     /* 1: eq. phipapprox2 (default); 0: eq. phipapprox */
  double tau_fixed;      /* > 0: fixed substep, every attempt accepted (diagnostics) */
  int64_t max_attempts;  /* limit on attempts (accepted + rejected); default 1e6 */
  int32_t workgroups;    /* 0: library choice; else workgroups cooperating on the solve */
  int32_t validate;      /* 1 (default): check CSR structure and finiteness on the device */
} phipm_opts;

#define PHIPM_M_CAP 128
#define PHIPM_P_MAX 8

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
  int64_t precision_rejects;   /* FP32 basis: attempts rejected for basis rounding */
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

/* Status of the last phipm() on this host thread as seen on the device
 * (synchronises the stream the call used). */
int phipm_last_status(void);

/* y = A x, the CSR product used inside the solver (device pointers, float64).
 * Same validity rules as phipm(); asynchronous. */
int phipm_spmv(const phipm_csr* A, const double* x, double* y, phipm_stream_t stream);

/* E = exp(H) for a dense row-major N x N float64 matrix on the device with the
 * solver's small-matrix exponential (degree-13 Pade, scaling and squaring).
 * N <= PHIPM_M_CAP + PHIPM_P_MAX + 1.  scratch: device, >= 8*N*N doubles. */
int phipm_expm(int N, const double* H, double* E, double* scratch, phipm_stream_t stream);

/* m steps of the solver's Krylov process started from v (device, n entries):
 * V (device, n x (m+1) column-major, leading dimension n) and H (device,
 * (m+1) x m row-major), in float64 with the Arnoldi (lanczos = 0) or Lanczos
 * (lanczos = 1) flavour.  Returns the number of steps done in *m_done (host). */
int phipm_krylov(const phipm_csr* A, const double* v, int m, int lanczos, double* V, double* H,
                 void* workspace, size_t ws_bytes, int* m_done, phipm_stream_t stream);

const char* phipm_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif
