// Host-side helpers shared by the single-solve and batched entry points:
// argument checks and the layout of a solver work buffer.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstddef>
#include <cstring>

#include "../../include/phipm.h"
#include "solver.hpp"

namespace pkr {

// device-side mirrors of the C ABI structures
static_assert(sizeof(Stats) == sizeof(phipm_stats), "Stats mirrors phipm_stats");
static_assert(sizeof(TraceStep) == sizeof(phipm_trace_step), "TraceStep mirrors phipm_trace_step");
static_assert(offsetof(TraceStep, H) == offsetof(phipm_trace_step, H), "trace layout");
static_assert(offsetof(Stats, proposals) == offsetof(phipm_stats, proposals), "stats layout");
static_assert(offsetof(Stats, bytes_ref) == offsetof(phipm_stats, bytes_ref), "stats layout");
static_assert(offsetof(Stats, krylov_ticks) == offsetof(phipm_stats, krylov_seconds),
              "stats layout");

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline long long pad64(long long x) { return (x + 63) / 64 * 64; }

// Byte offsets of one solver work buffer (everything a team needs for one
// instance except its barrier flags and reduction partials).
struct WorkLayout {
  long long ld;      // leading dimension of W and V (rows padded to 64)
  size_t W, V, y0, y1, H, ex, st, stats, total;
};

// The basis and its two work vectors are sized for float64 also with the
// FP32 basis: a step whose FP32 rounding would not fit the tolerance is
// built with the FP64 basis in the same buffer.
// hcopies: copies of H (one per workgroup of the launch; 0 when the caller
// places them elsewhere).
inline WorkLayout work_layout(int n, int p, int m_cap, int hcopies) {
  WorkLayout L{};
  const size_t tb = 8;
  L.ld = pad64(n);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  L.W = take(sizeof(double) * (size_t)L.ld * (size_t)std::max(p, 1));
  L.V = take(tb * (size_t)L.ld * (size_t)(m_cap + 1));
  L.y0 = take(tb * (size_t)L.ld);
  L.y1 = take(tb * (size_t)L.ld);
  L.H = take(sizeof(double) * H_WORDS * (size_t)hcopies);
  L.ex = take(sizeof(double) * 8 * (size_t)NMAX_EXPM * NMAX_EXPM);
  L.st = take(sizeof(State));
  L.stats = take(sizeof(Stats));
  L.total = off;
  return L;
}

template <typename T>
inline Work<T> work_at(char* base, const WorkLayout& L) {
  return Work<T>{reinterpret_cast<double*>(base + L.W), L.ld, reinterpret_cast<T*>(base + L.V),
                 L.ld, reinterpret_cast<T*>(base + L.y0), reinterpret_cast<T*>(base + L.y1),
                 reinterpret_cast<double*>(base + L.H), reinterpret_cast<double*>(base + L.ex),
                 reinterpret_cast<State*>(base + L.st), reinterpret_cast<Stats*>(base + L.stats),
                 reinterpret_cast<double*>(base + L.H)};
}

inline bool opts_ok(const phipm_opts* o) {
  return o && o->tol > 0.0 && std::isfinite(o->tol) && o->m_init >= 1 && o->m_max >= o->m_init &&
         o->m_max <= PHIPM_M_CAP && (o->symm >= -1 && o->symm <= 1) &&
         (o->precision == PHIPM_FP64 || o->precision == PHIPM_FP32_BASIS) && o->max_attempts >= 1 &&
         o->workgroups >= 0 && std::isfinite(o->tau_fixed) && o->tau_fixed >= 0.0 &&
         o->trace_cap >= 0 && (o->trace_cap == 0 || o->trace) &&
         (o->reorth == PHIPM_REORTH_LOCAL || o->reorth == PHIPM_REORTH_FULL) &&
         (o->fp32_flags & ~PHIPM_FP32_ONLY) == 0;
}

inline bool csr_ok(const phipm_csr* A) {
  return A && A->n > 0 && A->nnz >= 0 && A->row_ptr && (A->nnz == 0 || (A->col_idx && A->val)) &&
         (A->val_dtype == PHIPM_F64 || A->val_dtype == PHIPM_F32);
}

inline bool overlaps(const void* a, size_t na, const void* c, size_t nc) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(c);
  return x < y + nc && y < x + na;
}

// Seconds per tick of the device's constant-rate wall clock (wall_clock64).
inline double wall_tick_seconds(int device) {
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0)
    return 0.0;
  return 1e-3 / (double)khz;
}

// tick_s: seconds per wall-clock tick of the device the statistics come from.
inline void copy_stats(const Stats& hs, int status, double tick_s, phipm_stats* s) {
  s->steps = hs.steps;
  s->rejected = hs.rejected;
  s->matvecs = hs.matvecs;
  s->expms = hs.expms;
  s->t_reached = hs.t_reached;
  s->tau_last = hs.tau_last;
  s->m_last = hs.m_last;
  s->status = status;
  s->lanczos = hs.lanczos;
  s->workgroups = hs.workgroups;
  s->anorm = hs.anorm;
  s->setup_flags = hs.setup_flags;
  s->pad_ = 0;
  s->bytes = hs.bytes;
  s->phi_ratio_max = hs.rho_max;
  s->precision_rejects = hs.prec_rejects;
  s->fp32_error_estimate = hs.fp32_err;
  s->fp64_steps = hs.fp64_steps;
  s->trace_len = hs.trace_len;
  s->proposals = hs.proposals;
  s->bytes_ref = hs.bytes_ref;
  s->krylov_bytes_ref = hs.krylov_bytes_ref;
  s->krylov_seconds = hs.krylov_ticks * tick_s;
}

}  // namespace pkr
