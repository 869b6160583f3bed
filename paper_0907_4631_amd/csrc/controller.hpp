// Step-size and Krylov-dimension control of the adaptive solver (Sect. 3.3,
// 3.4; Algorithms 3 and 4), evaluated in float64 by one thread.
#pragma once
#include <hip/hip_runtime.h>

namespace pkr {

constexpr double CTRL_GAMMA = 0.8;  // safety factor of eq. 2 / eq. 3
constexpr double CTRL_DELTA = 1.2;  // acceptance threshold on omega

// Eq. tau_0: ten times the Expokit initial step for the average dimension.
__device__ inline double ctrl_tau0(double tol, double anorm, double bnorm, double m_ave) {
  const double k = m_ave + 1.0;
  const double num = tol * pow(k / 2.718281828459045, k) * sqrt(2.0 * 3.141592653589793 * k);
  return (10.0 / anorm) * pow(num / (4.0 * anorm * bnorm), 1.0 / m_ave);
}

// Eq. 8 (products and one division of the Pade method, in units of N^3).
__device__ inline double ctrl_M(double norm1) {
  double sq = 0.0;
  if (norm1 > 5.37) sq = ceil(log2(norm1 / 5.37));
  return 44.0 / 3.0 + 2.0 * (sq > 0.0 ? sq : 0.0);
}

// Eq. 4: cost of one step of dimension m (Lanczos or Arnoldi).
__device__ inline double ctrl_C1(bool lanczos, double m, int p, double nnz, double n, double M) {
  const double mp = m + p;
  const double small = M * (mp + 1.0) * (mp + 1.0) * (mp + 1.0);
  const double orth = lanczos ? 3.0 * mp * n : (m * m + 3.0 * p + 2.0) * n;
  return mp * nnz + orth + small;
}

// Eq. 5, with at least one step.
__device__ inline double ctrl_C(double remaining, double tau, double c1) {
  double steps = ceil(remaining / tau);
  if (!(steps >= 1.0)) steps = 1.0;
  return steps * c1;
}

// Memory of Algorithm 4 across the attempts of one time step.
struct Alg4Mem {
  int rejected;   // the previous attempt of this step was rejected
  int branch;     // what that attempt changed: 1 = tau, 2 = m
  int q_ok, k_ok; // eq. 6 / eq. 7 produced a usable value last time
  double q, kappa, eps, tau;
  int m;
};

// Algorithm 4.  eq. 6 is used with the ratio of logarithms the right way up
// (error ~ tau^(q+1)); "m was reduced" is taken as "m was changed".
__device__ inline void ctrl_alg4(Alg4Mem& s, double tau, int m, double eps, double omega,
                                 double* tau_new, double* m_new) {
  double q;
  if (s.rejected && s.branch == 1) {
    q = log(eps / s.eps) / log(tau / s.tau) - 1.0;
    s.q_ok = isfinite(q) && q > 0.0;
    if (!s.q_ok) q = 0.25 * m;
  } else if (s.rejected && s.q_ok) {
    q = s.q;
  } else {
    q = 0.25 * m;
    s.q_ok = 0;
  }
  s.q = q;
  *tau_new = tau * pow(CTRL_GAMMA / omega, 1.0 / (q + 1.0));

  double kap;
  if (s.rejected && s.branch == 2) {
    kap = pow(eps / s.eps, 1.0 / (double)(s.m - m));
    s.k_ok = isfinite(kap) && kap > 1.0;
    if (!s.k_ok) kap = 2.0;
  } else if (s.rejected && s.k_ok) {
    kap = s.kappa;
  } else {
    kap = 2.0;
    s.k_ok = 0;
  }
  s.kappa = kap;
  *m_new = ceil((double)m + log(omega / CTRL_GAMMA) / log(kap));
}

}  // namespace pkr
