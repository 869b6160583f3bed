// Learned (tau, m) proposer: a small FP32 multilayer perceptron
// 12 -> 64 -> 64 -> 2 with GELU (tanh form) hidden activations.
//
// It seeds each step of the adaptive solver (and the first step of a call)
// with a proposal of the substep and the Krylov dimension; the solver's own
// error estimate still accepts or rejects every attempt, and after a
// rejection the plain step control of Algorithm 4 takes over.  The features
// are scale-free summaries of the problem and of the step history; the
// outputs are log10(tau ||A||_inf) and m / 32.
//
// Parameter vector (float32, 5122 entries):
//   W1[64][12] b1[64] W2[64][64] b2[64] W3[2][64] b3[2]
#pragma once
#include <hip/hip_runtime.h>

#include "team.hpp"

namespace pkr {

constexpr int MLP_IN = 12;
constexpr int MLP_H = 64;
constexpr int MLP_OUT = 2;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + MLP_H * MLP_IN;
constexpr int OFF_W2 = OFF_B1 + MLP_H;
constexpr int OFF_B2 = OFF_W2 + MLP_H * MLP_H;
constexpr int OFF_W3 = OFF_B2 + MLP_H;
constexpr int OFF_B3 = OFF_W3 + MLP_OUT * MLP_H;
constexpr int MLP_PARAMS = OFF_B3 + MLP_OUT;
static_assert(MLP_PARAMS == 5122, "parameter count");
static_assert(MLP_H == WAVE, "one hidden unit per lane");

// Feature indices (all finite, clipped to a few decades).
enum {
  F_STIFF = 0,     // log10(||A||_inf t_end)
  F_RTOL = 1,      // log10(tol / max_k ||b_k||_inf)
  F_P = 2,         // p / 4
  F_SEED = 3,      // log10(beta / ||u_k||_2): size of the step's Krylov seed w_p
  F_PROGRESS = 4,  // t_k / t_end
  F_TAU_PREV = 5,  // log10(tau_prev ||A||_inf): last accepted substep
  F_M_PREV = 6,    // m_prev / 32
  F_OMEGA_PREV = 7,// log10(omega of the last accepted attempt)
  F_REJ_PREV = 8,  // rejected attempts of the previous step / 4
  F_TAU_PLAIN = 9, // log10(tau_plain ||A||_inf): the plain controller's proposal
  F_M_PLAIN = 10,  // m_plain / 32
  F_LANCZOS = 11   // 1 for the symmetric (Lanczos) process
};

// GELU, tanh form: 0.5 z (1 + tanh(c (z + 0.044715 z^3))), c = sqrt(2/pi).
__device__ __forceinline__ float gelu(float z) {
  const float c = 0.7978845608028654f;
  return 0.5f * z * (1.0f + tanhf(c * (z + 0.044715f * z * z * z)));
}

// d gelu / dz of the same form.
__device__ __forceinline__ float gelu_grad(float z) {
  const float c = 0.7978845608028654f;
  const float u = c * (z + 0.044715f * z * z * z);
  const float th = tanhf(u);
  const float du = c * (1.0f + 3.0f * 0.044715f * z * z);
  return 0.5f * (1.0f + th) + 0.5f * z * (1.0f - th * th) * du;
}

__device__ __forceinline__ float wave_sum_f(float v) {
  double d = wave_sum((double)v);
  return (float)d;
}

// Forward pass by one wave (lane j = hidden unit j).  x: 12 features (any
// memory), out: 2 outputs written by lane 0.  h (LDS, 64 floats) is scratch.
__device__ __forceinline__ void mlp_forward_wave(const float* __restrict__ P, const float* x,
                                                 float* h, float* out) {
  const int j = threadIdx.x % WAVE;
  float z = P[OFF_B1 + j];
#pragma unroll
  for (int i = 0; i < MLP_IN; ++i) z += P[OFF_W1 + j * MLP_IN + i] * x[i];
  h[j] = gelu(z);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  float z2 = P[OFF_B2 + j];
  for (int k = 0; k < MLP_H; ++k) z2 += P[OFF_W2 + j * MLP_H + k] * h[k];
  const float h2 = gelu(z2);
  const float o0 = wave_sum_f(P[OFF_W3 + j] * h2);
  const float o1 = wave_sum_f(P[OFF_W3 + MLP_H + j] * h2);
  if (j == 0) {
    out[0] = P[OFF_B3 + 0] + o0;
    out[1] = P[OFF_B3 + 1] + o1;
  }
}

__device__ __forceinline__ float clampf(float v, float lo, float hi) {
  if (!(v == v)) return 0.0f;
  return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ float log10c(double v, float lo, float hi) {
  if (!(v > 0.0) || !isfinite(v)) return lo;
  return clampf((float)log10(v), lo, hi);
}

}  // namespace pkr
