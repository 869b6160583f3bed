// Training side of the learned (tau, m) proposer: batched inference, the
// loss gradient, Adam training and the hindsight labels of recorded steps.
//
// Loss: mean squared error over all outputs of all rows,
//   L = 1/(2B) sum_r sum_o (y_ro - t_ro)^2,
// targets t = (log10(tau* ||A||_inf), m* / 32).  Adam (Kingma & Ba) with
// beta1 = 0.9, beta2 = 0.999, eps = 1e-8, one update per minibatch.
//
// Labels (hindsight): a recorded step's Krylov basis does not depend on tau,
// and its prefixes are the bases of smaller m (the trace extends it to m_cap
// columns).  For every candidate m' the largest tau with omega(tau, m') <=
// gamma is found by bisection on log tau (the exponential of the augmented
// matrix only), and the label is the (tau*, m') with the least cost per unit
// time: C1(m') / tau* (eq. 4 with the product count of eq. 8), or a measured
// time model of the step on the device divided by tau*.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "../../include/phipm.h"
#include "host_common.hpp"

using namespace pkr;

namespace {

constexpr int MB = 64;  // rows per minibatch chunk in LDS

struct MlpSmem {
  float P[MLP_PARAMS];
  float G[MLP_PARAMS];
  float X[MB][MLP_IN];
  float Z1[MB][MLP_H];  // pre-activations, then their gradients
  float A1[MB][MLP_H];
  float Z2[MB][MLP_H];
  float A2[MB][MLP_H];
  float E[MB][MLP_OUT]; // output errors, then dL/dy
  float red[NWAVES];
};

// Forward and backward over rows [r0, r0+B) (B <= MB): G += wgt * dL_B/dP
// where L_B is the mean loss of the chunk; returns the chunk's loss sum
// sum_r sum_o e^2 (in thread 0).
__device__ float chunk_grad(MlpSmem& s, const float* __restrict__ X, const float* __restrict__ T,
                            int r0, int B, float wgt) {
  const int tid = threadIdx.x;
  for (int e = tid; e < B * MLP_IN; e += BLOCK) s.X[e / MLP_IN][e % MLP_IN] = X[(size_t)r0 * MLP_IN + e];
  __syncthreads();
  for (int e = tid; e < B * MLP_H; e += BLOCK) {
    const int r = e / MLP_H, j = e % MLP_H;
    float z = s.P[OFF_B1 + j];
    for (int i = 0; i < MLP_IN; ++i) z += s.P[OFF_W1 + j * MLP_IN + i] * s.X[r][i];
    s.Z1[r][j] = z;
    s.A1[r][j] = gelu(z);
  }
  __syncthreads();
  for (int e = tid; e < B * MLP_H; e += BLOCK) {
    const int r = e / MLP_H, j = e % MLP_H;
    float z = s.P[OFF_B2 + j];
    for (int k = 0; k < MLP_H; ++k) z += s.P[OFF_W2 + j * MLP_H + k] * s.A1[r][k];
    s.Z2[r][j] = z;
    s.A2[r][j] = gelu(z);
  }
  __syncthreads();
  float lsum = 0.0f;
  if (tid < B * MLP_OUT) {
    const int r = tid / MLP_OUT, o = tid % MLP_OUT;
    float y = s.P[OFF_B3 + o];
    for (int j = 0; j < MLP_H; ++j) y += s.P[OFF_W3 + o * MLP_H + j] * s.A2[r][j];
    const float e = y - T[(size_t)(r0 + r) * MLP_OUT + o];
    s.E[r][o] = e;
  }
  __syncthreads();
  if (tid == 0) {
    for (int r = 0; r < B; ++r)
      for (int o = 0; o < MLP_OUT; ++o) lsum += s.E[r][o] * s.E[r][o];
  }
  __syncthreads();
  // dL_B/dy = e / B
  const float inv = 1.0f / (float)B;
  if (tid < B * MLP_OUT) s.E[tid / MLP_OUT][tid % MLP_OUT] *= inv;
  __syncthreads();
  // output layer
  for (int e = tid; e < MLP_OUT * MLP_H; e += BLOCK) {
    const int o = e / MLP_H, j = e % MLP_H;
    float g = 0.0f;
    for (int r = 0; r < B; ++r) g += s.E[r][o] * s.A2[r][j];
    s.G[OFF_W3 + e] += wgt * g;
  }
  if (tid < MLP_OUT) {
    float g = 0.0f;
    for (int r = 0; r < B; ++r) g += s.E[r][tid];
    s.G[OFF_B3 + tid] += wgt * g;
  }
  // dZ2 = (E W3) * gelu'(Z2), in place of Z2
  for (int e = tid; e < B * MLP_H; e += BLOCK) {
    const int r = e / MLP_H, j = e % MLP_H;
    float d = 0.0f;
    for (int o = 0; o < MLP_OUT; ++o) d += s.E[r][o] * s.P[OFF_W3 + o * MLP_H + j];
    s.Z2[r][j] = d * gelu_grad(s.Z2[r][j]);
  }
  __syncthreads();
  for (int e = tid; e < MLP_H * MLP_H; e += BLOCK) {
    const int j = e / MLP_H, k = e % MLP_H;
    float g = 0.0f;
    for (int r = 0; r < B; ++r) g += s.Z2[r][j] * s.A1[r][k];
    s.G[OFF_W2 + e] += wgt * g;
  }
  if (tid < MLP_H) {
    float g = 0.0f;
    for (int r = 0; r < B; ++r) g += s.Z2[r][tid];
    s.G[OFF_B2 + tid] += wgt * g;
  }
  // dZ1 = (dZ2 W2) * gelu'(Z1), in place of Z1
  for (int e = tid; e < B * MLP_H; e += BLOCK) {
    const int r = e / MLP_H, k = e % MLP_H;
    float d = 0.0f;
    for (int j = 0; j < MLP_H; ++j) d += s.Z2[r][j] * s.P[OFF_W2 + j * MLP_H + k];
    s.Z1[r][k] = d * gelu_grad(s.Z1[r][k]);
  }
  __syncthreads();
  for (int e = tid; e < MLP_H * MLP_IN; e += BLOCK) {
    const int j = e / MLP_IN, i = e % MLP_IN;
    float g = 0.0f;
    for (int r = 0; r < B; ++r) g += s.Z1[r][j] * s.X[r][i];
    s.G[OFF_W1 + e] += wgt * g;
  }
  if (tid < MLP_H) {
    float g = 0.0f;
    for (int r = 0; r < B; ++r) g += s.Z1[r][tid];
    s.G[OFF_B1 + tid] += wgt * g;
  }
  __syncthreads();
  return lsum;
}

// Gradient of the mean loss over all rows (chunks weighted by their size).
__global__ __launch_bounds__(BLOCK) void k_mlp_grad(const float* params, const float* X,
                                                   const float* T, int rows, float* grad,
                                                   float* loss) {
  __shared__ MlpSmem s;
  for (int e = threadIdx.x; e < MLP_PARAMS; e += BLOCK) {
    s.P[e] = params[e];
    s.G[e] = 0.0f;
  }
  __syncthreads();
  float lsum = 0.0f;
  for (int r0 = 0; r0 < rows; r0 += MB) {
    const int B = rows - r0 < MB ? rows - r0 : MB;
    lsum += chunk_grad(s, X, T, r0, B, (float)B / (float)rows);
  }
  for (int e = threadIdx.x; e < MLP_PARAMS; e += BLOCK) grad[e] = s.G[e];
  if (threadIdx.x == 0) *loss = lsum / (2.0f * (float)rows);
}

// Adam over minibatches of `batch` rows (<= MB), `epochs` passes over the
// rows in order.  loss[e] = mean loss of epoch e, measured with the
// parameters each minibatch saw.
__global__ __launch_bounds__(BLOCK) void k_mlp_train(float* params, float* am, float* av,
                                                    const float* X, const float* T, int rows,
                                                    int batch, int epochs, float lr, int step0,
                                                    float* loss) {
  __shared__ MlpSmem s;
  for (int e = threadIdx.x; e < MLP_PARAMS; e += BLOCK) s.P[e] = params[e];
  __syncthreads();
  long long step = step0;
  for (int ep = 0; ep < epochs; ++ep) {
    float lsum = 0.0f;
    for (int r0 = 0; r0 < rows; r0 += batch) {
      const int B = rows - r0 < batch ? rows - r0 : batch;
      for (int e = threadIdx.x; e < MLP_PARAMS; e += BLOCK) s.G[e] = 0.0f;
      __syncthreads();
      lsum += chunk_grad(s, X, T, r0, B, 1.0f);
      ++step;
      const double b1t = 1.0 - pow(0.9, (double)step);
      const double b2t = 1.0 - pow(0.999, (double)step);
      const float c1 = (float)(1.0 / b1t), c2 = (float)(1.0 / b2t);
      for (int e = threadIdx.x; e < MLP_PARAMS; e += BLOCK) {
        const float g = s.G[e];
        const float m = 0.9f * am[e] + 0.1f * g;
        const float v = 0.999f * av[e] + 0.001f * g * g;
        am[e] = m;
        av[e] = v;
        s.P[e] -= lr * (m * c1) / (sqrtf(v * c2) + 1e-8f);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) loss[ep] = lsum / (2.0f * (float)rows);
  }
  for (int e = threadIdx.x; e < MLP_PARAMS; e += BLOCK) params[e] = s.P[e];
}

// Inference for many rows: one wave per row, the solver's own routine.
__global__ __launch_bounds__(BLOCK) void k_mlp_forward(const float* params, const float* X,
                                                      int rows, float* Y) {
  __shared__ float h[NWAVES][MLP_H];
  __shared__ float y[NWAVES][MLP_OUT];
  const int wv = threadIdx.x / WAVE;
  const int r = blockIdx.x * NWAVES + wv;
  if (r < rows) {
    mlp_forward_wave(params, X + (size_t)r * MLP_IN, h[wv], y[wv]);
    __builtin_amdgcn_wave_barrier();
    if (threadIdx.x % WAVE == 0) {
      Y[(size_t)r * MLP_OUT + 0] = y[wv][0];
      Y[(size_t)r * MLP_OUT + 1] = y[wv][1];
    }
  }
}

// omega(tau) of eq. taunew for the first mm columns of a recorded step, with
// the augmented exponential of the decision step; returns ||tau K||_1 too.
__device__ double label_omega(const TraceStep& r, int mm, double tau, double* ex, double* L,
                              double* knorm) {
  __shared__ double s_c, s_norm;
  __shared__ int s_sq;
  const int p = r.p;
  const int N = mm + p + 1;
  for (int e = threadIdx.x; e < N * N; e += BLOCK) {
    const int i = e / N, j = e - i * N;
    double v = 0.0;
    if (i < mm && j < mm) v = tau * r.H[(size_t)i * M_CAP + j];
    else if (i == 0 && j == mm) v = tau;
    else if (i >= mm && i < mm + p && j == i + 1) v = tau;
    ex[e] = v;
  }
  __syncthreads();
  const double* E = wg_expm(N, ex, L, &s_norm, &s_sq, mm + p, mm + p);
  if (threadIdx.x == 0) s_c = E[(size_t)(mm - 1) * N + mm + p];
  __syncthreads();
  *knorm = s_norm;
  const double hn = r.H[(size_t)mm * M_CAP + (mm - 1)];
  const double eps = r.beta * fabs(hn) * fabs(s_c);
  return r.t_end * eps / (tau * r.tol);
}

// Time of one step of dimension mm under the device time model.
__device__ double label_step_time(const TraceStep& r, int mm, const phipm_label_costs& c) {
  const double s = 8.0, n = r.n, nnz = r.nnz;
  const int p = r.p;
  const double S = (s + 4.0) * nnz + 4.0 * (n + 1.0) + 2.0 * s * n;
  double bytes = p * S;
  for (int j = 1; j <= p; ++j) bytes += s * n * (p - j + 1);
  for (int j = 0; j < mm; ++j) {
    const double K = r.lanczos ? (j + 1 < 2 ? j + 1 : 2) : j + 1;
    bytes += S + (4.0 * K + 8.0) * s * n;
  }
  bytes += 2.0 * s * n + s * n * (p + 1 > 1 ? p + 1 : 1) + (mm + 1.0) * s * n;
  double G = ceil(n / 1024.0);
  if (G > c.workgroups) G = c.workgroups;
  if (G < 1.0) G = 1.0;
  const double bw = fmin(c.bw_bytes_per_s, G * c.wg_bytes_per_s);
  const double sync = G > 1.0 ? c.sync_s : c.sync1_s;
  const double syncs = 3.0 * mm + (p > 1 ? p : 1) + 2.0;
  return syncs * sync + bytes / bw + c.expm_s[mm + p + 1];
}

// Candidate dimensions: every m up to 16, then every 4th, and m_have.
__device__ __forceinline__ int label_next_m(int mm, int mh) {
  int nx = mm < 16 ? mm + 1 : (mm / 4 + 1) * 4;
  if (nx > mh && mm < mh) nx = mh;
  return nx;
}

__global__ __launch_bounds__(BLOCK) void k_label(const TraceStep* rec, int count, float* X,
                                                float* T, double* scratch, int use_costs,
                                                phipm_label_costs costs) {
  __shared__ double L[DENSE_LDS];
  double* ex = scratch + (size_t)blockIdx.x * 8 * NMAX_EXPM * NMAX_EXPM;
  for (int q = blockIdx.x; q < count; q += gridDim.x) {
    const TraceStep& r = rec[q];
    const int mh = r.m_have;
    const double rem = r.t_end - r.t;
    double best_cost = INFINITY, best_tau = r.tau;
    int best_m = r.m_use;
    for (int mm = 1; mm <= mh; mm = label_next_m(mm, mh)) {
      const double hn = r.H[(size_t)mm * M_CAP + (mm - 1)];
      double ts, kn;
      if (hn == 0.0) {
        ts = rem;  // invariant subspace: exact for any tau
        label_omega(r, mm, ts, ex, L, &kn);
      } else {
        double tlo = r.tau / 4096.0, thi = rem;
        if (tlo > thi) tlo = thi;
        if (label_omega(r, mm, thi, ex, L, &kn) <= CTRL_GAMMA) {
          ts = thi;
        } else if (label_omega(r, mm, tlo, ex, L, &kn) > CTRL_GAMMA) {
          ts = tlo;
        } else {
          for (int it = 0; it < 20; ++it) {
            const double mid = sqrt(tlo * thi);
            if (label_omega(r, mm, mid, ex, L, &kn) <= CTRL_GAMMA) tlo = mid;
            else thi = mid;
          }
          ts = tlo;
          label_omega(r, mm, ts, ex, L, &kn);
        }
      }
      const double work =
          use_costs ? label_step_time(r, mm, costs)
                    : ctrl_C1(r.lanczos != 0, (double)mm, r.p, (double)r.nnz, (double)r.n,
                              ctrl_M(kn));
      const double cost = work / ts;
      if (cost < best_cost) {
        best_cost = cost;
        best_tau = ts;
        best_m = mm;
      }
    }
    if (threadIdx.x < MLP_IN) X[(size_t)q * MLP_IN + threadIdx.x] = r.feat[threadIdx.x];
    if (threadIdx.x == 0) {
      T[(size_t)q * MLP_OUT + 0] = (float)log10(best_tau * r.anorm);
      T[(size_t)q * MLP_OUT + 1] = (float)best_m / 32.0f;
    }
    __syncthreads();
  }
}

constexpr int LABEL_GRID_MAX = 256;

}  // namespace

extern "C" {

int phipm_mlp_forward(const float* params, const float* X, int rows, float* Y,
                      phipm_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (!params || rows < 0 || (rows > 0 && (!X || !Y))) return PHIPM_EINVAL;
  if (rows == 0) return PHIPM_OK;
  const int grid = (rows + NWAVES - 1) / NWAVES;
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(BLOCK), 0, stream, params, X, rows, Y);
  return hipGetLastError() == hipSuccess ? PHIPM_OK : PHIPM_EHIP;
}

int phipm_mlp_grad(const float* params, const float* X, const float* T, int rows, float* grad,
                   float* loss, phipm_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (!params || !X || !T || !grad || !loss || rows < 1) return PHIPM_EINVAL;
  hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(BLOCK), 0, stream, params, X, T, rows, grad, loss);
  return hipGetLastError() == hipSuccess ? PHIPM_OK : PHIPM_EHIP;
}

int phipm_mlp_train(float* params, float* adam_m, float* adam_v, const float* X, const float* T,
                    int rows, int batch, int epochs, float lr, int step0, float* loss,
                    phipm_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (!params || !adam_m || !adam_v || !X || !T || !loss || rows < 1 || batch < 1 ||
      batch > MB || epochs < 0 || step0 < 0 || !(lr > 0.0f) || !std::isfinite(lr))
    return PHIPM_EINVAL;
  if (epochs == 0) return PHIPM_OK;
  hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(BLOCK), 0, stream, params, adam_m, adam_v, X, T,
                     rows, batch, epochs, lr, step0, loss);
  return hipGetLastError() == hipSuccess ? PHIPM_OK : PHIPM_EHIP;
}

size_t phipm_label_workspace_bytes(int count) {
  const int grid = std::max(1, std::min(count, LABEL_GRID_MAX));
  return sizeof(double) * 8 * (size_t)NMAX_EXPM * NMAX_EXPM * (size_t)grid;
}

int phipm_label_steps(const phipm_trace_step* rec, int count, float* X, float* T,
                      void* workspace, size_t ws_bytes, const phipm_label_costs* costs,
                      phipm_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (count < 0 || (count > 0 && (!rec || !X || !T || !workspace))) return PHIPM_EINVAL;
  if (costs && !(costs->sync_s >= 0.0 && costs->sync1_s >= 0.0 && costs->bw_bytes_per_s > 0.0 &&
                 costs->wg_bytes_per_s > 0.0 && costs->workgroups >= 1))
    return PHIPM_EINVAL;
  if (count == 0) return PHIPM_OK;
  if (ws_bytes < phipm_label_workspace_bytes(count)) return PHIPM_ENOMEM;
  const int grid = std::min(count, LABEL_GRID_MAX);
  phipm_label_costs c{};
  if (costs) c = *costs;
  hipLaunchKernelGGL(k_label, dim3(grid), dim3(BLOCK), 0, stream,
                     reinterpret_cast<const TraceStep*>(rec), count, X, T,
                     static_cast<double*>(workspace), costs ? 1 : 0, c);
  return hipGetLastError() == hipSuccess ? PHIPM_OK : PHIPM_EHIP;
}

}  // extern "C"
