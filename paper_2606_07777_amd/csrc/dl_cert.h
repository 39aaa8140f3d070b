// Device parts of the certificate (P_gamma(x~), g_gamma(lam), slack and gap,
// as the solver reports them), shared by the single-problem kernels and the
// batched ones: one 1024-thread workgroup per problem, fixed reduction trees,
// so the values do not depend on which launch computes them.
#pragma once
#include <hip/hip_runtime.h>

namespace {

// Deterministic block reduction helpers (fixed tree over 1024 threads).
__device__ inline double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}
__device__ inline double block_max(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Certificate, item part (one workgroup): repair factor r_j =
// rho min_k min(1, b_kj / (A_k x)_j), with rho = min(1, M / sum x) for a
// global-count row (1 without one), max slack, lam.b and -lam.(Ax - b) at the
// FP32 point mu the pass used, and the Lagrangian sum over workgroups.
//   out[0] = sum_w obj_part[w] - mu.b   (dual value g(mu))
//   out[1] = max_r (A x - b)_r^+
//   out[2] = -mu.(A x - b)
__device__ inline void cert_items_body(const double* ax, const double* b, const float* mu, int m, int J, int eq_mask,
                                       int glob, const double* obj_part, int n_wg, float* rfac, double* out,
                                       double* sh) {
  const int mJ = m * J;
  double lb = 0.0, slack = 0.0, lg = 0.0, rho = 1.0;
  if (glob) {
    const double G = ax[mJ], M = b[mJ];
    if (G > M) rho = M > 0.0 ? M / G : 0.0;
    if (threadIdx.x == 0) {
      slack = G - M;
      lb = (double)mu[mJ] * M;
      lg = -(double)mu[mJ] * (G - M);
    }
  }
  for (int j = threadIdx.x; j < J; j += blockDim.x) {
    double rj = rho;
    for (int k = 0; k < m; ++k) {
      const int r = k * J + j;
      const double viol = ax[r] - b[r];
      const bool eq = (eq_mask >> k) & 1;
      slack = fmax(slack, eq ? fabs(viol) : viol);
      lb += (double)mu[r] * b[r];
      lg -= (double)mu[r] * viol;
      if (!eq && ax[r] > b[r]) rj = fmin(rj, b[r] > 0.0 ? rho * (b[r] / ax[r]) : 0.0);
    }
    rfac[j] = (float)rj;
  }
  double os = 0.0;
  for (int w = threadIdx.x; w < n_wg; w += blockDim.x) os += obj_part[w];
  lb = block_sum(lb, sh);
  lg = block_sum(lg, sh);
  os = block_sum(os, sh);
  slack = block_max(slack, sh);
  if (threadIdx.x == 0) {
    out[0] = os - lb;
    out[1] = slack;
    out[2] = lg;
  }
}

// out[3] = sum_w pobj_part[w]   (primal value of the repaired point)
__device__ inline void cert_final_body(const double* pobj_part, int n_wg, double* out, double* sh) {
  double s = 0.0;
  for (int w = threadIdx.x; w < n_wg; w += blockDim.x) s += pobj_part[w];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[3] = s;
}

}  // namespace
