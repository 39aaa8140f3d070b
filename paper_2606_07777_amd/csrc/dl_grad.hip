// Gradient pass of the dual ascent on gfx950 (one launch per evaluation).
//
// Computes, for every user i, v_i = -(c_i + sum_k a_ki * lam_k[items of i]) / gamma
// and x_i = Pi_{C_i}(v_i) (eq. 3), then the per-item sums (A_k x)_j that give the
// gradient A x - b (eq. 4).  The paper evaluates these as two sparse products
// around a bucketed, fused simplex projection (Sections 4.1-4.3); here the three
// are one streaming pass over the user-major CSR:
//
//  * each workgroup (1024 lanes, one per CU) stages lam (m*J FP32) in LDS once
//    and gathers from there;
//  * users are reordered by degree, longest first, and served by groups of
//    2^glog lanes holding up to KMAX elements each in registers (lane, group or
//    whole-wavefront per user); rows longer than 64*KMAX loop over the row;
//  * the projection finds the simplex threshold by Newton steps from below on
//    f(theta) = sum max(v - theta, 0) - z (each step is the exact threshold of
//    the current active set, so it stops when the set stops shrinking), with
//    the paper's early exit when the positive part already fits;
//  * a_k * x is rounded to a per-family fixed-point grid and added with 64-bit
//    integer LDS atomics into a per-workgroup histogram over items; integer
//    addition is associative, so the sums are bitwise reproducible for any
//    schedule and no float atomics are used; the histogram is written once per
//    workgroup and summed over workgroups by the update kernel.
#include <string.h>

#include "dl_common.h"

namespace {

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float swz_xor16(float v) {
  // ds_swizzle bit mode: and_mask 0x1F, or_mask 0, xor_mask 0x10 (within 32 lanes)
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}

struct OpSum {
  __device__ __forceinline__ float operator()(float a, float b) const { return a + b; }
};
struct OpMax {
  __device__ __forceinline__ float operator()(float a, float b) const { return fmaxf(a, b); }
};

// All-reduce over aligned groups of 2^glog lanes.  Every lane of a group ends
// with the same bits (each combining step adds the same two operands).
template <typename Op>
__device__ __forceinline__ float group_allreduce(float v, int glog, Op op) {
  if (glog > 0) v = op(v, dpp_f<0xB1>(v));   // quad_perm(1,0,3,2): lane ^ 1
  if (glog > 1) v = op(v, dpp_f<0x4E>(v));   // quad_perm(2,3,0,1): lane ^ 2
  if (glog > 2) v = op(v, dpp_f<0x141>(v));  // row_half_mirror: pairs the two quads of 8
  if (glog > 3) v = op(v, dpp_f<0x140>(v));  // row_mirror: pairs the two halves of 16
  if (glog > 4) v = op(v, swz_xor16(v));
  if (glog > 5) v = op(v, __shfl_xor(v, 32, 64));
  return v;
}

template <typename TV>
__device__ __forceinline__ float load_val(const void* base, int64_t e);
template <>
__device__ __forceinline__ float load_val<float>(const void* base, int64_t e) {
  return __builtin_nontemporal_load(reinterpret_cast<const float*>(base) + e);
}
template <>
__device__ __forceinline__ float load_val<uint16_t>(const void* base, int64_t e) {
  uint32_t h = __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(base) + e);
  return __uint_as_float(h << 16);
}

__device__ __forceinline__ void hist_add(unsigned long long* h, int r, float w, float qs) {
  int q = __float2int_rn(w * qs);
  if (q != 0) atomicAdd(h + r, (unsigned long long)(long long)q);
}

// Threshold of the simplex projection for one group, given v in registers.
// Returns theta; the projection is max(v - theta, 0).  Lanes of invalid groups
// (no user) carry only -inf and return 0.
template <int KMAX>
__device__ __forceinline__ float simplex_theta(const float (&v)[KMAX], int K, int glog, float z, bool eq) {
  float vmax = -INFINITY, sp = 0.f, cp = 0.f;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
      vmax = fmaxf(vmax, v[k]);
      float p = fmaxf(v[k], 0.f);
      sp += p;
      cp += (v[k] > 0.f) ? 1.f : 0.f;
    }
  }
  vmax = group_allreduce(vmax, glog, OpMax());
  sp = group_allreduce(sp, glog, OpSum());
  cp = group_allreduce(cp, glog, OpSum());
  float theta = 0.f;
  bool done;
  if (vmax == -INFINITY) {
    done = true;                           // no user in this group
  } else if (!eq && sp <= z) {
    done = true;                           // positive part already in the simplex
  } else {
    done = false;
    theta = vmax - z;                      // f(vmax - z) >= 0: a point left of the root
    if (sp > z && cp > 0.f) theta = fmaxf(theta, (sp - z) / cp);  // Newton step from 0
  }
  float prev = -1.f;
  for (int it = 0; it < 64 && __any(!done); ++it) {
    float f = 0.f, cnt = 0.f;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < K) {
        float t = v[k] - theta;
        f += fmaxf(t, 0.f);
        cnt += (t > 0.f) ? 1.f : 0.f;
      }
    }
    f = group_allreduce(f, glog, OpSum());
    cnt = group_allreduce(cnt, glog, OpSum());
    if (!done) {
      // Newton step: exact threshold of the active set {v > theta}
      float nt = theta + (f - z) / cnt;
      bool stable = (cnt == prev) || (fabsf(f - z) <= z * 0x1p-22f);
      theta = nt;
      prev = cnt;
      done = stable;
    }
  }
  return theta;
}

template <int MF, bool HAS_A, int KMAX, typename TV, int MODE>
__device__ __forceinline__ void group_task(const dl_grad_args& A, int64_t t, const dl_bucket& B,
                                           const float* s_mu, const float* s_rf, unsigned long long* s_hist,
                                           int lane, double& acc) {
  const int glog = B.glog;
  const int g = 1 << glog;
  const int64_t u_first = B.user_begin + (t - B.task_begin) * (int64_t)(64 >> glog);
  const int grp = lane >> glog;
  const int lid = lane & (g - 1);
  const int64_t u = u_first + grp;
  const bool valid = u < B.user_end;
  int64_t s = 0;
  int d = 0;
  if (valid) {
    s = A.rp[u];
    d = (int)(A.rp[u + 1] - s);
  }
  // users are sorted longest first: lane 0 holds the longest row of the task
  const int d0 = __builtin_amdgcn_readfirstlane(d);
  const int K = (d0 + g - 1) >> glog;
  const int64_t os = ((MODE & M_VIN) || A.x_out) && valid ? A.orig_rp[u] : 0;

  float v[KMAX];
  int jj[KMAX];
  float cc[KMAX];
  float aa[HAS_A ? MF : 1][KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    v[k] = -INFINITY;
    jj[k] = 0;
    cc[k] = 0.f;
    if (k < K) {
      const int e = lid + (k << glog);
      if (e < d) {
        if (MODE & M_VIN) {
          v[k] = A.v_in[os + e];
        } else {
          const int j = A.idx[s + e];
          jj[k] = j;
          const float c = load_val<TV>(A.cval, s + e);
          float sdot = 0.f;
#pragma unroll
          for (int f = 0; f < MF; ++f) {
            if (f < A.m) {
              float af = 1.f;
              if (HAS_A && A.a_slot[f] >= 0) {
                af = load_val<TV>(A.aval, (int64_t)A.a_slot[f] * A.nnz + s + e);
              }
              if (HAS_A) aa[f][k] = af;
              sdot = fmaf(af, s_mu[f * A.J + j], sdot);
            }
          }
          cc[k] = c;
          v[k] = (c + sdot) * A.neg_inv_gamma;  // eq. 3 argument
        }
      }
    }
  }

  const float z = A.radius;
  float theta = 0.f;
  const bool box = (A.proj == DL_PROJ_BOX);
  if (!box) theta = simplex_theta<KMAX>(v, K, glog, z, A.proj == DL_PROJ_SIMPLEX_EQ);

  float lobj = 0.f;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
      const int e = lid + (k << glog);
      if (e < d) {
        float x = box ? fminf(fmaxf(v[k], 0.f), z) : fmaxf(v[k] - theta, 0.f);
        if (A.x_out) A.x_out[os + e] = x;
        if (MODE & M_HIST) {
#pragma unroll
          for (int f = 0; f < MF; ++f) {
            if (f < A.m) {
              float w = (HAS_A && A.a_slot[f] >= 0) ? aa[HAS_A ? f : 0][k] * x : x;
              hist_add(s_hist, f * A.J + jj[k], w, A.qscale[f]);
            }
          }
        }
        if (MODE & M_OBJ) {
          // (c + A^T lam) x + gamma/2 x^2, with c + A^T lam = -gamma v
          lobj += x * fmaf(0.5f * A.gamma, x, -A.gamma * v[k]);
        }
        if (MODE & M_REPAIR) {
          const float xt = s_rf[jj[k]] * x;
          lobj += xt * fmaf(0.5f * A.gamma, xt, cc[k]);
        }
      }
    }
  }
  if (MODE & (M_OBJ | M_REPAIR)) acc += (double)lobj;
}

// Rows longer than 64*KMAX: one wavefront per user, re-reading the row per
// Newton step (the row stays in L1/L2, so HBM sees it once).
template <int MF, bool HAS_A, typename TV, int MODE>
__device__ __forceinline__ float long_v(const dl_grad_args& A, const float* s_mu, int64_t s, int64_t os, int e,
                                        int& j, float& c, float (&af)[HAS_A ? MF : 1]) {
  if (MODE & M_VIN) return A.v_in[os + e];
  j = A.idx[s + e];
  c = load_val<TV>(A.cval, s + e);
  float sdot = 0.f;
#pragma unroll
  for (int f = 0; f < MF; ++f) {
    if (f < A.m) {
      float a = 1.f;
      if (HAS_A && A.a_slot[f] >= 0) a = load_val<TV>(A.aval, (int64_t)A.a_slot[f] * A.nnz + s + e);
      if (HAS_A) af[f] = a;
      sdot = fmaf(a, s_mu[f * A.J + j], sdot);
    }
  }
  return (c + sdot) * A.neg_inv_gamma;
}

template <int MF, bool HAS_A, typename TV, int MODE>
__device__ __forceinline__ void long_task(const dl_grad_args& A, int64_t t, const dl_bucket& B, const float* s_mu,
                                       const float* s_rf, unsigned long long* s_hist, int lane, double& acc) {
  const int64_t u = B.user_begin + (t - B.task_begin);
  const int64_t s = A.rp[u];
  const int d = (int)(A.rp[u + 1] - s);
  const int64_t os = ((MODE & M_VIN) || A.x_out) ? A.orig_rp[u] : 0;
  const float z = A.radius;
  const bool box = (A.proj == DL_PROJ_BOX);
  int j;
  float c;
  float af[HAS_A ? MF : 1];
  float theta = 0.f;
  if (!box) {
    float vmax = -INFINITY, sp = 0.f, cp = 0.f;
    for (int e = lane; e < d; e += 64) {
      float v = long_v<MF, HAS_A, TV, MODE>(A, s_mu, s, os, e, j, c, af);
      vmax = fmaxf(vmax, v);
      sp += fmaxf(v, 0.f);
      cp += v > 0.f ? 1.f : 0.f;
    }
    vmax = group_allreduce(vmax, 6, OpMax());
    sp = group_allreduce(sp, 6, OpSum());
    cp = group_allreduce(cp, 6, OpSum());
    const bool eq = A.proj == DL_PROJ_SIMPLEX_EQ;
    if (eq || sp > z) {
      theta = vmax - z;
      if (sp > z && cp > 0.f) theta = fmaxf(theta, (sp - z) / cp);
      float prev = -1.f;
      for (int it = 0; it < 64; ++it) {
        float f = 0.f, cnt = 0.f;
        for (int e = lane; e < d; e += 64) {
          float v = long_v<MF, HAS_A, TV, MODE>(A, s_mu, s, os, e, j, c, af);
          float tt = v - theta;
          f += fmaxf(tt, 0.f);
          cnt += tt > 0.f ? 1.f : 0.f;
        }
        f = group_allreduce(f, 6, OpSum());
        cnt = group_allreduce(cnt, 6, OpSum());
        float nt = theta + (f - z) / cnt;
        bool stable = (cnt == prev) || (fabsf(f - z) <= z * 0x1p-22f);
        theta = nt;
        prev = cnt;
        if (stable) break;
      }
    }
  }
  float lobj = 0.f;
  for (int e = lane; e < d; e += 64) {
    float v = long_v<MF, HAS_A, TV, MODE>(A, s_mu, s, os, e, j, c, af);
    float x = box ? fminf(fmaxf(v, 0.f), z) : fmaxf(v - theta, 0.f);
    if (A.x_out) A.x_out[os + e] = x;
    if (MODE & M_HIST) {
#pragma unroll
      for (int f = 0; f < MF; ++f) {
        if (f < A.m) {
          float w = (HAS_A && A.a_slot[f] >= 0) ? af[HAS_A ? f : 0] * x : x;
          hist_add(s_hist, f * A.J + j, w, A.qscale[f]);
        }
      }
    }
    if (MODE & M_OBJ) lobj += x * fmaf(0.5f * A.gamma, x, -A.gamma * v);
    if (MODE & M_REPAIR) {
      const float xt = s_rf[j] * x;
      lobj += xt * fmaf(0.5f * A.gamma, xt, c);
    }
  }
  if (MODE & (M_OBJ | M_REPAIR)) acc += (double)lobj;
}

template <int MF, bool HAS_A, int KMAX, typename TV, int MODE>
__global__ void __launch_bounds__(DL_WG) grad_pass(dl_grad_args A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int mJ = A.m * A.J;
  const bool need_mu = !(MODE & M_VIN);
  float* s_mu = reinterpret_cast<float*>(smem);
  const int mu_n = need_mu ? mJ : 0;
  float* s_rf = s_mu + mu_n;
  const int rf_n = (MODE & M_REPAIR) ? A.J : 0;
  size_t off = ((size_t)(mu_n + rf_n) * 4 + 15) & ~(size_t)15;
  unsigned long long* s_hist = reinterpret_cast<unsigned long long*>(smem + off);
  const int hist_n = (MODE & M_HIST) ? mJ : 0;
  double* s_obj = reinterpret_cast<double*>(smem + off + (size_t)hist_n * 8);

  const int tid = threadIdx.x;
  for (int r = tid; r < mu_n; r += DL_WG) s_mu[r] = A.mu[r];
  for (int r = tid; r < rf_n; r += DL_WG) s_rf[r] = A.rfac[r];
  for (int r = tid; r < hist_n; r += DL_WG) s_hist[r] = 0ull;
  __syncthreads();

  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int64_t t0 = A.wg_task[blockIdx.x];
  const int64_t t1 = A.wg_task[blockIdx.x + 1];
  double acc = 0.0;
  int b = 0;
  for (int64_t t = t0 + wave; t < t1; t += DL_WAVES) {
    while (b + 1 < A.n_buckets && t >= A.bk[b + 1].task_begin) ++b;
    const dl_bucket& B = A.bk[b];
    if (B.glog == DL_LONG) {
      long_task<MF, HAS_A, TV, MODE>(A, t, B, s_mu, s_rf, s_hist, lane, acc);
    } else {
      group_task<MF, HAS_A, KMAX, TV, MODE>(A, t, B, s_mu, s_rf, s_hist, lane, acc);
    }
  }
  if (MODE & (M_OBJ | M_REPAIR)) {
    // fixed-order FP64 reduction: lanes of a wavefront, then wavefronts in order
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) s_obj[wave] = acc;
  }
  __syncthreads();
  if (MODE & M_HIST) {
    unsigned long long* dst = A.part + (size_t)blockIdx.x * mJ;
    for (int r = tid; r < mJ; r += DL_WG) dst[r] = s_hist[r];
  }
  if ((MODE & (M_OBJ | M_REPAIR)) && tid == 0) {
    double tot = 0.0;
    for (int w = 0; w < DL_WAVES; ++w) tot += s_obj[w];
    A.obj_part[blockIdx.x] = tot;
  }
}

template <int MF, bool HAS_A, int KMAX, typename TV, int MODE>
dl_status launch_one(const dl_problem* P, const dl_grad_args& A, size_t lds) {
  hipLaunchKernelGGL((grad_pass<MF, HAS_A, KMAX, TV, MODE>), dim3(P->n_wg), dim3(DL_WG), lds, P->stream, A);
  DL_HIP_TRY(hipGetLastError());
  return DL_OK;
}

template <int MF, bool HAS_A, int KMAX, typename TV>
dl_status launch_mode(const dl_problem* P, int mode, const dl_grad_args& A, size_t lds) {
  switch (mode) {
    case M_HIST: return launch_one<MF, HAS_A, KMAX, TV, M_HIST>(P, A, lds);
    case M_HIST | M_OBJ: return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ>(P, A, lds);
    case M_REPAIR: return launch_one<MF, HAS_A, KMAX, TV, M_REPAIR>(P, A, lds);
    case M_VIN: return launch_one<MF, HAS_A, KMAX, TV, M_VIN>(P, A, lds);
    default: dl_set_error("internal: unknown gradient-pass mode"); return DL_EINVAL;
  }
}

template <int MF, bool HAS_A, int KMAX>
dl_status launch_storage(const dl_problem* P, int mode, const dl_grad_args& A, size_t lds) {
  if (P->storage == DL_BF16) return launch_mode<MF, HAS_A, KMAX, uint16_t>(P, mode, A, lds);
  return launch_mode<MF, HAS_A, KMAX, float>(P, mode, A, lds);
}

template <int MF, bool HAS_A, int KMAX, typename TV>
void set_attr_all() {
  const int big = 160 * 1024;
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_REPAIR>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_VIN>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

}  // namespace

size_t dl_grad_lds_bytes(const dl_problem* P, int mode) {
  const size_t mJ = (size_t)P->m * P->J;
  size_t mu_n = (mode & M_VIN) ? 0 : mJ;
  size_t rf_n = (mode & M_REPAIR) ? (size_t)P->J : 0;
  size_t off = ((mu_n + rf_n) * 4 + 15) & ~(size_t)15;
  size_t hist = (mode & M_HIST) ? mJ * 8 : 0;
  return off + hist + DL_WAVES * sizeof(double);
}

dl_status dl_grad_prepare(const dl_problem* P) {
  if (P->mf == 1 && !P->has_a) {
    set_attr_all<1, false, 16, float>();
    set_attr_all<1, false, 16, uint16_t>();
  } else if (P->mf == 1) {
    set_attr_all<1, true, 16, float>();
    set_attr_all<1, true, 16, uint16_t>();
  } else {
    set_attr_all<4, true, 8, float>();
    set_attr_all<4, true, 8, uint16_t>();
  }
  return DL_OK;
}

dl_status dl_launch_grad(const dl_problem* P, int mode, const float* mu, double gamma, const float* rfac,
                         const float* v_in, float* x_out, double* obj_part) {
  if (P->n_wg <= 0) return DL_OK;
  dl_grad_args A;
  memset(&A, 0, sizeof(A));
  A.rp = P->rp;
  A.idx = P->idx;
  A.cval = P->cval;
  A.aval = P->aval;
  A.orig_rp = P->orig_rp;
  A.nnz = P->nnz;
  A.J = P->J;
  A.m = P->m;
  for (int k = 0; k < DL_MAX_FAMILIES; ++k) {
    A.a_slot[k] = P->a_slot[k];
    A.qscale[k] = P->qscale[k];
  }
  A.wg_task = P->wg_task;
  A.n_buckets = (int32_t)P->buckets.size();
  for (size_t i = 0; i < P->buckets.size(); ++i) A.bk[i] = P->buckets[i];
  A.proj = P->proj;
  A.radius = (float)P->radius;
  A.neg_inv_gamma = (float)(-1.0 / gamma);
  A.gamma = (float)gamma;
  A.mu = mu;
  A.rfac = rfac;
  A.v_in = v_in;
  A.part = P->part;
  A.obj_part = obj_part;
  A.x_out = x_out;
  const size_t lds = dl_grad_lds_bytes(P, mode);
  if (P->mf == 1 && !P->has_a) return launch_storage<1, false, 16>(P, mode, A, lds);
  if (P->mf == 1) return launch_storage<1, true, 16>(P, mode, A, lds);
  return launch_storage<4, true, 8>(P, mode, A, lds);
}
