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
//    G = 2^glog lanes holding up to KMAX elements each in registers; G is a
//    compile-time constant per degree bucket so every load of a row uses an
//    immediate offset, and the arrays carry zero padding so loads past a row
//    end need no predication (masked by select); rows longer than 64*KMAX use
//    a wavefront-wide loop over the row;
//  * each wavefront prefetches the next task's row pointers and row data while
//    it computes the current task (software pipelining);
//  * the simplex threshold: the paper's early exit when the positive part
//    already fits, an exact exit when the largest entry leads the second by at
//    least z, otherwise Newton steps from below on f(theta) = sum max(v-theta,0)
//    - z (each step is the exact threshold of the current active set; the pass
//    that forms it also checks whether the set survives the step);
//  * a_k * x is rounded to a per-family fixed-point grid and added with 64-bit
//    integer LDS atomics into a per-workgroup histogram over items; integer
//    addition is associative, so the sums are bitwise reproducible for any
//    schedule and no float atomics are used; the histogram is written once per
//    workgroup and summed over workgroups by the update kernel.
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "dl_common.h"

// The kernel variants (dl_grad_variant.hip, one object per variant).
#define DL_GV_DECL(mf, a, bf)                                                                              \
  dl_status dl_grad_launch_v_##mf##_##a##_##bf(const dl_problem*, int, const dl_grad_args&, size_t);       \
  dl_status dl_grad_batch_v_##mf##_##a##_##bf(const dl_problem*, int, const dl_grad_args*, const dl_wg_desc*, \
                                              size_t, hipStream_t, int);                                    \
  void dl_grad_attr_v_##mf##_##a##_##bf();
DL_GV_DECL(1, 0, 0)
DL_GV_DECL(1, 0, 1)
DL_GV_DECL(1, 1, 0)
DL_GV_DECL(1, 1, 1)
DL_GV_DECL(2, 1, 0)
DL_GV_DECL(2, 1, 1)
DL_GV_DECL(4, 1, 0)
DL_GV_DECL(4, 1, 1)
#undef DL_GV_DECL

namespace {

// Fixed-point scale of each family for one histogram pass.  For every item j
// and user i, with a of any sign and lam of any sign:
//   v_ij = -(c_ij + sum_k a_kij mu_kj) / gamma
//        <= (max_i(-c_ij)^+ + sum_k max(-amin_kj mu_kj, -amax_kj mu_kj)) / gamma,
// and the FP32 value the pass forms differs from v_ij by at most
// (m + 2) 2^-24 (max|c_j| + sum_k max|a_kj| |mu_kj|) / gamma + 2^-24 |v| (one
// rounding per fused multiply-add, the sum and the scaling), so with the
// margin below x_ij <= min(z, max(0, v) + margin) (box, simplex <=; theta >= 0)
// or x_ij <= z (simplex =).  Hence |a_kij x_ij| <= B_k = max_j max|a_kj| xmax_j
// and the scale 2^(30 - ceil(log2 B_k)) keeps every addend below 2^31 (the
// relative roundings fit the factor-2 headroom above 2^30).  The grid is as
// fine as the pass allows and never coarser than for max|a_k| * radius.  One
// block of 1024 lanes; deterministic.
// The bound of item j: per family max|a_kj| xmax_j into bk[k], and xmax_j into bg
// (maxima over the items a thread has seen).
__device__ __forceinline__ void qscale_item(const dl_grad_args& A, int j, float mug, float (&bk)[DL_MAX_FAMILIES],
                                            float& bg) {
  const int J = A.J, m = A.m;
  const float ig = -A.neg_inv_gamma;
  const float z = A.radius;
  const bool eq = A.proj == DL_PROJ_SIMPLEX_EQ;
  const float ulp = 0x1p-24f * (float)(m + 5);
  const unsigned ec = A.ext[j];
  const float cneg = dl_ord_dec(ec), cabs = dl_ord_dec(A.ext[(size_t)J + j]);
  // the global-count dual shifts every v by -mu_g / gamma
  float t = cneg - mug, mag = cabs + fabsf(mug);
  float aab[DL_MAX_FAMILIES];
#pragma unroll
  for (int k = 0; k < DL_MAX_FAMILIES; ++k) {
    aab[k] = 0.f;
    if (k < m) {
      const int sl = A.a_slot[k];
      const float amx = sl >= 0 ? dl_ord_dec(A.ext[(size_t)(2 + 2 * sl) * J + j]) : 1.f;
      const float ang = sl >= 0 ? dl_ord_dec(A.ext[(size_t)(3 + 2 * sl) * J + j]) : -1.f;
      const float mu = A.mu[(size_t)k * J + j];
      t += mu >= 0.f ? ang * mu : amx * (-mu);
      aab[k] = fmaxf(fabsf(amx), fabsf(ang));
      mag += aab[k] * fabsf(mu);
    }
  }
  // the bound itself in FP32: its own roundings are covered by the margin
  const float v = t * ig;
  const float xm = eq ? z : fminf(z, fmaxf(0.f, v) + ulp * (mag * ig + fabsf(v)) * 2.f);
  const bool any = ec != DL_ORD_NEG_INF;  // some user is eligible for item j
#pragma unroll
  for (int k = 0; k < DL_MAX_FAMILIES; ++k)
    if (k < m && any) bk[k] = fmaxf(bk[k], aab[k] * xm);
  if (any) bg = fmaxf(bg, xm);
}

// The bounds of items [j0, j1) strided by the block, reduced over the block (every
// thread ends with the maxima).
__device__ void qscale_items(const dl_grad_args& A, int j0, int j1, float (&bk)[DL_MAX_FAMILIES], float& bg,
                             float* sh) {
#pragma unroll
  for (int k = 0; k < DL_MAX_FAMILIES; ++k) bk[k] = 0.f;
  bg = 0.f;  // global-count row: bound on x itself
  const float mug = A.glob ? A.mu[(size_t)A.m * A.J] : 0.f;
#pragma unroll 4
  for (int j = j0 + (int)threadIdx.x; j < j1; j += blockDim.x) qscale_item(A, j, mug, bk, bg);
  // block maxima (max is exact: the result does not depend on the split)
#pragma unroll
  for (int k = 0; k <= DL_MAX_FAMILIES; ++k) {
    float v = k < DL_MAX_FAMILIES ? bk[k] : bg;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s2 = blockDim.x / 2; s2 > 0; s2 >>= 1) {
      if ((int)threadIdx.x < s2) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s2]);
      __syncthreads();
    }
    v = sh[0];
    __syncthreads();
    if (k < DL_MAX_FAMILIES) bk[k] = v;
    else bg = v;
  }
}

// The scales from the pass-wide maxima (thread 0).
__device__ void qscale_finish(const dl_grad_args& A, const float (&bk)[DL_MAX_FAMILIES], float bg, float* out) {
  for (int k = 0; k < DL_MAX_FAMILIES && k < A.m; ++k) {
    const float B = bk[k] * (1.0f + 0x1p-16f);
    float qv = B > 0.f ? ldexpf(1.f, 30 - (int)ceilf(log2f(B))) : 0x1p60f;
    qv = fminf(fmaxf(qv, A.qscale[k]), 0x1p60f);
    out[k] = qv;
  }
  if (A.glob) {
    // |x| <= B_g per element: each addend below 2^31 on the grid 2^(30 - ceil log2 B_g),
    // never coarser than for x <= radius; n_nonzeros * 2^31 < 2^63 bounds the sum
    const float B = bg * (1.0f + 0x1p-16f);
    const float coarse = ldexpf(1.f, 30 - (int)ceilf(log2f(fmaxf(A.radius, 0x1p-30f))));
    float qv = B > 0.f ? ldexpf(1.f, 30 - (int)ceilf(log2f(B))) : 0x1p60f;
    out[DL_MAX_FAMILIES] = fminf(fmaxf(qv, coarse), 0x1p60f);
  }
}

// One block over every item (the batched form runs one such block per member).
__device__ void qscale_body(const dl_grad_args& A, float* out) {
  __shared__ float sh[1024];
  float bk[DL_MAX_FAMILIES], bg;
  qscale_items(A, 0, A.J, bk, bg, sh);
  if (threadIdx.x == 0) qscale_finish(A, bk, bg, out);
}

// Many blocks, one item per thread: each wavefront reduces its lanes' bounds with
// shuffles and folds them into five device words with integer atomic max (the
// bounds are >= 0, so their bit patterns order like the values); the last
// wavefront to arrive (an arrival counter) reads the words, writes the scales
// and clears the words and the counter for the next launch.  No wavefront waits.
constexpr int DL_QS_ITEMS = 256;
constexpr int DL_QS_VALS = DL_MAX_FAMILIES + 1;
__global__ void __launch_bounds__(DL_QS_ITEMS) qscale_multi(dl_grad_args A, float* out, unsigned* words,
                                                            unsigned* cnt) {
  float bk[DL_MAX_FAMILIES] = {0.f, 0.f, 0.f, 0.f};
  float bg = 0.f;
  const int j = (int)(blockIdx.x * DL_QS_ITEMS + threadIdx.x);
  if (j < A.J) qscale_item(A, j, A.glob ? A.mu[(size_t)A.m * A.J] : 0.f, bk, bg);
  float v[DL_QS_VALS] = {bk[0], bk[1], bk[2], bk[3], bg};
#pragma unroll
  for (int k = 0; k < DL_QS_VALS; ++k)
    for (int o = 32; o > 0; o >>= 1) v[k] = fmaxf(v[k], __shfl_xor(v[k], o, 64));
  if ((threadIdx.x & 63) != 0) return;
#pragma unroll
  for (int k = 0; k < DL_QS_VALS; ++k)
    if (v[k] > 0.f) atomicMax(words + k, __float_as_uint(v[k]));
  __threadfence();  // the maxima before the arrival
  const unsigned waves = gridDim.x * (DL_QS_ITEMS / 64);
  if (atomicAdd(cnt, 1u) != waves - 1) return;
  __threadfence();
#pragma unroll
  for (int k = 0; k < DL_QS_VALS; ++k) v[k] = __uint_as_float(atomicExch(words + k, 0u));
  const float fb[DL_MAX_FAMILIES] = {v[0], v[1], v[2], v[3]};
  qscale_finish(A, fb, v[4], out);
  atomicExch(cnt, 0u);  // ready for the next launch
}

__global__ void __launch_bounds__(1024) qscale_kernel(dl_grad_args A, float* out) { qscale_body(A, out); }

__global__ void __launch_bounds__(1024) qscale_batch_kernel(const dl_grad_args* __restrict__ args) {
  const dl_grad_args& A = args[blockIdx.x];
  if (A.qs_dev == nullptr || A.ext == nullptr) return;  // not a live instance
  qscale_body(A, const_cast<float*>(A.qs_dev));
}

}  // namespace

dl_status dl_launch_qscale(const dl_problem* P, const float* mu, double gamma) {
  dl_grad_args A = dl_make_grad_args(P, mu, gamma);
  const int nb = (P->J + DL_QS_ITEMS - 1) / DL_QS_ITEMS;
  if (nb <= 1) {
    hipLaunchKernelGGL(qscale_kernel, dim3(1), dim3(1024), 0, P->stream, A, P->qs_dev);
  } else {
    hipLaunchKernelGGL(qscale_multi, dim3(nb), dim3(DL_QS_ITEMS), 0, P->stream, A, P->qs_dev, P->qs_words,
                       P->qs_cnt);
  }
  DL_HIP_TRY(hipGetLastError());
  return DL_OK;
}

dl_status dl_launch_qscale_batch(const dl_grad_args* d_args, int n, hipStream_t st) {
  if (n <= 0) return DL_OK;
  hipLaunchKernelGGL(qscale_batch_kernel, dim3(n), dim3(1024), 0, st, d_args);
  DL_HIP_TRY(hipGetLastError());
  return DL_OK;
}

size_t dl_grad_lds_bytes(const dl_problem* P, int mode) {
  const size_t mJ = (size_t)P->m * P->J;
  size_t mu_n = (mode & M_VIN) ? 0 : (size_t)P->nrow();
  size_t rf_n = (mode & M_REPAIR) ? (size_t)P->J : 0;
  size_t off = ((mu_n + rf_n) * 4 + 15) & ~(size_t)15;
  size_t hist = (mode & M_HIST) ? (P->tile_rows > 0 ? (size_t)P->tile_rows : mJ) * 8 : 0;
  // per-wavefront objective sums, then per-wavefront global counts
  return off + hist + DL_WAVES * sizeof(double) + DL_WAVES * sizeof(unsigned long long);
}

dl_status dl_grad_prepare(const dl_problem* P) {
  if (P->mf == 1 && !P->has_a) {
    dl_grad_attr_v_1_0_0();
    dl_grad_attr_v_1_0_1();
  } else if (P->mf == 1) {
    dl_grad_attr_v_1_1_0();
    dl_grad_attr_v_1_1_1();
  } else if (P->mf == 2) {
    dl_grad_attr_v_2_1_0();
    dl_grad_attr_v_2_1_1();
  } else {
    dl_grad_attr_v_4_1_0();
    dl_grad_attr_v_4_1_1();
  }
  return DL_OK;
}

dl_status dl_launch_grad_batch(const dl_problem* P, int n_wg, const dl_grad_args* d_args, const dl_wg_desc* d_wgs,
                               size_t lds, hipStream_t st, int mode) {
  if (n_wg <= 0) return DL_OK;
  const bool bf = P->storage == DL_BF16;
  if (P->mf == 1 && !P->has_a)
    return bf ? dl_grad_batch_v_1_0_1(P, n_wg, d_args, d_wgs, lds, st, mode)
              : dl_grad_batch_v_1_0_0(P, n_wg, d_args, d_wgs, lds, st, mode);
  if (P->mf == 1)
    return bf ? dl_grad_batch_v_1_1_1(P, n_wg, d_args, d_wgs, lds, st, mode)
              : dl_grad_batch_v_1_1_0(P, n_wg, d_args, d_wgs, lds, st, mode);
  if (P->mf == 2)
    return bf ? dl_grad_batch_v_2_1_1(P, n_wg, d_args, d_wgs, lds, st, mode)
              : dl_grad_batch_v_2_1_0(P, n_wg, d_args, d_wgs, lds, st, mode);
  return bf ? dl_grad_batch_v_4_1_1(P, n_wg, d_args, d_wgs, lds, st, mode)
            : dl_grad_batch_v_4_1_0(P, n_wg, d_args, d_wgs, lds, st, mode);
}

dl_grad_args dl_make_grad_args(const dl_problem* P, const float* mu, double gamma) {
  dl_grad_args A;
  memset(&A, 0, sizeof(A));
  A.rp = P->rp;
  A.idx = P->idx;
  A.cval = P->cval;
  A.aval = P->aval;
  A.orig_rp = P->orig_rp;
  A.nnz = P->nnz;
  A.astride = dl_astride(P->nnz);
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
  A.upper = (float)P->upper;
  A.neg_inv_gamma = (float)(-1.0 / gamma);
  A.gamma = (float)gamma;
  A.glob = P->glob;
  A.mu = mu;
  A.qs_dev = P->qs_dev;
  A.ext = P->ext;
  A.part = P->part;
  A.wg_clock = P->clocking ? P->wg_clock : nullptr;
  return A;
}

dl_status dl_launch_grad(const dl_problem* P, int mode, const float* mu, double gamma, const float* rfac,
                         const float* v_in, float* x_out, double* obj_part, bool scaled) {
  if (P->n_wg <= 0) return DL_OK;
  if (x_out) mode |= M_XOUT;
  if (P->glob && (mode & M_HIST)) mode |= M_GLOB;
  if ((mode & M_HIST) && !scaled) DL_TRY(dl_launch_qscale(P, mu, gamma));
  dl_grad_args A = dl_make_grad_args(P, mu, gamma);
  A.rfac = rfac;
  A.v_in = v_in;
  A.obj_part = obj_part;
  A.x_out = x_out;
  const size_t lds = dl_grad_lds_bytes(P, mode);
  const bool bf = P->storage == DL_BF16;
  if (P->mf == 1 && !P->has_a)
    return bf ? dl_grad_launch_v_1_0_1(P, mode, A, lds) : dl_grad_launch_v_1_0_0(P, mode, A, lds);
  if (P->mf == 1) return bf ? dl_grad_launch_v_1_1_1(P, mode, A, lds) : dl_grad_launch_v_1_1_0(P, mode, A, lds);
  auto launch_multi = [&](int md) -> dl_status {
    if (P->mf == 2) return bf ? dl_grad_launch_v_2_1_1(P, md, A, lds) : dl_grad_launch_v_2_1_0(P, md, A, lds);
    return bf ? dl_grad_launch_v_4_1_1(P, md, A, lds) : dl_grad_launch_v_4_1_0(P, md, A, lds);
  };
  if (!(mode & M_HIST) || P->tile_rows == 0) return launch_multi(mode);
  // row windows: one launch each; the first also writes x, the objective and the
  // global count (every launch computes the same x)
  const int64_t mJ = (int64_t)P->m * P->J;
  for (int t = 0; t < P->n_tiles; ++t) {
    const int64_t r0 = (int64_t)t * P->tile_rows;
    const int64_t n = std::min<int64_t>(P->tile_rows, mJ - r0);
    A.tile_b0 = (int32_t)(8 * r0);
    A.tile_bn = (int32_t)(8 * n);
    const int mt = (t == 0) ? (mode | M_TILE) : ((mode & ~(M_OBJ | M_XOUT | M_GLOB)) | M_TILE);
    DL_TRY(launch_multi(mt));
  }
  return DL_OK;
}
