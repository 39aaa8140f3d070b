// Learned warm start: per-item features and a small MLP (16 -> H -> H -> 1,
// ReLU) trained and evaluated with BF16 matrix-core (MFMA) GEMMs and FP32
// accumulation.  Not part of the paper's method: it predicts a day's duals
// from item features and the previous day's duals, for recurring solves on
// slowly drifting inputs; the cold-start solve stays the judge and fallback.
//
// GEMM: 64x64 output tile per 256-lane workgroup, each wavefront a 32x32
// block of four 16x16 v_mfma_f32_16x16x16_bf16 tiles, K in steps of 16 staged
// through LDS (A as [m][k], B as [n][k] so each lane's 4-element operand is
// one 8-byte LDS read).  Long reductions (weight gradients, K = batch rows)
// split K over a grid dimension into FP32 partial tiles that a second kernel
// sums in fixed order: no float atomics, bitwise reproducible.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "dl_common.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int GT = 64;   // output tile
constexpr int GK = 16;   // K step
constexpr int LDK = GK + 4;

// Cp[z][M x N] = sum over k in slice z of A(m, k) B(k, n); A(m,k) = TA ? A[k*lda+m] : A[m*lda+k],
// B(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n].
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_bf16(const uint16_t* __restrict__ A, int lda,
                                                 const uint16_t* __restrict__ B, int ldb, float* __restrict__ Cp,
                                                 int M, int N, int K, int kslice) {
  __shared__ __align__(16) uint16_t As[GT][LDK];
  __shared__ __align__(16) uint16_t Bs[GT][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT, z = blockIdx.z;
  const int kb = z * kslice, ke = min(K, kb + kslice);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += GK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int id = tid * 4 + q;
      const int rl = id / GK, kl = id % GK;
      const int k = k0 + kl;
      const int m = m0 + rl, n = n0 + rl;
      uint16_t av = 0, bv = 0;
      if (m < M && k < ke) av = TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
      if (n < N && k < ke) bv = TB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
      As[rl][kl] = av;
      Bs[rl][kl] = bv;
    }
    __syncthreads();
    bf16x4 a[2], b[2];
    const int kq = 4 * (lane >> 4);
    for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x4*>(&As[wm + i * 16 + (lane & 15)][kq]);
    for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x4*>(&Bs[wn + j * 16 + (lane & 15)][kq]);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  float* Cz = Cp + (size_t)z * M * N;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int q = 0; q < 4; ++q) {
        // lane holds rows 4*(lane/16)+q, column lane%16 of each 16x16 tile
        const int r = m0 + wm + i * 16 + 4 * (lane >> 4) + q;
        const int c = n0 + wn + j * 16 + (lane & 15);
        if (r < M && c < N) Cz[(size_t)r * N + c] = acc[i][j][q];
      }
}

// out = sum_z Cp[z] (+ bias[c]) -> optional ReLU -> optional mask (m > 0) ->
// FP32 and / or BF16 copies; ncol columns of the M x N product are kept.
__global__ void gemm_epilogue(const float* __restrict__ Cp, int nz, int M, int N, int ncol,
                              const float* __restrict__ bias, int relu, const uint16_t* __restrict__ mask,
                              float* __restrict__ out32, uint16_t* __restrict__ out16) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)M * ncol) return;
  const int r = (int)(id / ncol), c = (int)(id % ncol);
  float s = 0.f;
  for (int z = 0; z < nz; ++z) s += Cp[(size_t)z * M * N + (size_t)r * N + c];
  if (bias) s += bias[c];
  if (relu) s = fmaxf(s, 0.f);
  if (mask && !(bf2f(mask[id]) > 0.f)) s = 0.f;
  if (out32) out32[id] = s;
  if (out16) out16[id] = dl_f32_to_bf16_rne(s);
}

__global__ void to_bf16(const float* __restrict__ in, int64_t n, uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = dl_f32_to_bf16_rne(in[i]);
}

// Network input: column k of X becomes (x - shift[k]) * scale[k], rounded once to BF16.
__global__ void input_to_bf16(const float* __restrict__ X, int64_t n16, const float* __restrict__ norm,
                              uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n16) return;
  const int k = (int)(i & 15);
  const float v = (X[i] - norm[k]) * norm[16 + k];
  out[i] = dl_f32_to_bf16_rne(v);
}

// Predicted duals: lam0 = max(0, lam_prev + s y), with a non-finite y giving
// lam_prev (the prediction then falls back to the previous day's value).
__global__ void predict_duals(const float* __restrict__ y, const double* __restrict__ lam_prev, int64_t n, double s,
                              double* __restrict__ lam0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double yi = (double)y[i];
  const double v = isfinite(yi) ? lam_prev[i] + s * yi : lam_prev[i];
  lam0[i] = fmax(v, 0.0);
}

// W3 (H) as an H x 16 BF16 matrix with the weights in column 0.
__global__ void pack_w3(const float* __restrict__ w3, int H, uint16_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < H * 16) out[i] = (i % 16 == 0) ? dl_f32_to_bf16_rne(w3[i / 16]) : (uint16_t)0;
}

// dz2 = dy * w3 (BF16 weight values) masked by h2 > 0, FP32 and BF16.
__global__ void dh2_kernel(const float* __restrict__ dy, const uint16_t* __restrict__ w3b, const uint16_t* __restrict__ h2,
                           int64_t n, int H, float* __restrict__ out32, uint16_t* __restrict__ out16) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * H) return;
  const int c = (int)(id % H);
  float v = (bf2f(h2[id]) > 0.f) ? dy[id / H] * bf2f(w3b[c * 16]) : 0.f;
  out32[id] = v;
  out16[id] = dl_f32_to_bf16_rne(v);
}

// Column sums of an n x H FP32 matrix in fixed order (one thread per column,
// rows split into 64 fixed slices summed in slice order).
__global__ void colsum_partial(const float* __restrict__ X, int64_t n, int H, float* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (c >= H) return;
  const int64_t r0 = n * s / gridDim.y, r1 = n * (s + 1) / gridDim.y;
  float acc = 0.f;
  for (int64_t r = r0; r < r1; ++r) acc += X[r * H + c];
  part[(size_t)s * H + c] = acc;
}
__global__ void colsum_final(const float* __restrict__ part, int ns, int H, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= H) return;
  float acc = 0.f;
  for (int s = 0; s < ns; ++s) acc += part[(size_t)s * H + c];
  out[c] = acc;
}

// MSE: dy = (y - t) / n; loss = sum (y - t)^2 / (2n) (fixed-order block reduction).
__global__ void mse_kernel(const float* __restrict__ y, const float* __restrict__ t, int64_t n, float* __restrict__ dy,
                           double* __restrict__ loss) {
  __shared__ double sh[1024];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float r = y[i] - t[i];
    dy[i] = r / (float)n;
    acc += (double)r * r;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sh[0] / (2.0 * (double)(n > 0 ? n : 1));
}

__global__ void add_bias_col0(const float* __restrict__ in, int64_t n, int ld, const float* __restrict__ b,
                              float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = in[i * ld] + b[0];
}

// AdamW on the flat FP32 master parameters; decay on [0, nd) (the weight matrices).
__global__ void adamw_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                             float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float wd,
                             float bc1, float bc2, const unsigned char* __restrict__ decay) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1, vh = vi / bc2;
  p[i] -= lr * (mh / (sqrtf(vh) + eps) + (decay[i] ? wd * p[i] : 0.f));
}

inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// Item features
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned ord_bits(float f) {
  const unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_ord(unsigned o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

template <typename TV>
__device__ inline float ldc(const void* p, int64_t e);
template <>
__device__ inline float ldc<float>(const void* p, int64_t e) { return reinterpret_cast<const float*>(p)[e]; }
template <>
__device__ inline float ldc<uint16_t>(const void* p, int64_t e) {
  return __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(p)[e] << 16);
}

// Per item: count, max |c|, max c, min c (integer atomics: order-free).
template <typename TV>
__global__ void feat_pass1(const uint16_t* __restrict__ idx, const void* __restrict__ cval, int64_t nnz,
                           unsigned long long* __restrict__ cnt, unsigned* __restrict__ amax,
                           unsigned* __restrict__ mx, unsigned* __restrict__ mn) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int j = idx[e] >> 2;  // the problem stores item byte offsets (4 j)
    const float c = ldc<TV>(cval, e);
    atomicAdd(cnt + j, 1ull);
    atomicMax(amax, __float_as_uint(fabsf(c)));
    atomicMax(mx + j, ord_bits(c));
    atomicMin(mn + j, ord_bits(c));
  }
}

// Per item: sum c and sum c^2 on fixed-point grids (exact integer sums).
template <typename TV>
__global__ void feat_pass2(const uint16_t* __restrict__ idx, const void* __restrict__ cval, int64_t nnz, double s1,
                           double s2, unsigned long long* __restrict__ q1, unsigned long long* __restrict__ q2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int j = idx[e] >> 2;  // the problem stores item byte offsets (4 j)
    const double c = (double)ldc<TV>(cval, e);
    atomicAdd(q1 + j, (unsigned long long)__double2ll_rn(c * s1));
    atomicAdd(q2 + j, (unsigned long long)__double2ll_rn(c * c * s2));
  }
}

__global__ void feat_final(int J, const unsigned long long* __restrict__ cnt, const unsigned long long* __restrict__ q1,
                           const unsigned long long* __restrict__ q2, const unsigned* __restrict__ mx,
                           const unsigned* __restrict__ mn, double s1, double s2, double mean_n,
                           const double* __restrict__ b, const double* __restrict__ b_prev,
                           const double* __restrict__ lam_prev, const double* __restrict__ g_prev,
                           float* __restrict__ F) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  const double n = (double)cnt[j];
  const double nn = n > 0 ? n : 1.0;
  const double mean = (double)(long long)q1[j] / s1 / nn;
  const double var = fmax((double)(long long)q2[j] / s2 / nn - mean * mean, 0.0);
  const bool has = n > 0;
  const double lp = lam_prev[j];
  const double bp = b_prev[j];
  float* f = F + (size_t)j * 16;
  f[0] = (float)(b[j] / nn);
  f[1] = (float)(log1p(n) / 10.0);
  f[2] = has ? (float)mean : 0.f;
  f[3] = has ? (float)sqrt(var) : 0.f;
  f[4] = has ? from_ord(mx[j]) : 0.f;
  f[5] = has ? from_ord(mn[j]) : 0.f;
  f[6] = (float)lp;
  f[7] = lp > 0.0 ? 1.f : 0.f;
  f[8] = (float)(bp / nn);
  f[9] = (float)fmin(1.0, fmax(-1.0, g_prev[j] / fmax(bp, 1e-12)));
  f[10] = (float)(10.0 * (b[j] / fmax(bp, 1e-12) - 1.0));
  f[11] = (float)(n / fmax(mean_n, 1e-12));
  for (int k = 12; k < 16; ++k) f[k] = 0.f;
}

}  // namespace

// ---------------------------------------------------------------------------
// MLP object
// ---------------------------------------------------------------------------
struct dl_mlp {
  int n_in = 16, H = 256;
  int64_t max_batch = 0;
  hipStream_t stream = nullptr;
  int64_t n_params = 0;
  int64_t off_W1 = 0, off_b1 = 0, off_W2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0;
  float *P = nullptr, *G = nullptr, *Mo = nullptr, *Vo = nullptr;
  unsigned char* decay = nullptr;
  uint16_t *W1b = nullptr, *W2b = nullptr, *W3b = nullptr;
  uint16_t *Xb = nullptr, *H1b = nullptr, *H2b = nullptr, *dH2b = nullptr, *dH1b = nullptr, *dyb = nullptr;
  float *dH2 = nullptr, *dH1 = nullptr, *y = nullptr, *dy = nullptr, *Cp = nullptr, *colpart = nullptr, *tmp = nullptr;
  float* norm = nullptr;  // [16 shifts, 16 scales] of the network input
  size_t cp_cap = 0;
  double* loss_dev = nullptr;
  double* loss_host = nullptr;
  int64_t step = 0;
};

namespace {

void free_mlp(dl_mlp* N) {
  if (!N) return;
  void* ptrs[] = {N->P, N->G, N->Mo, N->Vo, N->decay, N->W1b, N->W2b, N->W3b, N->Xb, N->H1b, N->H2b, N->dH2b,
                  N->dH1b, N->dyb, N->dH2, N->dH1, N->y, N->dy, N->Cp, N->colpart, N->tmp, N->loss_dev, N->norm};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (N->loss_host) (void)hipHostFree(N->loss_host);
  delete N;
}

template <typename T>
hipError_t dal(T** p, size_t n) {
  return hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T));
}

// C(ncol kept columns) = A(M x K) B(K x N); kslice = K (one slice) or the split.
dl_status gemm(dl_mlp* N, bool ta, bool tb, const uint16_t* A, int lda, const uint16_t* B, int ldb, int M, int Ncols,
               int K, int ncol, const float* bias, int relu, const uint16_t* mask, float* out32, uint16_t* out16,
               int kslice) {
  if (M <= 0 || Ncols <= 0) return DL_OK;
  if (kslice <= 0 || kslice > K) kslice = std::max(K, 1);
  kslice = (kslice + GK - 1) / GK * GK;
  const int nz = std::max(1, (K + kslice - 1) / kslice);
  if ((size_t)nz * M * Ncols > N->cp_cap) {
    dl_set_error("internal: GEMM partial buffer too small");
    return DL_EINVAL;
  }
  dim3 grid((unsigned)((Ncols + GT - 1) / GT), (unsigned)((M + GT - 1) / GT), (unsigned)nz);
  if (ta && tb)
    hipLaunchKernelGGL((gemm_bf16<true, true>), grid, dim3(256), 0, N->stream, A, lda, B, ldb, N->Cp, M, Ncols, K, kslice);
  else if (ta)
    hipLaunchKernelGGL((gemm_bf16<true, false>), grid, dim3(256), 0, N->stream, A, lda, B, ldb, N->Cp, M, Ncols, K, kslice);
  else if (tb)
    hipLaunchKernelGGL((gemm_bf16<false, true>), grid, dim3(256), 0, N->stream, A, lda, B, ldb, N->Cp, M, Ncols, K, kslice);
  else
    hipLaunchKernelGGL((gemm_bf16<false, false>), grid, dim3(256), 0, N->stream, A, lda, B, ldb, N->Cp, M, Ncols, K, kslice);
  DL_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(gemm_epilogue, dim3(nblk((int64_t)M * ncol)), dim3(256), 0, N->stream, N->Cp, nz, M, Ncols, ncol,
                     bias, relu, mask, out32, out16);
  DL_HIP_TRY(hipGetLastError());
  return DL_OK;
}

dl_status refresh_bf16(dl_mlp* N) {
  hipLaunchKernelGGL(to_bf16, dim3(nblk((int64_t)N->n_in * N->H)), dim3(256), 0, N->stream, N->P + N->off_W1,
                     (int64_t)N->n_in * N->H, N->W1b);
  hipLaunchKernelGGL(to_bf16, dim3(nblk((int64_t)N->H * N->H)), dim3(256), 0, N->stream, N->P + N->off_W2,
                     (int64_t)N->H * N->H, N->W2b);
  hipLaunchKernelGGL(pack_w3, dim3(nblk((int64_t)N->H * 16)), dim3(256), 0, N->stream, N->P + N->off_w3, N->H,
                     N->W3b);
  DL_HIP_TRY(hipGetLastError());
  return DL_OK;
}

dl_status forward_impl(dl_mlp* N, const float* X, int64_t n) {
  const int H = N->H;
  hipLaunchKernelGGL(input_to_bf16, dim3(nblk(n * 16)), dim3(256), 0, N->stream, X, n * 16, N->norm, N->Xb);
  DL_HIP_TRY(hipGetLastError());
  DL_TRY(gemm(N, false, false, N->Xb, 16, N->W1b, H, (int)n, H, 16, H, N->P + N->off_b1, 1, nullptr, nullptr, N->H1b,
              16));
  DL_TRY(gemm(N, false, false, N->H1b, H, N->W2b, H, (int)n, H, H, H, N->P + N->off_b2, 1, nullptr, nullptr, N->H2b,
              H));
  DL_TRY(gemm(N, false, false, N->H2b, H, N->W3b, 16, (int)n, 16, H, 16, nullptr, 0, nullptr, N->tmp, nullptr, H));
  hipLaunchKernelGGL(add_bias_col0, dim3(nblk(n)), dim3(256), 0, N->stream, N->tmp, n, 16, N->P + N->off_b3, N->y);
  DL_HIP_TRY(hipGetLastError());
  return DL_OK;
}

// Gradient of sum_i dy_i y_i into N->G (forward_impl must have run on the same
// rows and N->dy must hold dy).
dl_status backward_impl(dl_mlp* N, int64_t n) {
  const int H = N->H;
  const int ks = 512;  // split of the batch dimension for the weight gradients
  const int ns = (int)std::min<int64_t>(64, std::max<int64_t>(1, n));
  float* G = N->G;
  // output layer: dW3 = H2^T dy, db3 = sum dy
  hipLaunchKernelGGL(to_bf16, dim3(nblk(n)), dim3(256), 0, N->stream, N->dy, n, N->dyb);
  DL_HIP_TRY(hipGetLastError());
  DL_TRY(gemm(N, true, false, N->H2b, H, N->dyb, 1, H, 1, (int)n, 1, nullptr, 0, nullptr, G + N->off_w3, nullptr, ks));
  hipLaunchKernelGGL(colsum_partial, dim3(1, ns), dim3(64), 0, N->stream, N->dy, n, 1, N->colpart);
  hipLaunchKernelGGL(colsum_final, dim3(1), dim3(64), 0, N->stream, N->colpart, ns, 1, G + N->off_b3);
  // second layer: dz2 = dy w3 [h2 > 0]; dW2 = H1^T dz2; db2 = colsum dz2
  hipLaunchKernelGGL(dh2_kernel, dim3(nblk(n * H)), dim3(256), 0, N->stream, N->dy, N->W3b, N->H2b, n, H, N->dH2,
                     N->dH2b);
  DL_HIP_TRY(hipGetLastError());
  DL_TRY(gemm(N, true, false, N->H1b, H, N->dH2b, H, H, H, (int)n, H, nullptr, 0, nullptr, G + N->off_W2, nullptr, ks));
  hipLaunchKernelGGL(colsum_partial, dim3(nblk(H, 64), ns), dim3(64), 0, N->stream, N->dH2, n, H, N->colpart);
  hipLaunchKernelGGL(colsum_final, dim3(nblk(H, 64)), dim3(64), 0, N->stream, N->colpart, ns, H, G + N->off_b2);
  // first layer: dz1 = (dz2 W2^T) [h1 > 0]; dW1 = X^T dz1; db1 = colsum dz1
  DL_TRY(gemm(N, false, true, N->dH2b, H, N->W2b, H, (int)n, H, H, H, nullptr, 0, N->H1b, N->dH1, N->dH1b, H));
  DL_TRY(gemm(N, true, false, N->Xb, 16, N->dH1b, H, 16, H, (int)n, H, nullptr, 0, nullptr, G + N->off_W1, nullptr, ks));
  hipLaunchKernelGGL(colsum_partial, dim3(nblk(H, 64), ns), dim3(64), 0, N->stream, N->dH1, n, H, N->colpart);
  hipLaunchKernelGGL(colsum_final, dim3(nblk(H, 64)), dim3(64), 0, N->stream, N->colpart, ns, H, G + N->off_b1);
  DL_HIP_TRY(hipGetLastError());
  return DL_OK;
}

}  // namespace

extern "C" dl_status dl_mlp_create(const dl_mlp_desc* d, dl_mlp** out) {
  DL_CHECK_ARG(out, "out is NULL");
  *out = nullptr;
  DL_CHECK_ARG(d, "desc is NULL");
  DL_CHECK_ARG(d->n_in == 16, "n_in must be 16 (features are zero-padded to 16)");
  DL_CHECK_ARG(d->hidden >= 64 && d->hidden <= 1024 && d->hidden % 64 == 0, "hidden must be a multiple of 64 in [64, 1024]");
  DL_CHECK_ARG(d->max_batch >= 1 && d->max_batch <= (1 << 24), "max_batch must be in [1, 2^24]");
  dl_mlp* N = new (std::nothrow) dl_mlp();
  if (!N) {
    dl_set_error("host allocation failed");
    return DL_ENOMEM;
  }
  N->n_in = d->n_in;
  N->H = d->hidden;
  N->max_batch = d->max_batch;
  N->stream = (hipStream_t)d->stream;
  const int64_t H = N->H, n = N->max_batch;
  N->off_W1 = 0;
  N->off_b1 = N->off_W1 + 16 * H;
  N->off_W2 = N->off_b1 + H;
  N->off_b2 = N->off_W2 + H * H;
  N->off_w3 = N->off_b2 + H;
  N->off_b3 = N->off_w3 + H;
  N->n_params = N->off_b3 + 1;
  const int64_t nz = (n + 511) / 512;
  N->cp_cap = (size_t)std::max<int64_t>(n * H, nz * H * H);
  bool ok = dal(&N->P, N->n_params) == hipSuccess && dal(&N->G, N->n_params) == hipSuccess &&
            dal(&N->Mo, N->n_params) == hipSuccess && dal(&N->Vo, N->n_params) == hipSuccess &&
            dal(&N->decay, N->n_params) == hipSuccess && dal(&N->W1b, 16 * H) == hipSuccess &&
            dal(&N->W2b, H * H) == hipSuccess && dal(&N->W3b, H * 16) == hipSuccess &&
            dal(&N->Xb, n * 16) == hipSuccess && dal(&N->H1b, n * H) == hipSuccess &&
            dal(&N->H2b, n * H) == hipSuccess && dal(&N->dH2b, n * H) == hipSuccess &&
            dal(&N->dH1b, n * H) == hipSuccess && dal(&N->dyb, n) == hipSuccess &&
            dal(&N->dH2, n * H) == hipSuccess && dal(&N->dH1, n * H) == hipSuccess && dal(&N->y, n) == hipSuccess &&
            dal(&N->dy, n) == hipSuccess && dal(&N->Cp, N->cp_cap) == hipSuccess &&
            dal(&N->colpart, 64 * H) == hipSuccess && dal(&N->tmp, n * 16) == hipSuccess &&
            dal(&N->loss_dev, 1) == hipSuccess && dal(&N->norm, 32) == hipSuccess && hipHostMalloc((void**)&N->loss_host, sizeof(double)) == hipSuccess;
  if (!ok) {
    free_mlp(N);
    dl_set_error("device allocation failed");
    return DL_ENOMEM;
  }
  std::vector<unsigned char> dec((size_t)N->n_params, 0);
  for (int64_t i = N->off_W1; i < N->off_b1; ++i) dec[(size_t)i] = 1;
  for (int64_t i = N->off_W2; i < N->off_b2; ++i) dec[(size_t)i] = 1;
  for (int64_t i = N->off_w3; i < N->off_b3; ++i) dec[(size_t)i] = 1;
  hipStream_t st = N->stream;
  const float norm0[32] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                           1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f};
  if (hipMemcpyAsync(N->decay, dec.data(), dec.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(N->norm, norm0, sizeof(norm0), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemsetAsync(N->P, 0, sizeof(float) * N->n_params, st) != hipSuccess ||
      hipMemsetAsync(N->Mo, 0, sizeof(float) * N->n_params, st) != hipSuccess ||
      hipMemsetAsync(N->Vo, 0, sizeof(float) * N->n_params, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    free_mlp(N);
    dl_set_error("initialising the MLP failed");
    return DL_EHIP;
  }
  dl_status rs = refresh_bf16(N);
  if (rs != DL_OK) {
    free_mlp(N);
    return rs;
  }
  *out = N;
  return DL_OK;
}

extern "C" void dl_mlp_destroy(dl_mlp* N) { free_mlp(N); }

extern "C" int64_t dl_mlp_num_params(const dl_mlp* N) { return N ? N->n_params : 0; }

extern "C" dl_status dl_mlp_set_params(dl_mlp* N, const float* host) {
  DL_CHECK_ARG(N && host, "NULL argument");
  DL_HIP_TRY(hipMemcpyAsync(N->P, host, sizeof(float) * N->n_params, hipMemcpyHostToDevice, N->stream));
  DL_HIP_TRY(hipMemsetAsync(N->Mo, 0, sizeof(float) * N->n_params, N->stream));
  DL_HIP_TRY(hipMemsetAsync(N->Vo, 0, sizeof(float) * N->n_params, N->stream));
  N->step = 0;
  DL_TRY(refresh_bf16(N));
  DL_HIP_TRY(hipStreamSynchronize(N->stream));
  return DL_OK;
}

extern "C" dl_status dl_mlp_get_params(dl_mlp* N, float* host) {
  DL_CHECK_ARG(N && host, "NULL argument");
  DL_HIP_TRY(hipMemcpyAsync(host, N->P, sizeof(float) * N->n_params, hipMemcpyDeviceToHost, N->stream));
  DL_HIP_TRY(hipStreamSynchronize(N->stream));
  return DL_OK;
}

extern "C" dl_status dl_mlp_set_input_norm(dl_mlp* N, const float* shift, const float* scale) {
  DL_CHECK_ARG(N && shift && scale, "NULL argument");
  float h[32];
  for (int k = 0; k < 16; ++k) {
    DL_CHECK_ARG(isfinite(shift[k]) && isfinite(scale[k]), "non-finite input normalisation");
    h[k] = shift[k];
    h[16 + k] = scale[k];
  }
  DL_HIP_TRY(hipMemcpyAsync(N->norm, h, sizeof(h), hipMemcpyHostToDevice, N->stream));
  DL_HIP_TRY(hipStreamSynchronize(N->stream));
  return DL_OK;
}

extern "C" dl_status dl_mlp_predict_duals(dl_mlp* N, const float* X, int64_t n, const double* lam_prev, double s,
                                          double* lam0) {
  DL_CHECK_ARG(N && (n == 0 || (X && lam_prev && lam0)), "NULL argument");
  DL_CHECK_ARG(n >= 0 && n <= N->max_batch, "n exceeds max_batch");
  DL_CHECK_ARG(isfinite(s), "non-finite scale");
  if (n == 0) return DL_OK;
  DL_TRY(forward_impl(N, X, n));
  hipLaunchKernelGGL(predict_duals, dim3(nblk(n)), dim3(256), 0, N->stream, N->y, lam_prev, n, s, lam0);
  DL_HIP_TRY(hipGetLastError());
  return DL_OK;
}

extern "C" dl_status dl_mlp_forward(dl_mlp* N, const float* X, int64_t n, float* y) {
  DL_CHECK_ARG(N && (n == 0 || (X && y)), "NULL argument");
  DL_CHECK_ARG(n >= 0 && n <= N->max_batch, "n exceeds max_batch");
  if (n == 0) return DL_OK;
  DL_TRY(forward_impl(N, X, n));
  DL_HIP_TRY(hipMemcpyAsync(y, N->y, sizeof(float) * n, hipMemcpyDeviceToDevice, N->stream));
  return DL_OK;
}

extern "C" dl_status dl_mlp_gradients(dl_mlp* N, const float* X, const float* dy, int64_t n, float* y, float* grad) {
  DL_CHECK_ARG(N && X && dy && grad, "NULL argument");
  DL_CHECK_ARG(n >= 1 && n <= N->max_batch, "n out of range");
  DL_TRY(forward_impl(N, X, n));
  if (y) DL_HIP_TRY(hipMemcpyAsync(y, N->y, sizeof(float) * n, hipMemcpyDeviceToDevice, N->stream));
  DL_HIP_TRY(hipMemcpyAsync(N->dy, dy, sizeof(float) * n, hipMemcpyDeviceToDevice, N->stream));
  DL_TRY(backward_impl(N, n));
  DL_HIP_TRY(hipMemcpyAsync(grad, N->G, sizeof(float) * N->n_params, hipMemcpyDeviceToDevice, N->stream));
  return DL_OK;
}

extern "C" dl_status dl_mlp_train_step(dl_mlp* N, const float* X, const float* target, int64_t n, float lr, float wd,
                                       double* loss) {
  DL_CHECK_ARG(N && X && target, "NULL argument");
  DL_CHECK_ARG(n >= 1 && n <= N->max_batch, "n out of range");
  DL_CHECK_ARG(lr >= 0.f && wd >= 0.f, "lr and wd must be >= 0");
  DL_TRY(forward_impl(N, X, n));
  hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, N->stream, N->y, target, n, N->dy, N->loss_dev);
  DL_HIP_TRY(hipGetLastError());
  DL_TRY(backward_impl(N, n));
  N->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = (float)(1.0 - pow(0.9, (double)N->step)), bc2 = (float)(1.0 - pow(0.999, (double)N->step));
  hipLaunchKernelGGL(adamw_kernel, dim3(nblk(N->n_params)), dim3(256), 0, N->stream, N->P, N->G, N->Mo, N->Vo,
                     N->n_params, lr, b1, b2, 1e-8f, wd, bc1, bc2, N->decay);
  DL_HIP_TRY(hipGetLastError());
  DL_TRY(refresh_bf16(N));
  if (loss) {
    DL_HIP_TRY(hipMemcpyAsync(N->loss_host, N->loss_dev, sizeof(double), hipMemcpyDeviceToHost, N->stream));
    DL_HIP_TRY(hipStreamSynchronize(N->stream));
    *loss = *N->loss_host;
  }
  return DL_OK;
}

// ---------------------------------------------------------------------------
// Item features of a created problem (family 0)
// ---------------------------------------------------------------------------
extern "C" dl_status dl_item_features(dl_problem* P, const double* lam_prev, const double* g_prev,
                                      const double* b_prev, float* feats) {
  DL_CHECK_ARG(P && lam_prev && g_prev && b_prev && feats, "NULL argument");
  const int J = P->J;
  hipStream_t st = P->stream;
  unsigned long long *cnt = nullptr, *q1 = nullptr, *q2 = nullptr;
  unsigned *mx = nullptr, *mn = nullptr, *amax = nullptr;
  double* bp = nullptr;
  struct Guard {
    std::vector<void*> p;
    ~Guard() {
      for (void* q : p)
        if (q) (void)hipFree(q);
    }
  } g;
  DL_HIP_TRY(dal(&cnt, J));
  g.p.push_back(cnt);
  DL_HIP_TRY(dal(&q1, J));
  g.p.push_back(q1);
  DL_HIP_TRY(dal(&q2, J));
  g.p.push_back(q2);
  DL_HIP_TRY(dal(&mx, J));
  g.p.push_back(mx);
  DL_HIP_TRY(dal(&mn, J));
  g.p.push_back(mn);
  DL_HIP_TRY(dal(&amax, 1));
  g.p.push_back(amax);
  DL_HIP_TRY(dal(&bp, J));
  g.p.push_back(bp);
  DL_HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * J, st));
  DL_HIP_TRY(hipMemsetAsync(q1, 0, sizeof(unsigned long long) * J, st));
  DL_HIP_TRY(hipMemsetAsync(q2, 0, sizeof(unsigned long long) * J, st));
  DL_HIP_TRY(hipMemsetAsync(mx, 0, sizeof(unsigned) * J, st));
  DL_HIP_TRY(hipMemsetAsync(mn, 0xFF, sizeof(unsigned) * J, st));
  DL_HIP_TRY(hipMemsetAsync(amax, 0, sizeof(unsigned), st));
  DL_HIP_TRY(hipMemcpyAsync(bp, b_prev, sizeof(double) * J, hipMemcpyHostToDevice, st));
  const int blocks = (int)std::min<int64_t>((P->nnz + 255) / 256, (int64_t)P->n_cu * 32);
  const bool bf = P->storage == DL_BF16;
  if (P->nnz > 0) {
    if (bf)
      hipLaunchKernelGGL(feat_pass1<uint16_t>, dim3(blocks), dim3(256), 0, st, P->idx, P->cval, P->nnz, cnt, amax, mx, mn);
    else
      hipLaunchKernelGGL(feat_pass1<float>, dim3(blocks), dim3(256), 0, st, P->idx, P->cval, P->nnz, cnt, amax, mx, mn);
    DL_HIP_TRY(hipGetLastError());
  }
  unsigned ha = 0;
  DL_HIP_TRY(hipMemcpyAsync(&ha, amax, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  DL_HIP_TRY(hipStreamSynchronize(st));
  float cm;
  memcpy(&cm, &ha, 4);
  // fixed-point grids: |sum| <= I * max|c| (resp. max c^2) stays below 2^61
  const double bound = std::max(1.0, (double)P->I) * std::max((double)cm, 1e-30);
  const double s1 = ldexp(1.0, 61 - (int)ceil(log2(bound)));
  const double s2 = ldexp(1.0, 61 - (int)ceil(log2(std::max(1.0, (double)P->I) * std::max((double)cm * cm, 1e-30))));
  if (P->nnz > 0) {
    if (bf)
      hipLaunchKernelGGL(feat_pass2<uint16_t>, dim3(blocks), dim3(256), 0, st, P->idx, P->cval, P->nnz, s1, s2, q1, q2);
    else
      hipLaunchKernelGGL(feat_pass2<float>, dim3(blocks), dim3(256), 0, st, P->idx, P->cval, P->nnz, s1, s2, q1, q2);
    DL_HIP_TRY(hipGetLastError());
  }
  const double mean_n = (double)P->nnz / (double)J;
  hipLaunchKernelGGL(feat_final, dim3(nblk(J)), dim3(256), 0, st, J, cnt, q1, q2, mx, mn, s1, s2, mean_n, P->b, bp,
                     lam_prev, g_prev, feats);
  DL_HIP_TRY(hipGetLastError());
  DL_HIP_TRY(hipStreamSynchronize(st));
  return DL_OK;
}
