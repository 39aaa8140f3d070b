// Problem creation: validation, degree reordering, task table, item statistics,
// Jacobi scaling and the step bound (Appendix C), storage conversion.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "dl_common.h"

static thread_local std::string g_last_error;

void dl_set_error(const std::string& msg) { g_last_error = msg; }

extern "C" const char* dl_last_error(void) { return g_last_error.c_str(); }

namespace {

enum : int { F_RANGE = 1, F_ORDER = 2, F_CNAN = 4, F_ANAN = 8 };

// One thread per row of the caller's CSR: item range, strictly increasing
// items, finite values; per-family max |a| and whether a family is all ones.
__global__ void validate_rows(const int64_t* rp, const int32_t* idx, const float* c, const float* a, int64_t I,
                              int32_t J, int32_t m, int64_t nnz, int* flags, unsigned* amax_bits,
                              int* non_unit) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= I) return;
  int64_t s = rp[i], e = rp[i + 1];
  int bad = 0;
  int32_t prev = -1;
  for (int64_t k = s; k < e; ++k) {
    int32_t j = idx[k];
    if (j < 0 || j >= J) bad |= F_RANGE;
    if (j <= prev) bad |= F_ORDER;
    prev = j;
    if (!isfinite(c[k])) bad |= F_CNAN;
  }
  if (a) {
    for (int f = 0; f < m; ++f) {
      float mx = 0.f;
      int nu = 0;
      for (int64_t k = s; k < e; ++k) {
        float v = a[(int64_t)f * nnz + k];
        if (!isfinite(v)) bad |= F_ANAN;
        mx = fmaxf(mx, fabsf(v));
        nu |= (v != 1.0f);
      }
      if (mx > 0.f) atomicMax(amax_bits + f, __float_as_uint(mx));
      if (nu) atomicOr(non_unit + f, 1);
    }
  }
  if (bad) atomicOr(flags, bad);
}

// One wavefront per reordered user: copy its row from the caller's CSR.
__global__ void gather_rows(const int64_t* orig_rp, const int64_t* new_rp, int64_t I, const int32_t* idx_in,
                            const float* c_in, const float* a_in, int64_t nnz, int n_stored, const int* fam_of_slot,
                            int bf16, uint16_t* idx_out, void* c_out, void* a_out) {
  int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (u >= I) return;
  int64_t os = orig_rp[u], ns = new_rp[u];
  int64_t d = new_rp[u + 1] - ns;
  for (int64_t e = lane; e < d; e += 64) {
    idx_out[ns + e] = (uint16_t)(4 * idx_in[os + e]);  // the byte offset of the item's 4-byte word
    float cv = c_in[os + e];
    if (bf16) reinterpret_cast<uint16_t*>(c_out)[ns + e] = dl_f32_to_bf16_rne(cv);
    else reinterpret_cast<float*>(c_out)[ns + e] = cv;
    for (int sl = 0; sl < n_stored; ++sl) {
      float av = a_in[(int64_t)fam_of_slot[sl] * nnz + os + e];
      int64_t dst = (int64_t)sl * dl_astride(nnz) + ns + e;
      if (bf16) reinterpret_cast<uint16_t*>(a_out)[dst] = dl_f32_to_bf16_rne(av);
      else reinterpret_cast<float*>(a_out)[dst] = av;
    }
  }
}

// Item statistics over the stored layout, as exact integer sums:
//   cnt[j]                       number of users eligible for item j
//   M[(j*m + k)*m + l], k <= l   sum_i a_kij a_lij, on a 2^-E_kl fixed-point grid
//   S[j*m + k]                   sum_i a_kij (stored families), on a 2^-F_k grid
// Values are those the kernels will read (after any BF16 rounding).
template <typename TV>
__device__ inline float ld(const void* p, int64_t e);
template <>
__device__ inline float ld<float>(const void* p, int64_t e) { return reinterpret_cast<const float*>(p)[e]; }
template <>
__device__ inline float ld<uint16_t>(const void* p, int64_t e) {
  return __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(p)[e] << 16);
}

template <typename TV>
__global__ void item_stats(const uint16_t* idx, const void* aval, int64_t nnz, int32_t J, int32_t m,
                           const int* slot, const double* escale, const double* sscale, unsigned long long* cnt,
                           unsigned long long* M, unsigned long long* S) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = idx[e] >> 2;  // stored byte offsets
    atomicAdd(cnt + j, 1ull);
    for (int k = 0; k < m; ++k) {
      double ak = slot[k] >= 0 ? (double)ld<TV>(aval, (int64_t)slot[k] * dl_astride(nnz) + e) : 1.0;
      if (slot[k] >= 0) atomicAdd(S + (int64_t)j * m + k, (unsigned long long)__double2ll_rn(ak * sscale[k]));
      for (int l = k; l < m; ++l) {
        if (slot[k] < 0 && slot[l] < 0) continue;  // 1*1: equals cnt
        double al = slot[l] >= 0 ? (double)ld<TV>(aval, (int64_t)slot[l] * dl_astride(nnz) + e) : 1.0;
        long long q = __double2ll_rn(ak * al * escale[k * m + l]);
        atomicAdd(M + ((int64_t)j * m + k) * m + l, (unsigned long long)q);
      }
    }
  }
}

// New costs on the same eligibility pattern: one wavefront per reordered user
// copies its c row (caller order -> library order) and flags non-finite values.
__global__ void regather_c(const int64_t* orig_rp, const int64_t* new_rp, int64_t I, const float* c_in, int bf16,
                           void* c_out, int* flag) {
  int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (u >= I) return;
  int64_t os = orig_rp[u], ns = new_rp[u];
  int64_t d = new_rp[u + 1] - ns;
  int bad = 0;
  for (int64_t e = lane; e < d; e += 64) {
    float cv = c_in[os + e];
    bad |= !isfinite(cv);
    if (bf16) reinterpret_cast<uint16_t*>(c_out)[ns + e] = dl_f32_to_bf16_rne(cv);
    else reinterpret_cast<float*>(c_out)[ns + e] = cv;
  }
  if (bad) atomicOr(flag, 1);
}

// Per-item maximum of one stored quantity (kind 0: max(0, -c); 1: a; 2: -a; 3: |c|)
// in the order-preserving encoding: block-local LDS maxima, then one global
// atomic maximum per item and block.
template <typename TV>
__global__ void item_extreme(const uint16_t* __restrict__ idx, const TV* __restrict__ val, int64_t nnz, int J,
                             int kind, unsigned* __restrict__ out) {
  extern __shared__ unsigned s_ext[];
  for (int j = threadIdx.x; j < J; j += blockDim.x) s_ext[j] = DL_ORD_NEG_INF;
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    float v = ld<TV>(val, e);
    float q = kind == 0 ? fmaxf(0.f, -v) : (kind == 1 ? v : (kind == 2 ? -v : fabsf(v)));
    atomicMax(&s_ext[idx[e] >> 2], dl_ord_enc(q));  // stored byte offsets
  }
  __syncthreads();
  for (int j = threadIdx.x; j < J; j += blockDim.x)
    if (s_ext[j] != DL_ORD_NEG_INF) atomicMax(&out[j], s_ext[j]);
}

__global__ void fill_u32(unsigned* p, int64_t n, unsigned v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
dl_status dmalloc(dl_problem* P, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  DL_HIP_TRY(hipMalloc((void**)p, n * sizeof(T)));
  P->device_bytes += (double)(n * sizeof(T));
  return DL_OK;
}

void free_problem(dl_problem* P) {
  if (!P) return;
  void* ptrs[] = {P->rp, P->idx, P->cval, P->aval, P->orig_rp, P->wg_task, P->wg_clock, P->b, P->D, P->part, P->acc,
                  P->obj_part, P->pobj_part, P->mu, P->rfac, P->lam_tmp, P->cert_out, P->ext, P->qs_dev,
                  P->qs_words, P->qs_cnt, P->upd_flag};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (P->cert_host) (void)hipHostFree(P->cert_host);
  delete P;
}

dl_status create_impl(const dl_problem_desc* d, dl_problem* P) {
  const int64_t I = d->n_users;
  const int32_t J = d->n_items, m = d->n_families;
  P->I = I;
  P->J = J;
  P->m = m;
  P->proj = d->proj;
  P->storage = d->storage;
  P->radius = d->radius;
  P->upper = d->upper;
  P->eq_mask = d->eq_families & ((1 << d->n_families) - 1);
  P->glob = d->global_count ? 1 : 0;
  P->gcap = P->glob ? d->global_cap : 0.0;
  P->jacobi = d->jacobi ? 1 : 0;
  P->stream = (hipStream_t)d->stream;
  DL_HIP_TRY(hipGetDevice(&P->device));
  hipStream_t st = P->stream;

  // ---- row pointers on the host: validation, degree order, tasks ----
  std::vector<int64_t> rp((size_t)I + 1);
  DL_HIP_TRY(hipMemcpyAsync(rp.data(), d->row_ptr, sizeof(int64_t) * (size_t)(I + 1), hipMemcpyDeviceToHost, st));
  DL_HIP_TRY(hipStreamSynchronize(st));
  DL_CHECK_ARG(rp[0] == 0, "row_ptr[0] must be 0");
  int64_t maxdeg = 0;
  for (int64_t i = 0; i < I; ++i) {
    int64_t dg = rp[i + 1] - rp[i];
    DL_CHECK_ARG(dg >= 0, "row_ptr must be nondecreasing");
    DL_CHECK_ARG(dg <= J, "a row has more entries than there are items");
    maxdeg = std::max(maxdeg, dg);
  }
  const int64_t nnz = rp[I];
  DL_CHECK_ARG(nnz == 0 || (d->item_idx && d->c), "item_idx and c are required");
  P->nnz = nnz;
  P->max_degree = (int32_t)maxdeg;

  // stable counting sort of users by degree, longest first
  std::vector<int64_t> count((size_t)maxdeg + 2, 0);
  for (int64_t i = 0; i < I; ++i) count[(size_t)(maxdeg - (rp[i + 1] - rp[i]))]++;
  std::vector<int64_t> pos((size_t)maxdeg + 2, 0);
  for (int64_t k = 1; k <= maxdeg + 1; ++k) pos[k] = pos[k - 1] + count[k - 1];
  std::vector<int64_t> perm((size_t)I);
  for (int64_t i = 0; i < I; ++i) perm[(size_t)pos[(size_t)(maxdeg - (rp[i + 1] - rp[i]))]++] = i;
  std::vector<int64_t> new_rp((size_t)I + 1), orig_rp((size_t)std::max<int64_t>(I, 1));
  new_rp[0] = 0;
  int64_t I_active = 0;
  for (int64_t u = 0; u < I; ++u) {
    int64_t old = perm[(size_t)u];
    int64_t dg = rp[old + 1] - rp[old];
    new_rp[u + 1] = new_rp[u] + dg;
    orig_rp[u] = rp[old];
    if (dg > 0) I_active = u + 1;
  }
  P->I_active = I_active;

  // ---- device validation of the caller's arrays ----
  int* dflags = nullptr;
  DL_HIP_TRY(hipMalloc((void**)&dflags, sizeof(int) * 16));
  struct FreeGuard {
    void* p;
    ~FreeGuard() { if (p) (void)hipFree(p); }
  } fg{dflags};
  DL_HIP_TRY(hipMemsetAsync(dflags, 0, sizeof(int) * 16, st));
  unsigned* d_amax = reinterpret_cast<unsigned*>(dflags + 4);
  int* d_nonunit = dflags + 8;
  if (I > 0) {
    hipLaunchKernelGGL(validate_rows, dim3((unsigned)((I + 255) / 256)), dim3(256), 0, st, d->row_ptr, d->item_idx,
                       d->c, d->a, I, J, m, nnz, dflags, d_amax, d_nonunit);
    DL_HIP_TRY(hipGetLastError());
  }
  int hflags[16];
  DL_HIP_TRY(hipMemcpyAsync(hflags, dflags, sizeof(hflags), hipMemcpyDeviceToHost, st));
  DL_HIP_TRY(hipStreamSynchronize(st));
  DL_CHECK_ARG(!(hflags[0] & F_RANGE), "item_idx out of range [0, n_items)");
  DL_CHECK_ARG(!(hflags[0] & F_ORDER), "item_idx must be strictly increasing within each row");
  DL_CHECK_ARG(!(hflags[0] & F_CNAN), "c has a non-finite entry");
  DL_CHECK_ARG(!(hflags[0] & F_ANAN), "a has a non-finite entry");
  float amax[DL_MAX_FAMILIES] = {1.f, 1.f, 1.f, 1.f};
  int fam_of_slot[DL_MAX_FAMILIES] = {0, 0, 0, 0};
  P->n_stored = 0;
  for (int k = 0; k < m; ++k) {
    if (d->a && hflags[8 + k]) {
      P->a_slot[k] = P->n_stored;
      fam_of_slot[P->n_stored++] = k;
      float mx;
      memcpy(&mx, &hflags[4 + k], 4);
      amax[k] = mx;
    } else {
      P->a_slot[k] = -1;
      amax[k] = 1.f;
    }
  }
  P->has_a = P->n_stored > 0;

  // degree buckets: 2^glog lanes per user, at most kmax elements per lane
  // coupling blocks beyond one LDS histogram run a multi-family kernel, one
  // launch per window of histogram rows
  if ((int64_t)m * J > DL_MAX_MJ) {
    // histogram windows beside the dual rows in LDS, of equal size
    const int64_t mJ = (int64_t)m * J;
    const size_t mu_b = ((size_t)P->nrow() * 4 + 15) & ~(size_t)15;
    const int64_t cap = (int64_t)((DL_LDS_BYTES - mu_b - 2 * DL_WAVES * 8) / 8);
    P->n_tiles = (int32_t)((mJ + cap - 1) / cap);
    P->tile_rows = (int32_t)((mJ + P->n_tiles - 1) / P->n_tiles);
  }
  // kernel variant by family count: one family (unless windowed), two, or up to four
  P->mf = (m == 1 && P->tile_rows == 0) ? 1 : (m <= 2 ? 2 : 4);
  P->kmax = (P->mf == 1) ? DL_KMAX_PLAIN : DL_KMAX_A;
  const int kmax = P->kmax;
  DL_CHECK_ARG(d->layout == DL_LAYOUT_BUCKETED || d->layout == DL_LAYOUT_WAVEFRONT, "unknown layout");
  const bool wavefront = d->layout == DL_LAYOUT_WAVEFRONT;
  auto code_of = [&](int64_t dg) -> int {
    if (dl_slots(dg, 6) > kmax) return DL_LONG;
    if (wavefront) return 6;
    for (int gl = 0; gl <= 6; ++gl)
      if (dl_slots(dg, gl) <= kmax) return gl;
    return DL_LONG;
  };
  P->buckets.clear();
  std::vector<double> task_cost;
  int64_t u = 0;
  while (u < I_active) {
    int code = code_of(new_rp[u + 1] - new_rp[u]);
    int64_t ue = u;
    while (ue < I_active && code_of(new_rp[ue + 1] - new_rp[ue]) == code) ++ue;
    dl_bucket B;
    B.task_begin = (int64_t)task_cost.size();
    B.user_begin = u;
    B.user_end = ue;
    B.glog = code;
    B.pad = 0;
    if ((int)P->buckets.size() >= DL_MAX_BUCKETS) {
      dl_set_error("internal: too many degree buckets");
      return DL_EUNSUPPORTED;
    }
    P->buckets.push_back(B);
    if (code == DL_LONG) {
      for (int64_t x = u; x < ue; ++x) task_cost.push_back(3.0 * (double)(new_rp[x + 1] - new_rp[x]) + 64.0);
    } else {
      const int64_t upt = 64 >> code;
      for (int64_t x = u; x < ue; x += upt) {
        int64_t d0 = new_rp[x + 1] - new_rp[x];
        int64_t K = dl_slots(d0, code);
        if (K > kmax) {
          dl_set_error("internal: bucket bound violated");
          return DL_EUNSUPPORTED;
        }
        task_cost.push_back(64.0 * (double)K + 64.0);
      }
    }
    u = ue;
  }
  P->n_tasks = (int64_t)task_cost.size();

  int n_cu = 0;
  DL_HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, P->device));
  P->n_cu = n_cu;
  const int wpc = d->wg_per_cu > 0 ? d->wg_per_cu : 4;
  int64_t n_wg = std::min<int64_t>((int64_t)n_cu * wpc, (P->n_tasks + DL_WAVES - 1) / DL_WAVES);
  if (P->n_tasks > 0 && n_wg < 1) n_wg = 1;
  P->task_cost.assign(task_cost.begin(), task_cost.end());
  P->n_wg_cap = (int)std::max<int64_t>(n_wg, 1);
  std::vector<int64_t> wg_task = dl_model_partition(P, (int)n_wg);
  // ---- library-owned layout ----
  const bool bf16 = P->storage == DL_BF16;
  const size_t vb = bf16 ? 2 : 4;
  DL_TRY(dmalloc(P, &P->rp, (size_t)I + 1));
  const int64_t stride = dl_astride(nnz);
  DL_TRY(dmalloc(P, &P->idx, (size_t)stride));
  DL_HIP_TRY(hipMemsetAsync(P->idx + nnz, 0, sizeof(uint16_t) * (size_t)(stride - nnz), st));
  {
    unsigned char* cv = nullptr;
    DL_TRY(dmalloc(P, &cv, (size_t)stride * vb));
    DL_HIP_TRY(hipMemsetAsync(cv + (size_t)nnz * vb, 0, (size_t)(stride - nnz) * vb, st));
    P->cval = cv;
  }
  if (P->n_stored > 0) {
    unsigned char* av = nullptr;
    DL_TRY(dmalloc(P, &av, (size_t)stride * vb * (size_t)P->n_stored));
    DL_HIP_TRY(hipMemsetAsync(av, 0, (size_t)stride * vb * (size_t)P->n_stored, st));
    P->aval = av;
  }
  DL_TRY(dmalloc(P, &P->orig_rp, (size_t)std::max<int64_t>(I, 1)));
  DL_TRY(dmalloc(P, &P->wg_task, (size_t)P->n_wg_cap + 1));
  DL_TRY(dmalloc(P, &P->wg_clock, 2 * (size_t)P->n_wg_cap));
  DL_HIP_TRY(hipMemcpyAsync(P->rp, new_rp.data(), sizeof(int64_t) * (size_t)(I + 1), hipMemcpyHostToDevice, st));
  if (I > 0)
    DL_HIP_TRY(hipMemcpyAsync(P->orig_rp, orig_rp.data(), sizeof(int64_t) * (size_t)I, hipMemcpyHostToDevice, st));
  DL_TRY(dl_set_partition(P, wg_task));
  int* d_slot = dflags + 12;  // fam_of_slot (n_stored <= 4)
  DL_HIP_TRY(hipMemcpyAsync(d_slot, fam_of_slot, sizeof(int) * 4, hipMemcpyHostToDevice, st));
  if (I > 0) {
    const int64_t threads = I * 64;
    hipLaunchKernelGGL(gather_rows, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, P->orig_rp, P->rp, I,
                       d->item_idx, d->c, d->a, nnz, P->n_stored, d_slot, bf16 ? 1 : 0, P->idx, P->cval, P->aval);
    DL_HIP_TRY(hipGetLastError());
  }

  // ---- item statistics: counts and the m x m blocks of A A^T per item ----
  const int64_t mJ = (int64_t)m * J;
  const int64_t nrow = P->nrow();
  std::vector<double> esc((size_t)m * m + m, 0.0);  // the M grids, then the S grids
  for (int k = 0; k < m; ++k) {
    for (int l = k; l < m; ++l) {
      double bound = std::max<double>(1.0, (double)I) * (double)amax[k] * (double)amax[l];
      int E = 61 - (int)ceil(log2(std::max(bound, 1e-300)));
      esc[(size_t)k * m + l] = ldexp(1.0, E);
    }
    const double sb = std::max<double>(1.0, (double)I) * (double)amax[k];
    esc[(size_t)m * m + k] = ldexp(1.0, 61 - (int)ceil(log2(std::max(sb, 1e-300))));
  }
  unsigned long long *d_cnt = nullptr, *d_M = nullptr, *d_S = nullptr;
  double* d_esc = nullptr;
  int* d_aslot = nullptr;
  DL_HIP_TRY(hipMalloc((void**)&d_cnt, sizeof(unsigned long long) * (size_t)J));
  FreeGuard g1{d_cnt};
  DL_HIP_TRY(hipMalloc((void**)&d_M, sizeof(unsigned long long) * (size_t)J * m * (m + 1)));
  FreeGuard g2{d_M};
  d_S = d_M + (size_t)J * m * m;
  DL_HIP_TRY(hipMalloc((void**)&d_esc, sizeof(double) * esc.size() + sizeof(int) * DL_MAX_FAMILIES));
  FreeGuard g3{d_esc};
  d_aslot = reinterpret_cast<int*>(d_esc + esc.size());
  DL_HIP_TRY(hipMemsetAsync(d_cnt, 0, sizeof(unsigned long long) * (size_t)J, st));
  DL_HIP_TRY(hipMemsetAsync(d_M, 0, sizeof(unsigned long long) * (size_t)J * m * (m + 1), st));
  DL_HIP_TRY(hipMemcpyAsync(d_esc, esc.data(), sizeof(double) * esc.size(), hipMemcpyHostToDevice, st));
  DL_HIP_TRY(hipMemcpyAsync(d_aslot, P->a_slot, sizeof(int) * DL_MAX_FAMILIES, hipMemcpyHostToDevice, st));
  if (nnz > 0) {
    int blocks = (int)std::min<int64_t>((nnz + 255) / 256, (int64_t)n_cu * 64);
    if (bf16)
      hipLaunchKernelGGL(item_stats<uint16_t>, dim3(blocks), dim3(256), 0, st, P->idx, P->aval, nnz, J, m, d_aslot,
                         d_esc, d_esc + (size_t)m * m, d_cnt, d_M, d_S);
    else
      hipLaunchKernelGGL(item_stats<float>, dim3(blocks), dim3(256), 0, st, P->idx, P->aval, nnz, J, m, d_aslot,
                         d_esc, d_esc + (size_t)m * m, d_cnt, d_M, d_S);
    DL_HIP_TRY(hipGetLastError());
  }
  std::vector<unsigned long long> cnt((size_t)J), Mq((size_t)J * m * (m + 1));
  DL_HIP_TRY(hipMemcpyAsync(cnt.data(), d_cnt, sizeof(unsigned long long) * (size_t)J, hipMemcpyDeviceToHost, st));
  DL_HIP_TRY(hipMemcpyAsync(Mq.data(), d_M, sizeof(unsigned long long) * (size_t)J * m * (m + 1),
                            hipMemcpyDeviceToHost, st));
  DL_HIP_TRY(hipStreamSynchronize(st));

  // M_j[k][l] in FP64, D = diag(1/||A_kj||_2) (1 on zero rows), lhat >= ||DA||^2
  auto Mkl = [&](int32_t j, int k, int l) -> double {
    if (k > l) std::swap(k, l);
    if (P->a_slot[k] < 0 && P->a_slot[l] < 0) return (double)cnt[(size_t)j];
    long long q = (long long)Mq[((size_t)j * m + k) * m + l];
    return (double)q / esc[(size_t)k * m + l];
  };
  P->D_host.assign((size_t)mJ, 1.0);
  if (P->jacobi) {
    for (int k = 0; k < m; ++k)
      for (int32_t j = 0; j < J; ++j) {
        double n2 = Mkl(j, k, k);
        P->D_host[(size_t)k * J + j] = n2 > 0.0 ? 1.0 / sqrt(n2) : 1.0;
      }
  }
  double L = 0.0;
  for (int32_t j = 0; j < J; ++j)
    for (int k = 0; k < m; ++k) {
      double row = 0.0;
      for (int l = 0; l < m; ++l)
        row += fabs(P->D_host[(size_t)k * J + j] * Mkl(j, k, l) * P->D_host[(size_t)l * J + j]);
      L = std::max(L, row);
    }
  if (P->glob) {
    // The global-count row g (coefficients 1, scaled by D_g = 1/sqrt(nnz)) adds
    // the diagonal entry d_g = D_g^2 nnz and the couplings c_kj = D_kj D_g
    // sum_i a_kij to A'A'^T; Weyl's inequality on the split into the block
    // diagonal and [[0, c], [c^T, 0]] (largest eigenvalue ||c||_2) gives
    // lambda_max <= max(L_items, d_g) + ||c||_2.
    const double Dg = (P->jacobi && nnz > 0) ? 1.0 / sqrt((double)nnz) : 1.0;
    double c2 = 0.0;
    for (int32_t j = 0; j < J; ++j)
      for (int k = 0; k < m; ++k) {
        const double colsum = P->a_slot[k] < 0 ? (double)cnt[(size_t)j]
                                               : (double)(long long)Mq[(size_t)J * m * m + (size_t)j * m + k] /
                                                     esc[(size_t)m * m + k];
        const double c = P->D_host[(size_t)k * J + j] * Dg * colsum;
        c2 += c * c;
      }
    const double dg = Dg * Dg * (double)nnz;
    L = std::max(L, dg) + sqrt(c2);
    P->D_host.push_back(Dg);
  }
  P->lhat = L > 0.0 ? L : 1.0;

  // fixed-point grid of each family's accumulation: |a x| <= amax * radius -> 2^30
  for (int k = 0; k < m; ++k) {
    double bound = (double)amax[k] * d->radius;
    int t = 30 - (int)ceil(log2(std::max(bound, 1e-30)));
    P->qscale[k] = (float)ldexp(1.0, t);
  }

  // ---- item space and scratch ----
  P->b_host.assign(d->b, d->b + mJ);
  if (P->glob) P->b_host.push_back(P->gcap);
  DL_TRY(dmalloc(P, &P->b, (size_t)nrow));
  DL_TRY(dmalloc(P, &P->D, (size_t)nrow));
  DL_HIP_TRY(hipMemcpyAsync(P->b, P->b_host.data(), sizeof(double) * (size_t)nrow, hipMemcpyHostToDevice, st));
  DL_HIP_TRY(hipMemcpyAsync(P->D, P->D_host.data(), sizeof(double) * (size_t)nrow, hipMemcpyHostToDevice, st));
  DL_TRY(dmalloc(P, &P->part, (size_t)P->n_wg_cap * (size_t)nrow));
  DL_TRY(dmalloc(P, &P->acc, (size_t)nrow));
  DL_HIP_TRY(hipMemsetAsync(P->acc, 0, sizeof(unsigned long long) * (size_t)nrow, st));
  DL_TRY(dmalloc(P, &P->obj_part, (size_t)P->n_wg_cap));
  DL_TRY(dmalloc(P, &P->pobj_part, (size_t)P->n_wg_cap));
  DL_TRY(dmalloc(P, &P->mu, (size_t)nrow));
  DL_TRY(dmalloc(P, &P->rfac, (size_t)J));
  DL_TRY(dmalloc(P, &P->lam_tmp, (size_t)nrow));
  DL_TRY(dmalloc(P, &P->cert_out, 16));
  DL_HIP_TRY(hipHostMalloc((void**)&P->cert_host, sizeof(double) * 16, hipHostMallocDefault));
  DL_TRY(dmalloc(P, &P->qs_dev, (size_t)DL_MAX_FAMILIES + 4));
  DL_TRY(dmalloc(P, &P->qs_words, (size_t)DL_MAX_FAMILIES + 1));
  DL_TRY(dmalloc(P, &P->qs_cnt, 1));
  DL_HIP_TRY(hipMemsetAsync(P->qs_words, 0, sizeof(unsigned) * (DL_MAX_FAMILIES + 1), st));
  DL_HIP_TRY(hipMemsetAsync(P->qs_cnt, 0, sizeof(unsigned), st));
  DL_TRY(dmalloc(P, &P->upd_flag, 1));
  {
    // the families' coarsest scales, then the global-count row's (x <= radius per element)
    float q0[DL_MAX_FAMILIES + 4] = {0};
    for (int k = 0; k < DL_MAX_FAMILIES; ++k) q0[k] = P->qscale[k];
    q0[DL_MAX_FAMILIES] = (float)ldexp(1.0, 30 - (int)ceil(log2(std::max(d->radius, 1e-30))));
    DL_HIP_TRY(hipMemcpyAsync(P->qs_dev, q0, sizeof(q0), hipMemcpyHostToDevice, st));
    DL_HIP_TRY(hipStreamSynchronize(st));
  }
  DL_TRY(dmalloc(P, &P->ext, (size_t)J * (size_t)(2 + 2 * P->n_stored)));
  DL_TRY(dl_item_extremes(P, false));
  DL_TRY(dl_grad_prepare(P));
  DL_HIP_TRY(hipStreamSynchronize(st));
  return DL_OK;
}

}  // namespace

std::vector<int64_t> dl_model_partition(const dl_problem* P, int n_wg) {
  std::vector<int64_t> bounds((size_t)std::max(n_wg, 0) + 1, 0);
  if (n_wg <= 0) return bounds;
  double tot = 0.0;
  for (float c : P->task_cost) tot += c;
  double run = 0.0;
  int64_t t = 0;
  for (int w = 1; w < n_wg; ++w) {
    const double target = tot * (double)w / (double)n_wg;
    while (t < P->n_tasks && run + 0.5 * P->task_cost[(size_t)t] < target) run += P->task_cost[(size_t)t++];
    bounds[(size_t)w] = t;
  }
  bounds[(size_t)n_wg] = P->n_tasks;
  return bounds;
}

dl_status dl_set_partition(dl_problem* P, const std::vector<int64_t>& bounds) {
  const int n_wg = (int)bounds.size() - 1;
  if (n_wg < 0 || n_wg > P->n_wg_cap || bounds.front() != 0 || bounds.back() != P->n_tasks) {
    dl_set_error("internal: bad partition");
    return DL_EINVAL;
  }
  for (int w = 0; w < n_wg; ++w)
    if (bounds[(size_t)w + 1] < bounds[(size_t)w]) {
      dl_set_error("internal: partition not monotone");
      return DL_EINVAL;
    }
  DL_HIP_TRY(hipMemcpyAsync(P->wg_task, bounds.data(), sizeof(int64_t) * bounds.size(), hipMemcpyHostToDevice,
                            P->stream));
  DL_HIP_TRY(hipStreamSynchronize(P->stream));
  P->n_wg = n_wg;
  return DL_OK;
}

extern "C" dl_status dl_problem_create(const dl_problem_desc* d, dl_problem** out) {
  if (!out) {
    dl_set_error("out is NULL");
    return DL_EINVAL;
  }
  *out = nullptr;
  DL_CHECK_ARG(d != nullptr, "desc is NULL");
  DL_CHECK_ARG(d->n_users >= 0 && d->n_users < ((int64_t)1 << 40), "n_users out of range");
  DL_CHECK_ARG(d->n_items >= 1, "n_items must be >= 1");
  DL_CHECK_ARG(d->n_families >= 1 && d->n_families <= DL_MAX_FAMILIES, "n_families must be in 1..4");
  DL_CHECK_ARG(d->row_ptr && d->b, "row_ptr and b are required");
  DL_CHECK_ARG(d->proj >= DL_PROJ_SIMPLEX_LE && d->proj <= DL_PROJ_BOXCUT, "unknown projection kind");
  DL_CHECK_ARG((d->eq_families & ~((1 << d->n_families) - 1)) == 0, "eq_families names a family beyond n_families");
  DL_CHECK_ARG(d->proj != DL_PROJ_BOXCUT || (d->upper > 0.0 && isfinite(d->upper)),
               "box-cut needs a positive, finite upper bound");
  DL_CHECK_ARG(d->storage == DL_F32 || d->storage == DL_BF16, "unknown storage");
  DL_CHECK_ARG(d->radius > 0.0 && isfinite(d->radius), "radius must be positive and finite");
  const int64_t mJ = (int64_t)d->n_items * d->n_families;
  for (int64_t r = 0; r < mJ; ++r) DL_CHECK_ARG(isfinite(d->b[r]), "b has a non-finite entry");
  DL_CHECK_ARG(d->global_count == 0 || d->global_count == 1, "global_count must be 0 or 1");
  DL_CHECK_ARG(!d->global_count || (isfinite(d->global_cap) && d->global_cap >= 0.0),
               "global_cap must be finite and >= 0");
  if (d->n_items > DL_MAX_ITEMS) {
    dl_set_error("n_items exceeds the 16-bit item offsets of this build (16383)");
    return DL_EUNSUPPORTED;
  }
  // LDS of a workgroup: the dual rows and, in the repair pass, one factor per item
  const int64_t rows = mJ + (d->global_count ? 1 : 0);
  if ((size_t)(rows + d->n_items) * 4 + 512 > DL_LDS_BYTES) {
    dl_set_error("n_rows + n_items exceeds what one workgroup stages in LDS (40,832 words)");
    return DL_EUNSUPPORTED;
  }
  dl_problem* P = new (std::nothrow) dl_problem();
  if (!P) {
    dl_set_error("host allocation failed");
    return DL_ENOMEM;
  }
  dl_status s = create_impl(d, P);
  if (s != DL_OK) {
    free_problem(P);
    return s;
  }
  *out = P;
  return DL_OK;
}

dl_status dl_item_extremes(dl_problem* P, bool c_only) {
  const int J = P->J;
  const int n_q = c_only ? 2 : 2 + 2 * P->n_stored;
  hipStream_t st = P->stream;
  const int64_t tot = (int64_t)J * n_q;
  hipLaunchKernelGGL(fill_u32, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, P->ext, tot, DL_ORD_NEG_INF);
  DL_HIP_TRY(hipGetLastError());
  if (P->nnz == 0) return DL_OK;
  const unsigned blocks = (unsigned)std::min<int64_t>(1024, (P->nnz + 1023) / 1024);
  const size_t lds = sizeof(unsigned) * (size_t)J;
  const bool bf16 = P->storage == DL_BF16;
  for (int q = 0; q < n_q; ++q) {
    // columns: max(0, -c), |c|, then max a and max -a of every stored slot
    const int kind = q == 0 ? 0 : (q == 1 ? 3 : (q % 2 == 0 ? 1 : 2));
    const int slot = q < 2 ? 0 : (q - 2) / 2;
    const void* val = q < 2 ? P->cval
                             : (const void*)((const char*)P->aval + (size_t)slot * (size_t)dl_astride(P->nnz) *
                                                                       (bf16 ? 2 : 4));
    unsigned* out = P->ext + (size_t)q * J;
    if (bf16)
      hipLaunchKernelGGL(item_extreme<uint16_t>, dim3(blocks), dim3(1024), lds, st, P->idx,
                         (const uint16_t*)val, P->nnz, J, kind, out);
    else
      hipLaunchKernelGGL(item_extreme<float>, dim3(blocks), dim3(1024), lds, st, P->idx, (const float*)val, P->nnz,
                         J, kind, out);
    DL_HIP_TRY(hipGetLastError());
  }
  return DL_OK;
}

extern "C" void dl_problem_destroy(dl_problem* P) { free_problem(P); }

extern "C" dl_status dl_problem_update(dl_problem* P, const float* c, const double* b) {
  DL_CHECK_ARG(P, "NULL problem");
  hipStream_t st = P->stream;
  const int64_t mJ = (int64_t)P->m * P->J;
  if (b)
    for (int64_t r = 0; r < mJ; ++r) DL_CHECK_ARG(isfinite(b[r]), "b has a non-finite entry");
  if (c && P->nnz > 0) {
    int* flag = P->upd_flag;
    DL_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
    const int64_t threads = P->I * 64;
    hipLaunchKernelGGL(regather_c, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, P->orig_rp, P->rp, P->I,
                       c, P->storage == DL_BF16 ? 1 : 0, P->cval, flag);
    DL_HIP_TRY(hipGetLastError());
    int hf = 0;
    DL_HIP_TRY(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    DL_HIP_TRY(hipStreamSynchronize(st));
    DL_CHECK_ARG(!hf, "c has a non-finite entry (the problem's c is now partly updated)");
    DL_TRY(dl_item_extremes(P, true));
  }
  if (b) {
    P->b_host.assign(b, b + mJ);
    if (P->glob) P->b_host.push_back(P->gcap);  // the global cap is kept
    DL_HIP_TRY(hipMemcpyAsync(P->b, P->b_host.data(), sizeof(double) * mJ, hipMemcpyHostToDevice, st));
    DL_HIP_TRY(hipStreamSynchronize(st));
  }
  return DL_OK;
}

extern "C" dl_status dl_problem_get_info(const dl_problem* P, dl_problem_info* o) {
  DL_CHECK_ARG(P && o, "NULL argument");
  memset(o, 0, sizeof(*o));
  o->n_users = P->I;
  o->nnz = P->nnz;
  o->n_items = P->J;
  o->n_families = P->m;
  o->n_stored_families = P->n_stored;
  o->n_workgroups = P->n_wg;
  o->n_tasks = P->n_tasks;
  o->lhat = P->lhat;
  const double vb = P->storage == DL_BF16 ? 2.0 : 4.0;
  // per nnz: 16-bit item offset + c + stored a's; per user: row pointer; per item: lam in
  o->bytes_per_pass = (double)P->nnz * (2.0 + vb * (1 + P->n_stored)) + 8.0 * (double)(P->I + 1) +
                      (double)P->nrow() * 4.0;
  o->n_rows = P->nrow();
  o->n_windows = P->n_tiles;
  o->device_bytes = P->device_bytes;
  o->max_degree = P->max_degree;
  o->n_buckets = (int32_t)P->buckets.size();
  for (size_t i = 0; i < P->buckets.size() && i < 8; ++i) {
    o->bucket_glog[i] = P->buckets[i].glog;
    o->bucket_users[i] = P->buckets[i].user_end - P->buckets[i].user_begin;
  }
  for (int k = 0; k < DL_MAX_FAMILIES; ++k) o->qscale[k] = P->qscale[k];
  return DL_OK;
}
