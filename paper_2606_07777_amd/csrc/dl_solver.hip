// Item-space kernels and the Maximizer of the dual ascent (Sections 4.4 and 6,
// Appendix C): fixed-order reduction of the per-workgroup partial sums, the
// accelerated projected step on lam >= 0 in Jacobi-scaled units, the
// certificate (feasible repair, primal and dual values, gap, slack), and the
// host loop over the gamma schedule.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <utility>

#include "dl_cert.h"
#include "dl_common.h"

namespace {

struct upd_args {
  unsigned long long* acc;  // reduced per-item sums (read and cleared)
  const unsigned long long* part;  // per-workgroup partial sums, n_wg x nrow (the fused step reads them)
  int n_wg;
  int mJ, J;        // item rows m*J, items J
  int nrow;         // dual rows: m*J, then the global-count row when present
  const float* qs;  // fixed-point scale of each family in the pass being reduced (device)
  int eq_mask;      // bit k: family k has free duals (equality rows)
  const double* D;
  const double* b;
  double* lam;      // scaled lam'
  double* y;        // scaled momentum point y'
  float* mu_y;      // FP32 D y' (problem units), gathered by the next pass
  float* mu_lam;    // FP32 D lam'
  double eta, beta;
  int* flag;
  double* ax_out;   // nullable: A x (problem units)
  double* grad_out; // nullable: A x - b
};

// First level of the partial-sum reduction: block (x, y) adds rows
// [y*DL_RED_ROWS, (y+1)*DL_RED_ROWS) of the per-workgroup histograms for 256
// items and adds the result into acc with a 64-bit integer atomic (exact, so
// the total does not depend on the order).  acc is cleared by its reader.
constexpr int DL_RED_ROWS = 16;
__global__ void reduce_partials(const unsigned long long* __restrict__ part, int n_wg, int mJ,
                                unsigned long long* __restrict__ acc) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mJ) return;
  const int w0 = blockIdx.y * DL_RED_ROWS;
  const int w1 = min(n_wg, w0 + DL_RED_ROWS);
  long long s = 0;
  for (int w = w0; w < w1; ++w) s += (long long)part[(size_t)w * mJ + r];
  if (s != 0) atomicAdd(acc + r, (unsigned long long)s);
}

// Reads and clears the reduced sum of item r.
__device__ __forceinline__ double take_sum(unsigned long long* acc, int r) {
  const long long v = (long long)acc[r];
  acc[r] = 0ull;
  return (double)v;
}

// The accelerated step of row r from its reduced fixed-point sum: take
// lam'_+ = max(0, y' + eta D (A x - b)), y'_+ = lam'_+ + beta (lam'_+ - lam'),
// and publish the next gather point D y'_+ (FP32).
__device__ __forceinline__ void step_row(const upd_args& U, int r, long long sum) {
  const int k = r < U.mJ ? r / U.J : DL_MAX_FAMILIES;  // the global-count row has its own scale
  const double ax = (double)sum / (double)U.qs[k];
  const double Dr = U.D[r];
  const double gs = Dr * (ax - U.b[r]);
  const double lo = U.lam[r];
  const double st = U.y[r] + U.eta * gs;
  const double ln = ((U.eq_mask >> k) & 1) ? st : fmax(0.0, st);
  const double yn = ln + U.beta * (ln - lo);
  U.lam[r] = ln;
  U.y[r] = yn;
  U.mu_y[r] = (float)(Dr * yn);
  U.mu_lam[r] = (float)(Dr * ln);
  if (!isfinite(ln) || !isfinite(yn)) atomicOr(U.flag, 1);
}

// Reduction and step in one launch: a block takes 64 dual rows; its 16 slices
// of 64 lanes each add every 16th workgroup's partial sums of those rows
// (512 contiguous bytes per slot and wavefront), the slices are added in LDS,
// and one slice applies the step.  Integer sums: exact, so the result is the
// two-launch reduction's bitwise.
constexpr int DL_RU_ROWS = 64;
constexpr int DL_RU_SLICES = 16;
__global__ void __launch_bounds__(DL_RU_ROWS * DL_RU_SLICES) reduce_update_kernel(upd_args U) {
  __shared__ long long sh[DL_RU_SLICES][DL_RU_ROWS];
  const int rl = (int)threadIdx.x % DL_RU_ROWS;
  const int sl = (int)threadIdx.x / DL_RU_ROWS;
  const int r = (int)blockIdx.x * DL_RU_ROWS + rl;
  long long sum = 0;
  if (r < U.nrow) {
#pragma unroll 4
    for (int w = sl; w < U.n_wg; w += DL_RU_SLICES) sum += (long long)U.part[(size_t)w * U.nrow + r];
  }
  sh[sl][rl] = sum;
  __syncthreads();
  if (sl != 0 || r >= U.nrow) return;
  for (int q = 1; q < DL_RU_SLICES; ++q) sum += sh[q][rl];
  step_row(U, r, sum);
}

// A x (and A x - b) from the partials, no step.
__global__ void reduce_kernel(upd_args U) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= U.nrow) return;
  const int k = r < U.mJ ? r / U.J : DL_MAX_FAMILIES;
  const double ax = take_sum(U.acc, r) / (double)U.qs[k];
  if (U.ax_out) U.ax_out[r] = ax;
  if (U.grad_out) U.grad_out[r] = ax - U.b[r];
}

// lam' = max(0, lam0 / D), y' = lam', gather points; or (lam0 == NULL) zeros.
__global__ void init_state(const double* lam0, const double* D, int mJ, int J, int eq_mask, double* lam, double* y,
                           float* mu_y, float* mu_lam) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mJ) return;
  const double l0 = lam0 ? lam0[r] / D[r] : 0.0;
  double l = ((eq_mask >> (r / J)) & 1) ? l0 : fmax(0.0, l0);
  lam[r] = l;
  y[r] = l;
  float m = (float)(D[r] * l);
  mu_y[r] = m;
  mu_lam[r] = m;
}

// Momentum restart at a stage switch: y' = lam'.
__global__ void reset_momentum(const double* D, int mJ, const double* lam, double* y, float* mu_y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mJ) return;
  y[r] = lam[r];
  mu_y[r] = (float)(D[r] * lam[r]);
}

__global__ void scaled_to_units(const double* D, int mJ, const double* lam, double* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mJ) return;
  out[r] = D[r] * lam[r];
}

__global__ void to_f32(const double* in, int n, float* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[r] = (float)in[r];
}

// Certificate, item part (one workgroup): see cert_items_body.
__global__ void cert_items(const double* ax, const double* b, const float* mu, int m, int J, int eq_mask, int glob,
                           const double* obj_part, int n_wg, float* rfac, double* out) {
  __shared__ double sh[1024];
  cert_items_body(ax, b, mu, m, J, eq_mask, glob, obj_part, n_wg, rfac, out, sh);
}

// out[3] = sum_w pobj_part[w]   (primal value of the repaired point)
__global__ void cert_final(const double* pobj_part, int n_wg, double* out) {
  __shared__ double sh[1024];
  cert_final_body(pobj_part, n_wg, out, sh);
}

inline unsigned blocks_for(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

dl_status launch_reduce(const dl_problem* P) {
  const int mJ = (int)P->nrow();  // dual rows
  if (P->n_wg <= 0) return DL_OK;
  dim3 grid(blocks_for(mJ), (unsigned)((P->n_wg + DL_RED_ROWS - 1) / DL_RED_ROWS));
  hipLaunchKernelGGL(reduce_partials, grid, dim3(256), 0, P->stream, P->part, P->n_wg, mJ, P->acc);
  DL_HIP_TRY(hipGetLastError());
  return DL_OK;
}

}  // namespace

dl_status dl_cert_stats(const double* c, int flag, double gamma, int eq_mask, dl_solve_stats* st);

struct dl_solver {
  dl_problem* P = nullptr;
  double* lam = nullptr;   // m*J scaled
  double* y = nullptr;
  double* ax = nullptr;    // certificate scratch
  float* mu_y = nullptr;
  float* mu_lam = nullptr;
  int* flag = nullptr;
  double gamma = 1.0, eta = 1.0, tk = 1.0;
  int64_t iters = 0;
  bool timing = false;
  // timing: (start, end) of each gradient pass, and the end of the reduction +
  // update that follows it (which starts at the pass's end event)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_grad;
  std::vector<hipEvent_t> ev_upd;
  size_t n_ev_grad = 0, n_ev_upd = 0;
};

namespace {

upd_args make_upd(const dl_problem* P) {
  upd_args U;
  memset(&U, 0, sizeof(U));
  U.acc = P->acc;
  U.part = P->part;
  U.n_wg = P->n_wg;
  U.mJ = P->m * P->J;
  U.nrow = (int)P->nrow();
  U.J = P->J;
  U.qs = P->qs_dev;
  U.eq_mask = P->eq_mask;
  U.D = P->D;
  U.b = P->b;
  return U;
}

dl_status next_event_pair(std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, size_t& n,
                          std::pair<hipEvent_t, hipEvent_t>** out) {
  if (n == v.size()) {
    hipEvent_t a, b;
    DL_HIP_TRY(hipEventCreate(&a));
    DL_HIP_TRY(hipEventCreate(&b));
    v.emplace_back(a, b);
  }
  *out = &v[n++];
  return DL_OK;
}

dl_status next_event(std::vector<hipEvent_t>& v, size_t& n, hipEvent_t* out) {
  if (n == v.size()) {
    hipEvent_t a;
    DL_HIP_TRY(hipEventCreate(&a));
    v.push_back(a);
  }
  *out = v[n++];
  return DL_OK;
}

// Certificate at the solver's current lam (Table 4 metrics, certified gap).
// Enqueues the certificate at the solver's lam on the problem's stream; its
// values and the non-finite flag land in the problem's pinned host words
// (cert_host[0..3], and the flag as an int at cert_host + 8) once the stream
// has passed them.
dl_status certificate_enqueue(dl_solver* S) {
  dl_problem* P = S->P;
  const int mJ = (int)P->nrow();  // dual rows
  DL_TRY(dl_launch_grad(P, M_HIST | M_OBJ, S->mu_lam, S->gamma, nullptr, nullptr, nullptr, P->obj_part));
  DL_TRY(launch_reduce(P));
  upd_args U = make_upd(P);
  U.ax_out = S->ax;
  hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(mJ)), dim3(256), 0, P->stream, U);
  DL_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(cert_items, dim3(1), dim3(1024), 0, P->stream, S->ax, P->b, S->mu_lam, P->m, P->J,
                     P->eq_mask, P->glob, P->obj_part, P->n_wg, P->rfac, P->cert_out);
  DL_HIP_TRY(hipGetLastError());
  DL_TRY(dl_launch_grad(P, M_REPAIR, S->mu_lam, S->gamma, P->rfac, nullptr, nullptr, P->pobj_part));
  hipLaunchKernelGGL(cert_final, dim3(1), dim3(1024), 0, P->stream, P->pobj_part, P->n_wg, P->cert_out);
  DL_HIP_TRY(hipGetLastError());
  DL_HIP_TRY(hipMemcpyAsync(P->cert_host, P->cert_out, sizeof(double) * 4, hipMemcpyDeviceToHost, P->stream));
  DL_HIP_TRY(hipMemcpyAsync(reinterpret_cast<int*>(P->cert_host + 8), S->flag, sizeof(int), hipMemcpyDeviceToHost,
                            P->stream));
  return DL_OK;
}

// The statistics of a certificate enqueued earlier; the caller has
// synchronised the stream past it.
dl_status certificate_read(dl_solver* S, dl_solve_stats* st) {
  dl_problem* P = S->P;
  const int hflag = *reinterpret_cast<const int*>(P->cert_host + 8);
  const dl_status rc = dl_cert_stats(P->cert_host, hflag, S->gamma, P->eq_mask, st);
  st->iters = S->iters;
  return rc;
}

dl_status certificate(dl_solver* S, dl_solve_stats* st) {
  DL_TRY(certificate_enqueue(S));
  DL_HIP_TRY(hipStreamSynchronize(S->P->stream));
  return certificate_read(S, st);
}

}  // namespace

// Statistics of a certificate from its four values (dual value, max slack,
// Lagrangian gap, repaired primal value) and the iterate's non-finite flag.
dl_status dl_cert_stats(const double* c, int flag, double gamma, int eq_mask, dl_solve_stats* st) {
  const double g = c[0], pobj = c[3];
  st->gamma = gamma;
  st->dual_obj = g;
  st->primal_obj = pobj;
  // equality rows have no feasible repair: the certified gap is undefined
  st->rel_gap = eq_mask ? NAN : (pobj - g) / fmax(1.0, fabs(g));
  st->max_slack = c[1];
  st->lagr_gap = c[2];
  if (flag) {
    dl_set_error("non-finite dual iterate");
    return DL_DIVERGED;
  }
  if (!isfinite(g) || !isfinite(pobj)) {
    dl_set_error("non-finite dual objective or certificate");
    return DL_NUMERIC;
  }
  return DL_OK;
}


// ---------------------------------------------------------------------------
// ObjectiveFunction and ProjectionMap
// ---------------------------------------------------------------------------
extern "C" dl_status dl_dual_grad(dl_problem* P, const double* lambda, double gamma, double* grad, double* dual_obj,
                                  float* x) {
  DL_CHECK_ARG(P && lambda, "NULL argument");
  DL_CHECK_ARG(gamma > 0.0 && isfinite(gamma), "gamma must be positive and finite");
  const int mJ = (int)P->nrow();  // dual rows
  hipLaunchKernelGGL(to_f32, dim3(blocks_for(mJ)), dim3(256), 0, P->stream, lambda, mJ, P->mu);
  DL_HIP_TRY(hipGetLastError());
  const bool want_obj = dual_obj != nullptr;
  DL_TRY(dl_launch_grad(P, want_obj ? (M_HIST | M_OBJ) : M_HIST, P->mu, gamma, nullptr, nullptr, x, P->obj_part));
  DL_TRY(launch_reduce(P));
  upd_args U = make_upd(P);
  U.ax_out = P->lam_tmp;
  U.grad_out = grad;
  hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(mJ)), dim3(256), 0, P->stream, U);
  DL_HIP_TRY(hipGetLastError());
  if (want_obj) {
    hipLaunchKernelGGL(cert_items, dim3(1), dim3(1024), 0, P->stream, P->lam_tmp, P->b, P->mu, P->m, P->J,
                       P->eq_mask, P->glob, P->obj_part, P->n_wg, P->rfac, P->cert_out);
    DL_HIP_TRY(hipGetLastError());
    DL_HIP_TRY(hipMemcpyAsync(P->cert_host, P->cert_out, sizeof(double), hipMemcpyDeviceToHost, P->stream));
    DL_HIP_TRY(hipStreamSynchronize(P->stream));
    *dual_obj = P->cert_host[0];
  }
  return DL_OK;
}

extern "C" dl_status dl_project(dl_problem* P, const float* v, float* x) {
  DL_CHECK_ARG(P && ((v && x) || P->nnz == 0), "NULL argument");
  return dl_launch_grad(P, M_VIN, nullptr, 1.0, nullptr, v, x, nullptr);
}

// ---------------------------------------------------------------------------
// Maximizer
// ---------------------------------------------------------------------------
extern "C" dl_status dl_solver_create(dl_problem* P, const double* lambda0, dl_solver** out) {
  DL_CHECK_ARG(P && out, "NULL argument");
  *out = nullptr;
  dl_solver* S = new (std::nothrow) dl_solver();
  if (!S) {
    dl_set_error("host allocation failed");
    return DL_ENOMEM;
  }
  S->P = P;
  const int mJ = (int)P->nrow();  // dual rows
  auto fail = [&](dl_status s) {
    dl_solver_destroy(S);
    return s;
  };
  if (hipMalloc((void**)&S->lam, sizeof(double) * mJ) != hipSuccess ||
      hipMalloc((void**)&S->y, sizeof(double) * mJ) != hipSuccess ||
      hipMalloc((void**)&S->ax, sizeof(double) * mJ) != hipSuccess ||
      hipMalloc((void**)&S->mu_y, sizeof(float) * mJ) != hipSuccess ||
      hipMalloc((void**)&S->mu_lam, sizeof(float) * mJ) != hipSuccess ||
      hipMalloc((void**)&S->flag, sizeof(int)) != hipSuccess) {
    dl_set_error("device allocation failed");
    return fail(DL_ENOMEM);
  }
  if (hipMemsetAsync(S->flag, 0, sizeof(int), P->stream) != hipSuccess) return fail(DL_EHIP);
  hipLaunchKernelGGL(init_state, dim3(blocks_for(mJ)), dim3(256), 0, P->stream, lambda0, P->D, mJ, P->J, P->eq_mask,
                     S->lam, S->y,
                     S->mu_y, S->mu_lam);
  if (hipGetLastError() != hipSuccess) {
    dl_set_error("init_state launch failed");
    return fail(DL_EHIP);
  }
  *out = S;
  return DL_OK;
}

// Device state of a solver, for the batched iteration.
dl_status dl_solver_state(dl_solver* S, double** lam, double** y, float** mu_y, float** mu_lam, int** flag,
                          double** ax) {
  DL_CHECK_ARG(S, "NULL solver");
  if (ax) *ax = S->ax;
  *lam = S->lam;
  *y = S->y;
  *mu_y = S->mu_y;
  *mu_lam = S->mu_lam;
  *flag = S->flag;
  return DL_OK;
}

extern "C" void dl_solver_destroy(dl_solver* S) {
  if (!S) return;
  void* ptrs[] = {S->lam, S->y, S->ax, S->mu_y, S->mu_lam, S->flag};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (auto& e : S->ev_grad) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (hipEvent_t e : S->ev_upd) (void)hipEventDestroy(e);
  delete S;
}

extern "C" dl_status dl_solver_set_stage(dl_solver* S, double gamma, double step_scale, int32_t reset) {
  DL_CHECK_ARG(S, "NULL solver");
  DL_CHECK_ARG(gamma > 0.0 && isfinite(gamma), "gamma must be positive and finite");
  DL_CHECK_ARG(step_scale > 0.0 && isfinite(step_scale), "step_scale must be positive");
  dl_problem* P = S->P;
  S->gamma = gamma;
  S->eta = step_scale * gamma / P->lhat;  // step proportional to gamma (L <= ||A'||^2/gamma)
  if (reset) {
    S->tk = 1.0;
    const int mJ = (int)P->nrow();  // dual rows
    hipLaunchKernelGGL(reset_momentum, dim3(blocks_for(mJ)), dim3(256), 0, P->stream, P->D, mJ, S->lam, S->y,
                       S->mu_y);
    DL_HIP_TRY(hipGetLastError());
  }
  return DL_OK;
}

extern "C" dl_status dl_solver_step(dl_solver* S, int64_t n) {
  DL_CHECK_ARG(S && n >= 0, "bad argument");
  dl_problem* P = S->P;
  const int mJ = (int)P->nrow();  // dual rows
  upd_args U = make_upd(P);
  U.lam = S->lam;
  U.y = S->y;
  U.mu_y = S->mu_y;
  U.mu_lam = S->mu_lam;
  U.eta = S->eta;
  U.flag = S->flag;
  for (int64_t it = 0; it < n; ++it) {
    std::pair<hipEvent_t, hipEvent_t>* eg = nullptr;
    // the pass's fixed-point scales first, so the timing events bracket the gradient kernel alone
    DL_TRY(dl_launch_qscale(P, S->mu_y, S->gamma));
    if (S->timing) {
      DL_TRY(next_event_pair(S->ev_grad, S->n_ev_grad, &eg));
      DL_HIP_TRY(hipEventRecord(eg->first, P->stream));
    }
    DL_TRY(dl_launch_grad(P, M_HIST, S->mu_y, S->gamma, nullptr, nullptr, nullptr, nullptr, true));
    hipEvent_t eu = nullptr;
    if (S->timing) {
      DL_HIP_TRY(hipEventRecord(eg->second, P->stream));
      DL_TRY(next_event(S->ev_upd, S->n_ev_upd, &eu));
    }
    // FISTA momentum: t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, beta = (t_k - 1) / t_{k+1}
    const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * S->tk * S->tk));
    U.beta = (S->tk - 1.0) / tn;
    S->tk = tn;
    hipLaunchKernelGGL(reduce_update_kernel, dim3(blocks_for(mJ, DL_RU_ROWS)), dim3(DL_RU_ROWS * DL_RU_SLICES), 0,
                       P->stream, U);
    DL_HIP_TRY(hipGetLastError());
    if (S->timing) DL_HIP_TRY(hipEventRecord(eu, P->stream));
    ++S->iters;
  }
  return DL_OK;
}

// Checkpoint / resume: the scaled dual state (lam', y') is copied as is, so a
// resumed run continues bitwise where the exported one stood.
namespace {
__global__ void state_gather_points(const double* D, int mJ, const double* lam, const double* y, float* mu_y,
                                    float* mu_lam) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mJ) return;
  mu_y[r] = (float)(D[r] * y[r]);
  mu_lam[r] = (float)(D[r] * lam[r]);
}
}  // namespace

extern "C" dl_status dl_solver_export(dl_solver* S, double* state, dl_solver_meta* meta) {
  DL_CHECK_ARG(S && state && meta, "NULL argument");
  dl_problem* P = S->P;
  const size_t mJ = (size_t)P->nrow();  // dual rows
  DL_HIP_TRY(hipMemcpyAsync(state, S->lam, sizeof(double) * mJ, hipMemcpyDeviceToDevice, P->stream));
  DL_HIP_TRY(hipMemcpyAsync(state + mJ, S->y, sizeof(double) * mJ, hipMemcpyDeviceToDevice, P->stream));
  meta->gamma = S->gamma;
  meta->eta = S->eta;
  meta->tk = S->tk;
  meta->iters = S->iters;
  meta->m_times_j = (int64_t)mJ;
  return DL_OK;
}

extern "C" dl_status dl_solver_import(dl_solver* S, const double* state, const dl_solver_meta* meta) {
  DL_CHECK_ARG(S && state && meta, "NULL argument");
  dl_problem* P = S->P;
  const int mJ = (int)P->nrow();  // dual rows
  DL_CHECK_ARG(meta->m_times_j == mJ, "state was exported from a problem of another size");
  DL_CHECK_ARG(meta->gamma > 0.0 && isfinite(meta->gamma) && meta->eta > 0.0 && isfinite(meta->eta) &&
                   meta->tk >= 1.0 && isfinite(meta->tk) && meta->iters >= 0,
               "invalid solver state");
  DL_HIP_TRY(hipMemcpyAsync(S->lam, state, sizeof(double) * mJ, hipMemcpyDeviceToDevice, P->stream));
  DL_HIP_TRY(hipMemcpyAsync(S->y, state + mJ, sizeof(double) * mJ, hipMemcpyDeviceToDevice, P->stream));
  hipLaunchKernelGGL(state_gather_points, dim3(blocks_for(mJ)), dim3(256), 0, P->stream, P->D, mJ, S->lam, S->y,
                     S->mu_y, S->mu_lam);
  DL_HIP_TRY(hipGetLastError());
  S->gamma = meta->gamma;
  S->eta = meta->eta;
  S->tk = meta->tk;
  S->iters = meta->iters;
  return DL_OK;
}

extern "C" dl_status dl_solver_get_lambda(dl_solver* S, double* out) {
  DL_CHECK_ARG(S && out, "NULL argument");
  dl_problem* P = S->P;
  const int mJ = (int)P->nrow();  // dual rows
  hipLaunchKernelGGL(scaled_to_units, dim3(blocks_for(mJ)), dim3(256), 0, P->stream, P->D, mJ, S->lam, out);
  DL_HIP_TRY(hipGetLastError());
  return DL_OK;
}

extern "C" dl_status dl_solver_certificate(dl_solver* S, dl_solve_stats* out) {
  DL_CHECK_ARG(S && out, "NULL argument");
  memset(out, 0, sizeof(*out));
  dl_status s = certificate(S, out);
  out->status = s;
  return s;
}

extern "C" dl_status dl_solver_enable_timing(dl_solver* S, int32_t on) {
  DL_CHECK_ARG(S, "NULL solver");
  S->timing = on != 0;
  S->n_ev_grad = S->n_ev_upd = 0;
  return DL_OK;
}

extern "C" dl_status dl_solver_get_timing(dl_solver* S, dl_timing* out) {
  DL_CHECK_ARG(S && out, "NULL argument");
  DL_HIP_TRY(hipStreamSynchronize(S->P->stream));
  memset(out, 0, sizeof(*out));
  for (size_t i = 0; i < S->n_ev_grad; ++i) {
    float ms = 0.f;
    DL_HIP_TRY(hipEventElapsedTime(&ms, S->ev_grad[i].first, S->ev_grad[i].second));
    out->grad_ms_total += ms;
  }
  for (size_t i = 0; i < S->n_ev_upd; ++i) {
    float ms = 0.f;
    DL_HIP_TRY(hipEventElapsedTime(&ms, S->ev_grad[i].second, S->ev_upd[i]));
    out->update_ms_total += ms;
  }
  out->n_grad = (int64_t)S->n_ev_grad;
  out->n_update = (int64_t)S->n_ev_upd;
  return DL_OK;
}

namespace {

// Runs `reps` histogram passes at the solver's point with workgroup clocks on;
// returns the mean pass time and the last pass's per-workgroup durations.
// Mean time of reps gradient passes, each followed by the reduction of its
// partial sums (the part of an iteration the split decides), and the per-
// workgroup durations of the last pass.  The reduced sums are discarded, so
// the solver state is unchanged.
dl_status measure_pass(dl_solver* S, int reps, double* ms, std::vector<double>* dur) {
  dl_problem* P = S->P;
  hipEvent_t e0, e1;
  DL_HIP_TRY(hipEventCreate(&e0));
  DL_HIP_TRY(hipEventCreate(&e1));
  P->clocking = true;
  dl_status rc = DL_OK;
  if (hipEventRecord(e0, P->stream) != hipSuccess) rc = DL_EHIP;
  for (int r = 0; r < reps && rc == DL_OK; ++r) {
    rc = dl_launch_grad(P, M_HIST, S->mu_y, S->gamma, nullptr, nullptr, nullptr, nullptr);
    if (rc == DL_OK) rc = launch_reduce(P);
  }
  P->clocking = false;
  if (rc == DL_OK && hipEventRecord(e1, P->stream) != hipSuccess) rc = DL_EHIP;
  if (rc == DL_OK &&
      hipMemsetAsync(P->acc, 0, sizeof(unsigned long long) * (size_t)P->nrow(), P->stream) != hipSuccess)
    rc = DL_EHIP;
  std::vector<unsigned long long> clk(2 * (size_t)std::max(P->n_wg, 1));
  if (rc == DL_OK && P->n_wg > 0 &&
      hipMemcpyAsync(clk.data(), P->wg_clock, sizeof(unsigned long long) * 2 * P->n_wg, hipMemcpyDeviceToHost,
                     P->stream) != hipSuccess)
    rc = DL_EHIP;
  if (rc == DL_OK && hipStreamSynchronize(P->stream) != hipSuccess) rc = DL_EHIP;
  float t = 0.f;
  if (rc == DL_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = DL_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != DL_OK) {
    dl_set_error("timing a gradient pass failed");
    return rc;
  }
  *ms = t / reps;
  dur->assign((size_t)P->n_wg, 0.0);
  for (int w = 0; w < P->n_wg; ++w) (*dur)[(size_t)w] = (double)(clk[2 * w + 1] - clk[2 * w]);
  return DL_OK;
}

double imbalance(const std::vector<double>& d) {
  if (d.empty()) return 1.0;
  double mx = 0.0, sum = 0.0;
  for (double v : d) {
    mx = std::max(mx, v);
    sum += v;
  }
  return sum > 0 ? mx / (sum / (double)d.size()) : 1.0;
}

// New split with equal measured time: the measured cost of a workgroup's range
// is spread evenly over its tasks and the cumulative cost is cut into equal parts.
std::vector<int64_t> rebalance(const std::vector<int64_t>& b, const std::vector<double>& dur) {
  const int n = (int)dur.size();
  std::vector<double> cum((size_t)n + 1, 0.0);
  for (int w = 0; w < n; ++w) cum[(size_t)w + 1] = cum[(size_t)w] + std::max(dur[(size_t)w], 1.0);
  std::vector<int64_t> nb(b.size());
  nb[0] = b[0];
  nb[(size_t)n] = b[(size_t)n];
  int v = 0;
  for (int w = 1; w < n; ++w) {
    const double target = cum[(size_t)n] * (double)w / (double)n;
    while (v + 1 < n && cum[(size_t)v + 1] <= target) ++v;
    const double frac = (target - cum[(size_t)v]) / (cum[(size_t)v + 1] - cum[(size_t)v]);
    int64_t t = b[(size_t)v] + (int64_t)llround(frac * (double)(b[(size_t)v + 1] - b[(size_t)v]));
    nb[(size_t)w] = std::max(nb[(size_t)w - 1], std::min(t, b[(size_t)n]));
  }
  return nb;
}

}  // namespace

extern "C" dl_status dl_solver_autotune(dl_solver* S, int32_t rounds, dl_tune_result* out) {
  DL_CHECK_ARG(S && out && rounds >= 0, "bad argument");
  dl_problem* P = S->P;
  memset(out, 0, sizeof(*out));
  out->rounds = rounds;
  if (P->n_tasks == 0) return DL_OK;
  const int reps = 3, final_reps = 10;
  // per grid size: the best split found by the balancing rounds; the finalists
  // are timed again with more passes before one is kept (a minimum over short,
  // noisy timings would favour whichever candidate happened to run fastest)
  struct cand {
    int nw;
    std::vector<int64_t> b;
    double ms_model, imb_model, imb;
  };
  std::vector<cand> cands;
  for (int k = 1;; k *= 2) {
    int nw = (int)std::min<int64_t>((int64_t)P->n_cu * k, (P->n_tasks + DL_WAVES - 1) / DL_WAVES);
    nw = std::max(1, std::min(nw, P->n_wg_cap));
    std::vector<int64_t> b = dl_model_partition(P, nw);
    DL_TRY(dl_set_partition(P, b));
    double ms;
    std::vector<double> dur;
    DL_TRY(measure_pass(S, reps, &ms, &dur));
    const double ms_model = ms, imb_model = imbalance(dur);
    double cur_ms = ms, cur_imb = imb_model;
    std::vector<int64_t> cur = b;
    for (int r = 0; r < rounds; ++r) {
      std::vector<int64_t> nb = rebalance(b, dur);
      DL_TRY(dl_set_partition(P, nb));
      DL_TRY(measure_pass(S, reps, &ms, &dur));
      b = nb;
      if (ms < cur_ms) {
        cur_ms = ms;
        cur_imb = imbalance(dur);
        cur = nb;
      }
    }
    cands.push_back({nw, cur, ms_model, imb_model, cur_imb});
    if (nw >= P->n_wg_cap || (int64_t)P->n_cu * k * 2 > P->n_wg_cap) break;
  }
  double best_ms = 1e300;
  size_t best = 0;
  for (size_t q = 0; q < cands.size(); ++q) {
    DL_TRY(dl_set_partition(P, cands[q].b));
    double ms;
    std::vector<double> dur;
    DL_TRY(measure_pass(S, final_reps, &ms, &dur));
    if (ms < best_ms) {
      best_ms = ms;
      best = q;
    }
  }
  const cand& c = cands[best];
  out->n_workgroups = c.nw;
  out->pass_ms_model = c.ms_model;
  out->imbalance_model = c.imb_model;
  out->pass_ms_tuned = best_ms;
  out->imbalance_tuned = c.imb;
  return dl_set_partition(P, c.b);
}

namespace {

dl_status check_schedule(const dl_solve_opts* o) {
  DL_CHECK_ARG(o->n_stages >= 1 && o->gammas && o->iters, "empty schedule");
  for (int s = 0; s < o->n_stages; ++s) {
    DL_CHECK_ARG(o->gammas[s] > 0.0 && isfinite(o->gammas[s]), "gamma must be positive and finite");
    DL_CHECK_ARG(o->iters[s] >= 0 || s == o->n_stages - 1, "only the last stage may run until tol");
  }
  DL_CHECK_ARG(o->max_iters >= 0 && o->check_every >= 0, "negative limits");
  return DL_OK;
}

// The schedule of dl_solve on a solver already at its starting point; writes the
// final lam (problem units) and the stats.  Allocates nothing itself (the
// workgroup tuner, when asked for, creates timing events).
dl_status run_schedule(dl_solver* S, const dl_solve_opts* o, double* lambda_out, dl_solve_stats* st,
                       std::chrono::steady_clock::time_point t0) {
  dl_problem* P = S->P;
  const double step_scale = o->step_scale > 0.0 ? o->step_scale : 1.0;
  dl_status rc = DL_OK;
  bool converged = false;
  int64_t n_checks = 0;
  int stage = 0;
  for (stage = 0; stage < o->n_stages && rc == DL_OK && !converged; ++stage) {
    rc = dl_solver_set_stage(S, o->gammas[stage], step_scale, stage == 0 ? 1 : o->reset_momentum);
    if (rc != DL_OK) break;
    const bool last = stage == o->n_stages - 1;
    const int64_t n_it = o->iters[stage];
    int64_t done = 0;
    if (stage == 0 && o->autotune_rounds > 0) {
      const int64_t pre = std::min<int64_t>(n_it < 0 ? 50 : std::min<int64_t>(n_it, 50), o->max_iters);
      rc = dl_solver_step(S, pre);
      if (rc != DL_OK) break;
      done = pre;
      dl_tune_result tr;
      rc = dl_solver_autotune(S, o->autotune_rounds, &tr);
      if (rc != DL_OK) break;
    }
    while ((n_it < 0 || done < n_it) && S->iters < o->max_iters) {
      int64_t chunk = (n_it < 0) ? o->max_iters - S->iters : n_it - done;
      if (last && o->check_every > 0) chunk = std::min<int64_t>(chunk, o->check_every - (done % o->check_every));
      chunk = std::min<int64_t>(chunk, o->max_iters - S->iters);
      rc = dl_solver_step(S, chunk);
      if (rc != DL_OK) break;
      done += chunk;
      if (last && o->check_every > 0 && done % o->check_every == 0) {
        rc = certificate(S, st);
        ++n_checks;
        if (rc != DL_OK) break;
        if (st->rel_gap <= o->tol) {
          converged = true;
          break;
        }
      }
      if (n_it < 0 && o->check_every == 0) break;  // nothing would ever stop it
    }
    if (S->iters >= o->max_iters) {
      ++stage;
      break;
    }
  }
  if (rc == DL_OK && !converged) {
    rc = certificate(S, st);
    ++n_checks;
    if (rc == DL_OK) converged = st->rel_gap <= o->tol;
  }
  dl_status lrc = dl_solver_get_lambda(S, lambda_out);
  if (rc == DL_OK) rc = lrc;
  if (rc == DL_OK) DL_HIP_TRY(hipStreamSynchronize(P->stream));
  st->iters = S->iters;
  st->stage = stage - 1;
  st->n_checks = n_checks;
  st->status = (rc == DL_OK) ? (converged ? DL_OK : DL_NOT_CONVERGED) : rc;
  st->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rc != DL_OK) return rc;
  return converged ? DL_OK : DL_NOT_CONVERGED;
}

}  // namespace

extern "C" dl_status dl_solve(dl_problem* P, const dl_solve_opts* o, const double* lambda0, double* lambda_out,
                              dl_solve_stats* st) {
  DL_CHECK_ARG(P && o && st && lambda_out, "NULL argument");
  DL_TRY(check_schedule(o));
  auto t0 = std::chrono::steady_clock::now();
  memset(st, 0, sizeof(*st));
  dl_solver* S = nullptr;
  DL_TRY(dl_solver_create(P, lambda0, &S));
  const dl_status rc = run_schedule(S, o, lambda_out, st, t0);
  dl_solver_destroy(S);
  return rc;
}

// ---------------------------------------------------------------------------
// dl_solve without allocation: the solver state lives in a fixed device array
// ---------------------------------------------------------------------------
namespace {

// Rows (m*J) the array holds: lam', y' and A x in FP64, the two FP32 gather
// points, i.e. 32 bytes per row, plus the divergence flag.
constexpr int64_t DL_NOALLOC_MAX_MJ = 16384;
constexpr size_t DL_NOALLOC_BYTES = 32 * (size_t)DL_NOALLOC_MAX_MJ + 256;
__device__ __align__(256) unsigned char scratch[DL_NOALLOC_BYTES];

// Device address of `scratch` on each device (the host-side symbol is not one).
constexpr int DL_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[DL_MAX_DEVICES] = {};

__global__ void fill_i32(int* p, int n, int v) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) p[r] = v;
}

dl_status scratch_on_device(int dev, unsigned char** out) {
  DL_CHECK_ARG(dev >= 0 && dev < DL_MAX_DEVICES, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    DL_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
      dl_set_error("hipGetSymbolAddress returned NULL for the solver scratch");
      return DL_EHIP;
    }
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return DL_OK;
}

}  // namespace

extern "C" dl_status dl_solve_noalloc(dl_problem* P, const dl_solve_opts* o, const double* lambda0,
                                      double* lambda_out, dl_solve_stats* st) {
  DL_CHECK_ARG(P && o && st && lambda_out, "NULL argument");
  DL_TRY(check_schedule(o));
  DL_CHECK_ARG(o->autotune_rounds == 0, "dl_solve_noalloc does not run the workgroup tuner (autotune_rounds must be 0)");
  const int64_t mJ = P->nrow();  // dual rows
  if (mJ > DL_NOALLOC_MAX_MJ) {
    dl_set_error("dl_solve_noalloc: the problem's dual rows exceed its fixed state array (16384 rows)");
    return DL_EUNSUPPORTED;
  }
  int dev = -1;
  DL_HIP_TRY(hipGetDevice(&dev));
  DL_CHECK_ARG(dev == P->device, "dl_solve_noalloc: make the problem's device current first");
  unsigned char* base = nullptr;
  DL_TRY(scratch_on_device(dev, &base));
  auto t0 = std::chrono::steady_clock::now();
  memset(st, 0, sizeof(*st));
  // state of a solver without its own memory: nothing here is freed
  dl_solver S;
  S.P = P;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  S.lam = reinterpret_cast<double*>(take(sizeof(double) * mJ));
  S.y = reinterpret_cast<double*>(take(sizeof(double) * mJ));
  S.ax = reinterpret_cast<double*>(take(sizeof(double) * mJ));
  S.mu_y = reinterpret_cast<float*>(take(sizeof(float) * mJ));
  S.mu_lam = reinterpret_cast<float*>(take(sizeof(float) * mJ));
  S.flag = reinterpret_cast<int*>(take(sizeof(int)));
  if (off > DL_NOALLOC_BYTES) {
    dl_set_error("internal: solver scratch layout exceeds its array");
    return DL_EUNSUPPORTED;
  }
  // the previous call's contents stay in the array: clear the flag, set the start
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, P->stream, S.flag, 1, 0);
  DL_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(init_state, dim3(blocks_for(mJ)), dim3(256), 0, P->stream, lambda0, P->D, (int)mJ, P->J,
                     P->eq_mask, S.lam, S.y, S.mu_y, S.mu_lam);
  DL_HIP_TRY(hipGetLastError());
  const dl_status rc = run_schedule(&S, o, lambda_out, st, t0);
  // the state belongs to the array: make sure nothing of it is released
  S.lam = S.y = S.ax = nullptr;
  S.mu_y = S.mu_lam = nullptr;
  S.flag = nullptr;
  return rc;
}

// ---------------------------------------------------------------------------
// Judged warm start: the candidate with the largest dual value starts the solve
// ---------------------------------------------------------------------------
namespace {
__global__ void project_candidate(const double* in, int n, int J, int eq_mask, double* out, int* bad) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double v = in ? in[r] : 0.0;
  if (!isfinite(v)) atomicOr(bad, 1);
  const double w = isfinite(v) ? v : 0.0;
  out[r] = ((eq_mask >> (r / J)) & 1) ? w : fmax(w, 0.0);
}
}  // namespace

extern "C" dl_status dl_solve_warm(dl_problem* P, const dl_solve_opts* o, int32_t n_cand,
                                   const double* const* cands, double* lambda_out, dl_solve_stats* stats,
                                   int32_t* chosen, double* cand_dual) {
  DL_CHECK_ARG(P && o && stats && lambda_out && n_cand >= 1 && cands, "bad argument");
  DL_CHECK_ARG(o->n_stages >= 1 && o->gammas, "empty schedule");
  const int mJ = (int)P->nrow();  // dual rows
  const double gamma0 = o->gammas[0];
  double* tmp = nullptr;
  int* bad = nullptr;
  DL_HIP_TRY(hipMalloc((void**)&tmp, sizeof(double) * (size_t)mJ * 2 + sizeof(int)));
  bad = reinterpret_cast<int*>(tmp + 2 * (size_t)mJ);
  double* grad = tmp + mJ;
  int best = -1;
  double best_g = -INFINITY;
  dl_status rc = DL_OK;
  for (int q = 0; q < n_cand && rc == DL_OK; ++q) {
    if (hipMemsetAsync(bad, 0, sizeof(int), P->stream) != hipSuccess) { rc = DL_EHIP; break; }
    hipLaunchKernelGGL(project_candidate, dim3(blocks_for(mJ)), dim3(256), 0, P->stream, cands[q], mJ, P->J,
                       P->eq_mask, tmp, bad);
    double g = -INFINITY;
    rc = dl_dual_grad(P, tmp, gamma0, grad, &g, nullptr);
    if (rc != DL_OK) break;
    int hb = 0;
    if (hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, P->stream) != hipSuccess ||
        hipStreamSynchronize(P->stream) != hipSuccess) { rc = DL_EHIP; break; }
    if (hb || !isfinite(g)) g = -INFINITY;  // a non-finite candidate never wins
    if (cand_dual) cand_dual[q] = g;
    if (g > best_g) {
      best_g = g;
      best = q;
    }
  }
  if (rc == DL_OK && best < 0) {
    dl_set_error("no finite candidate start");
    rc = DL_NUMERIC;
  }
  if (rc == DL_OK) {
    hipLaunchKernelGGL(project_candidate, dim3(blocks_for(mJ)), dim3(256), 0, P->stream, cands[best], mJ, P->J,
                       P->eq_mask, tmp, bad);
    if (hipGetLastError() != hipSuccess) rc = DL_EHIP;
  }
  dl_status sr = rc;
  if (rc == DL_OK) sr = dl_solve(P, o, tmp, lambda_out, stats);
  (void)hipStreamSynchronize(P->stream);
  (void)hipFree(tmp);
  if (chosen) *chosen = best;
  return sr;
}
