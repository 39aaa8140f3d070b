// Many independent instances solved together: per iteration, one scale launch,
// one gradient-pass launch, one slot-reduction launch and one update launch
// serve every live instance, whatever its size.
//
// Workgroups are dealt to instances in proportion to their pass cost (several
// per compute unit, so the hardware's workgroup dispatch evens out what the
// static split leaves uneven).  The cost is the problem's own per-task model
// until the tuner has timed the batched pass; from then on it is the measured
// time of every workgroup's range, spread over the range's tasks by the model.
// Each workgroup serves a contiguous task range of one instance and writes its
// integer histogram into that instance's own partial slots, so every
// instance's gradient is bitwise the one its solo pass gives, whatever the
// split.  All instances follow the same gamma schedule in lockstep; the
// certificate runs per instance at the check points of the final stage, and
// converged instances leave the launch tables.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <numeric>

#include "dl_cert.h"
#include "dl_common.h"
#include "dl_split.h"

struct dl_solver;  // dl_solver.hip
dl_status dl_solver_state(dl_solver* S, double** lam, double** y, float** mu_y, float** mu_lam, int** flag,
                          double** ax);
dl_status dl_cert_stats(const double* c, int flag, double gamma, int eq_mask, dl_solve_stats* st);

namespace {

struct bupd {
  const unsigned long long* part;
  unsigned long long* acc;  // the member's reduced sums (its problem's accumulator, zero between passes)
  double* cert_ax;          // the certificate's A x (its solver's scratch)
  int n_slot;
  int mJ, J;        // item rows m*J, items J
  int nrow;         // dual rows: m*J, then the global-count row when present
  const float* qs;  // the instance's fixed-point scales of the pass (device)
  int eq_mask;      // bit k: family k has free duals
  const double* D;
  const double* b;
  double* lam;
  double* y;
  float* mu_y;
  float* mu_lam;
  int* flag;
  double lhat;
};

struct bblk {
  int inst;
  int r0;
};

// A block of the slot reduction: slots [s0, s0 + DL_BRED_SLOTS) of member inst
// for the 256 rows from r0.
struct bred {
  int inst;
  int r0;
  int s0;
};
constexpr int DL_BRED_SLOTS = 16;

// Sums a block of a member's partial histograms into its accumulator (64-bit
// integer atomics: exact in any order).  Short chains of loads per thread keep
// the reduction parallel however many workgroups a member was dealt.
__global__ void reduce_batch(const bupd* __restrict__ U, const bred* __restrict__ red) {
  const bred R = red[blockIdx.x];
  const bupd& u = U[R.inst];
  const int r = R.r0 + (int)threadIdx.x;
  if (r >= u.nrow) return;
  const int s1 = min(u.n_slot, R.s0 + DL_BRED_SLOTS);
  long long sum = 0;
  for (int w = R.s0; w < s1; ++w) sum += (long long)u.part[(size_t)w * u.nrow + r];
  if (sum != 0) atomicAdd(u.acc + r, (unsigned long long)sum);
}

// The fused accelerated step of every live instance (same arithmetic as the
// single-instance update): take and clear the reduced sum, step on the
// Jacobi-scaled dual, FISTA momentum, next gather point.
__global__ void update_batch(const bupd* __restrict__ U, const bblk* __restrict__ blk, double gamma,
                             double step_scale, double beta) {
  const bblk B = blk[blockIdx.x];
  const bupd& u = U[B.inst];
  const int r = B.r0 + (int)threadIdx.x;
  if (r >= u.nrow) return;
  const long long acc = (long long)u.acc[r];
  u.acc[r] = 0ull;
  const int k = r < u.mJ ? r / u.J : DL_MAX_FAMILIES;  // the global-count row has its own scale
  const double ax = (double)acc / (double)u.qs[k];
  const double Dr = u.D[r];
  const double eta = step_scale * gamma / u.lhat;
  const double gs = Dr * (ax - u.b[r]);
  const double lo = u.lam[r];
  const double st = u.y[r] + eta * gs;
  const double ln = ((u.eq_mask >> k) & 1) ? st : fmax(0.0, st);
  const double yn = ln + beta * (ln - lo);
  u.lam[r] = ln;
  u.y[r] = yn;
  u.mu_y[r] = (float)(Dr * yn);
  u.mu_lam[r] = (float)(Dr * ln);
  if (!isfinite(ln) || !isfinite(yn)) atomicOr(u.flag, 1);
}

// A check point of every live member at once.  The certificate's two passes
// run as batched launches over the iteration's workgroup table; these kernels
// do the rest: decode A x, the item part, and the final sums.
struct bcert {
  const double* ax;
  const double* b;
  const float* mu;  // the member's FP32 lam, the point both passes used
  int m, J, eq_mask, glob;
  const double* obj_part;   // per workgroup slot of the member
  const double* pobj_part;
  int n_slot;
  float* rfac;
  double* out;              // the member's 4 certificate values (device)
  const int* flag;          // non-finite iterate flag
};

// A x of every live member from its reduced sums (the update's decode, without the step).
__global__ void cert_decode_batch(const bupd* __restrict__ U, const bblk* __restrict__ blk) {
  const bblk B = blk[blockIdx.x];
  const bupd& u = U[B.inst];
  const int r = B.r0 + (int)threadIdx.x;
  if (r >= u.nrow) return;
  const long long acc = (long long)u.acc[r];
  u.acc[r] = 0ull;
  const int k = r < u.mJ ? r / u.J : DL_MAX_FAMILIES;
  u.cert_ax[r] = (double)acc / (double)u.qs[k];
}

// The certificate's item part, one workgroup per live member.
__global__ void __launch_bounds__(1024) cert_items_batch(const bcert* __restrict__ C) {
  __shared__ double sh[1024];
  const bcert& c = C[blockIdx.x];
  cert_items_body(c.ax, c.b, c.mu, c.m, c.J, c.eq_mask, c.glob, c.obj_part, c.n_slot, c.rfac, c.out, sh);
}

// The repaired primal value, then each member's 4 values and its flag, gathered
// for one copy to the host (5 doubles per live member).
__global__ void __launch_bounds__(1024) cert_final_batch(const bcert* __restrict__ C, double* __restrict__ res) {
  __shared__ double sh[1024];
  const bcert& c = C[blockIdx.x];
  cert_final_body(c.pobj_part, c.n_slot, c.out, sh);
  if (threadIdx.x == 0) {
    double* o = res + 5 * (size_t)blockIdx.x;
    for (int k = 0; k < 4; ++k) o[k] = c.out[k];
    o[4] = (double)*c.flag;
  }
}

}  // namespace

struct dl_batch {
  int n = 0;
  std::vector<dl_problem*> probs;
  std::vector<dl_solver*> solvers;
  hipStream_t stream = nullptr;
  int n_cu = 0;
  int wg_per_cu = 4;
  // device tables
  dl_grad_args* d_args = nullptr;
  dl_grad_args* d_cargs = nullptr;  // the certificate's histogram + objective pass (at lam)
  dl_grad_args* d_rargs = nullptr;  // the certificate's repair pass
  bcert* d_cert = nullptr;          // per live position
  double* d_cres = nullptr;         // 5 per live position
  double* h_cres = nullptr;         // pinned copy of d_cres
  size_t lds_rep = 0;
  dl_wg_desc* d_wgs = nullptr;
  bupd* d_upd = nullptr;
  bblk* d_blk = nullptr;
  bred* d_red = nullptr;
  unsigned long long* d_part = nullptr;
  size_t part_cap = 0;
  // the certificate's per-workgroup objective sums (histogram pass, repair pass): a
  // member's region has one entry per workgroup the batch deals it, which can exceed
  // the slots its problem allocated for its own grid
  double* d_obj = nullptr;
  size_t obj_cap = 0;
  int n_wg = 0, n_blk = 0, n_red = 0;
  size_t lds = 0;
  bool glob = false;  // some live member has a global-count row
  // host mirrors
  std::vector<dl_grad_args> h_args, h_cargs, h_rargs;
  std::vector<bcert> h_cert;
  std::vector<dl_wg_desc> h_wgs;
  std::vector<bupd> h_upd;
  std::vector<bblk> h_blk;
  std::vector<bred> h_red;
  std::vector<int> live;           // the instances the tables were built for
  std::vector<size_t> wg_first;    // per live position: its first workgroup in h_wgs
  // per-workgroup (start, end) clock stamps of a timed pass; clock_cap entries
  unsigned long long* d_clock = nullptr;
  size_t clock_cap = 0;
  std::vector<std::vector<double>> cmodel;  // per instance: prefix sums of its tasks' model weights
  std::vector<double> model_tot;   // per instance: total cost-model weight of its tasks
  std::vector<dl_inst_profile> prof;  // per instance: measured cost profile (empty: cost model)
  dl_tune_result tune;             // last tuning result (zeros before any)
};

static void free_batch(dl_batch* B) {
  if (!B) return;
  for (dl_solver* s : B->solvers) dl_solver_destroy(s);
  void* ptrs[] = {B->d_args, B->d_cargs, B->d_rargs, B->d_cert, B->d_cres, B->d_obj,
                  B->d_wgs,  B->d_upd,   B->d_blk,   B->d_red,  B->d_part, B->d_clock};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (B->h_cres) (void)hipHostFree(B->h_cres);
  delete B;
}

// Rebuilds the launch tables for the live instances at gamma.
static dl_status build_tables(dl_batch* B, const std::vector<int>& live, double gamma) {
  // earlier launches may still read the tables about to be replaced
  DL_HIP_TRY(hipStreamSynchronize(B->stream));
  // pass cost per instance: measured ticks where profiled, else the cost model
  // in the ticks-per-weight ratio of the profiled ones
  double meas = 0.0, meas_model = 0.0;
  for (int i : live)
    if (!B->prof[i].ticks.empty()) {
      for (double v : B->prof[i].ticks) meas += std::max(v, 1.0);
      meas_model += B->model_tot[i];
    }
  const double ratio = (meas > 0.0 && meas_model > 0.0) ? meas / meas_model : 1.0;
  std::vector<double> cost(live.size());
  double tot = 0.0;
  for (size_t q = 0; q < live.size(); ++q) {
    const int i = live[q];
    if (B->prof[i].ticks.empty()) {
      cost[q] = B->model_tot[i] * ratio;
    } else {
      cost[q] = 0.0;
      for (double v : B->prof[i].ticks) cost[q] += std::max(v, 1.0);
    }
    tot += cost[q];
  }
  const int budget = std::max<int>((int)live.size(), B->n_cu * B->wg_per_cu);
  // workgroups per instance: largest-remainder rounding of the cost share, >= 1 with tasks
  std::vector<int> w(live.size(), 0);
  std::vector<std::pair<double, int>> rem;
  int used = 0;
  for (size_t q = 0; q < live.size(); ++q) {
    const dl_problem* P = B->probs[live[q]];
    if (P->n_tasks == 0) continue;
    double share = tot > 0 ? cost[q] / tot * budget : 1.0;
    w[q] = std::max(1, (int)floor(share));
    w[q] = (int)std::min<int64_t>(w[q], P->n_tasks);
    used += w[q];
    rem.push_back({share - floor(share), (int)q});
  }
  std::sort(rem.begin(), rem.end(), [](auto& a, auto& b) { return a.first > b.first; });
  for (auto& r : rem) {
    if (used >= budget) break;
    const dl_problem* P = B->probs[live[r.second]];
    if (w[r.second] < P->n_tasks) {
      ++w[r.second];
      ++used;
    }
  }
  B->h_wgs.clear();
  B->h_upd.clear();
  B->h_blk.clear();
  B->h_red.clear();
  size_t part_need = 0, lds = 0;
  std::vector<size_t> part_off(live.size(), 0);
  for (size_t q = 0; q < live.size(); ++q) {
    const dl_problem* P = B->probs[live[q]];
    part_off[q] = part_need;
    part_need += (size_t)std::max(1, w[q]) * (size_t)P->nrow();
    lds = std::max(lds, dl_grad_lds_bytes(P, M_HIST));
  }
  if (part_need > B->part_cap) {
    if (B->d_part) DL_HIP_TRY(hipFree(B->d_part));
    B->d_part = nullptr;
    DL_HIP_TRY(hipMalloc((void**)&B->d_part, part_need * sizeof(unsigned long long)));
    B->part_cap = part_need;
  }
  // objective slots: two per dealt workgroup (histogram pass, then repair pass)
  std::vector<size_t> obj_off(live.size(), 0);
  size_t obj_need = 0;
  for (size_t q = 0; q < live.size(); ++q) {
    obj_off[q] = obj_need;
    obj_need += 2 * (size_t)std::max(1, w[q]);
  }
  if (obj_need > B->obj_cap) {
    if (B->d_obj) DL_HIP_TRY(hipFree(B->d_obj));
    B->d_obj = nullptr;
    DL_HIP_TRY(hipMalloc((void**)&B->d_obj, obj_need * sizeof(double)));
    B->obj_cap = obj_need;
  }
  B->h_args.assign(B->n, dl_grad_args());
  B->h_cargs.assign(B->n, dl_grad_args());
  B->h_rargs.assign(B->n, dl_grad_args());
  B->h_cert.clear();
  size_t lds_rep = 0;
  B->live = live;
  B->wg_first.assign(live.size(), 0);
  for (size_t q = 0; q < live.size(); ++q) {
    const int i = live[q];
    const dl_problem* P = B->probs[i];
    double *lam, *y;
    float *mu_y, *mu_lam;
    int* flag;
    double* cax;
    DL_TRY(dl_solver_state(B->solvers[i], &lam, &y, &mu_y, &mu_lam, &flag, &cax));
    dl_grad_args A = dl_make_grad_args(P, mu_y, gamma);
    A.part = B->d_part + part_off[q];
    B->h_args[i] = A;
    // the certificate's passes: same workgroup table and partial slots, at lam, with
    // the batch's own objective slots
    double* objs = B->d_obj + obj_off[q];
    double* pobjs = objs + std::max(1, w[q]);
    dl_grad_args C = A;
    C.mu = mu_lam;
    C.obj_part = objs;
    B->h_cargs[i] = C;
    C.rfac = P->rfac;
    C.obj_part = pobjs;
    B->h_rargs[i] = C;
    lds_rep = std::max(lds_rep, dl_grad_lds_bytes(P, M_REPAIR));
    bcert ce;
    ce.ax = cax;
    ce.b = P->b;
    ce.mu = mu_lam;
    ce.m = P->m;
    ce.J = P->J;
    ce.eq_mask = P->eq_mask;
    ce.glob = P->glob;
    ce.obj_part = objs;
    ce.pobj_part = pobjs;
    ce.n_slot = w[q];
    ce.rfac = P->rfac;
    ce.out = P->cert_out;
    ce.flag = flag;
    B->h_cert.push_back(ce);
    // contiguous task ranges of this instance with equal estimated time
    B->wg_first[q] = B->h_wgs.size();
    if (w[q] > 0) {
      const std::vector<int64_t> bd = dl_split_tasks(w[q], B->prof[i], B->cmodel[i]);
      for (int k = 0; k < w[q]; ++k) {
        dl_wg_desc d;
        d.inst = i;
        d.slot = k;
        d.t0 = bd[(size_t)k];
        d.t1 = bd[(size_t)k + 1];
        B->h_wgs.push_back(d);
      }
    }
    bupd u;
    memset(&u, 0, sizeof(u));
    u.part = A.part;
    u.acc = P->acc;
    u.cert_ax = cax;
    u.n_slot = w[q];
    u.mJ = P->m * P->J;
    u.nrow = (int)P->nrow();
    u.J = P->J;
    u.qs = P->qs_dev;
    u.eq_mask = P->eq_mask;
    u.D = P->D;
    u.b = P->b;
    u.lam = lam;
    u.y = y;
    u.mu_y = mu_y;
    u.mu_lam = mu_lam;
    u.flag = flag;
    u.lhat = P->lhat;
    const int ui = (int)B->h_upd.size();
    B->h_upd.push_back(u);
    for (int r0 = 0; r0 < u.nrow; r0 += 256) {
      B->h_blk.push_back({ui, r0});
      for (int s0 = 0; s0 < u.n_slot; s0 += DL_BRED_SLOTS) B->h_red.push_back({ui, r0, s0});
    }
  }
  B->n_wg = (int)B->h_wgs.size();
  B->n_blk = (int)B->h_blk.size();
  B->n_red = (int)B->h_red.size();
  B->lds_rep = lds_rep;
  B->lds = lds;
  B->glob = false;
  for (int i : live) B->glob = B->glob || B->probs[i]->glob;
  if (B->d_wgs) DL_HIP_TRY(hipFree(B->d_wgs));
  if (B->d_upd) DL_HIP_TRY(hipFree(B->d_upd));
  if (B->d_blk) DL_HIP_TRY(hipFree(B->d_blk));
  if (B->d_red) DL_HIP_TRY(hipFree(B->d_red));
  B->d_wgs = nullptr;
  B->d_upd = nullptr;
  B->d_blk = nullptr;
  B->d_red = nullptr;
  DL_HIP_TRY(hipMalloc((void**)&B->d_wgs, sizeof(dl_wg_desc) * std::max<size_t>(1, B->h_wgs.size())));
  DL_HIP_TRY(hipMalloc((void**)&B->d_upd, sizeof(bupd) * std::max<size_t>(1, B->h_upd.size())));
  DL_HIP_TRY(hipMalloc((void**)&B->d_blk, sizeof(bblk) * std::max<size_t>(1, B->h_blk.size())));
  DL_HIP_TRY(hipMalloc((void**)&B->d_red, sizeof(bred) * std::max<size_t>(1, B->h_red.size())));
  hipStream_t st = B->stream;
  DL_HIP_TRY(hipMemcpyAsync(B->d_args, B->h_args.data(), sizeof(dl_grad_args) * B->n, hipMemcpyHostToDevice, st));
  DL_HIP_TRY(hipMemcpyAsync(B->d_cargs, B->h_cargs.data(), sizeof(dl_grad_args) * B->n, hipMemcpyHostToDevice, st));
  DL_HIP_TRY(hipMemcpyAsync(B->d_rargs, B->h_rargs.data(), sizeof(dl_grad_args) * B->n, hipMemcpyHostToDevice, st));
  if (!B->h_cert.empty())
    DL_HIP_TRY(hipMemcpyAsync(B->d_cert, B->h_cert.data(), sizeof(bcert) * B->h_cert.size(), hipMemcpyHostToDevice,
                              st));
  if (!B->h_wgs.empty())
    DL_HIP_TRY(hipMemcpyAsync(B->d_wgs, B->h_wgs.data(), sizeof(dl_wg_desc) * B->h_wgs.size(), hipMemcpyHostToDevice,
                              st));
  if (!B->h_upd.empty())
    DL_HIP_TRY(hipMemcpyAsync(B->d_upd, B->h_upd.data(), sizeof(bupd) * B->h_upd.size(), hipMemcpyHostToDevice, st));
  if (!B->h_blk.empty())
    DL_HIP_TRY(hipMemcpyAsync(B->d_blk, B->h_blk.data(), sizeof(bblk) * B->h_blk.size(), hipMemcpyHostToDevice, st));
  if (!B->h_red.empty())
    DL_HIP_TRY(hipMemcpyAsync(B->d_red, B->h_red.data(), sizeof(bred) * B->h_red.size(), hipMemcpyHostToDevice, st));
  DL_HIP_TRY(hipStreamSynchronize(st));  // host tables must outlive the copies
  return DL_OK;
}

// Turns the per-workgroup clock stamps of the batched pass on or off (the
// stamps of live position q start at workgroup wg_first[q] of the buffer).
static dl_status set_clocking(dl_batch* B, bool on) {
  for (size_t q = 0; q < B->live.size(); ++q)
    B->h_args[B->live[q]].wg_clock = on ? B->d_clock + 2 * B->wg_first[q] : nullptr;
  DL_HIP_TRY(hipMemcpyAsync(B->d_args, B->h_args.data(), sizeof(dl_grad_args) * B->n, hipMemcpyHostToDevice,
                            B->stream));
  DL_HIP_TRY(hipStreamSynchronize(B->stream));
  return DL_OK;
}

// Grows the clock-stamp buffer to two entries per workgroup of the largest grid
// the tuner tries.
static dl_status ensure_clock(dl_batch* B, size_t need) {
  if (need <= B->clock_cap) return DL_OK;
  DL_HIP_TRY(hipStreamSynchronize(B->stream));
  if (B->d_clock) DL_HIP_TRY(hipFree(B->d_clock));
  B->d_clock = nullptr;
  B->clock_cap = 0;
  DL_HIP_TRY(hipMalloc((void**)&B->d_clock, need * sizeof(unsigned long long)));
  B->clock_cap = need;
  return DL_OK;
}

// The measured profile of the current tables: each live instance's workgroup
// ranges and their durations.
static std::vector<dl_inst_profile> profile_of(const dl_batch* B, const std::vector<double>& dur) {
  std::vector<dl_inst_profile> pr = B->prof;
  for (size_t q = 0; q < B->live.size(); ++q) {
    const int i = B->live[q];
    const size_t f = B->wg_first[q];
    const size_t e = (q + 1 < B->live.size()) ? B->wg_first[q + 1] : B->h_wgs.size();
    dl_inst_profile p;
    if (e > f) {
      for (size_t w = f; w < e; ++w) {
        p.b.push_back(B->h_wgs[w].t0);
        p.ticks.push_back(dur[w]);
      }
      p.b.push_back(B->h_wgs[e - 1].t1);
    }
    pr[(size_t)i] = p;
  }
  return pr;
}

static double wg_imbalance(const std::vector<double>& d) {
  if (d.empty()) return 1.0;
  double mx = 0.0, sum = 0.0;
  for (double v : d) {
    mx = std::max(mx, v);
    sum += v;
  }
  return sum > 0 ? mx / (sum / (double)d.size()) : 1.0;
}

// The batch tuner.  It times the solve's own iterations, so it costs no extra
// gradient passes: each trial configuration serves kTrialIters consecutive
// iterations with per-workgroup clock stamps on and HIP events around them.
// The trials are, for grids of 4, 2 and 1 workgroups per compute unit, the
// cost-model split followed by `rounds` splits re-dealt from the previous
// trial's measured workgroup times.  After the last trial the fastest
// configuration serves the rest of the solve.  A split never changes an
// iterate, so the trials differ only in time per iteration.
struct loop_tuner {
  static constexpr int kTrialIters = 4;
  static constexpr int kGrids = 3;
  static int grid_wpc(int g) { return 4 >> g; }
  int rounds = 0;
  bool running = false;
  int grid = 0, round = 0, left = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<dl_inst_profile> start, best;
  int best_wpc = 4;
  double best_ms = 1e300, best_imb = 1.0;
  // iterations one tuning takes
  static int64_t span(int rounds) { return (int64_t)kGrids * (1 + rounds) * kTrialIters; }
  ~loop_tuner() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// Builds the tables of the current trial configuration and starts its timing.
static dl_status trial_begin(dl_batch* B, loop_tuner& T, double gamma) {
  DL_TRY(build_tables(B, B->live, gamma));
  DL_TRY(set_clocking(B, true));
  DL_HIP_TRY(hipEventRecord(T.e0, B->stream));
  T.left = loop_tuner::kTrialIters;
  return DL_OK;
}

static dl_status tuner_start(dl_batch* B, loop_tuner& T, double gamma, int rounds) {
  memset(&B->tune, 0, sizeof(B->tune));
  T.rounds = rounds;
  if (!T.e0) DL_HIP_TRY(hipEventCreate(&T.e0));
  if (!T.e1) DL_HIP_TRY(hipEventCreate(&T.e1));
  DL_TRY(ensure_clock(B, 2 * (size_t)std::max<int>((int)B->live.size(), B->n_cu * loop_tuner::grid_wpc(0))));
  T.start = B->prof;
  T.best = B->prof;
  T.best_wpc = B->wg_per_cu;
  T.best_ms = 1e300;
  T.grid = 0;
  T.round = 0;
  B->wg_per_cu = loop_tuner::grid_wpc(0);
  T.running = true;
  return trial_begin(B, T, gamma);
}

// Ends the current trial (after its last iteration was enqueued): reads its
// time and workgroup durations, then starts the next trial or keeps the best.
static dl_status trial_end(dl_batch* B, loop_tuner& T, double gamma) {
  DL_HIP_TRY(hipEventRecord(T.e1, B->stream));
  std::vector<unsigned long long> clk(2 * (size_t)B->n_wg);
  if (B->n_wg > 0)
    DL_HIP_TRY(hipMemcpyAsync(clk.data(), B->d_clock, sizeof(unsigned long long) * clk.size(), hipMemcpyDeviceToHost,
                              B->stream));
  DL_HIP_TRY(hipStreamSynchronize(B->stream));
  float t = 0.f;
  DL_HIP_TRY(hipEventElapsedTime(&t, T.e0, T.e1));
  const double ms = (double)t / loop_tuner::kTrialIters;
  std::vector<double> dur((size_t)B->n_wg);
  for (size_t w = 0; w < dur.size(); ++w) dur[w] = (double)(clk[2 * w + 1] - clk[2 * w]);
  const double imb = wg_imbalance(dur);
  dl_tune_result& out = B->tune;
  if (T.grid == 0 && T.round == 0) {
    out.pass_ms_model = ms;
    out.imbalance_model = imb;
  }
  if (ms < T.best_ms) {
    T.best_ms = ms;
    T.best_imb = imb;
    T.best = B->prof;
    T.best_wpc = B->wg_per_cu;
  }
  if (T.round < T.rounds) {
    B->prof = profile_of(B, dur);
    ++T.round;
  } else if (T.grid + 1 < loop_tuner::kGrids) {
    ++T.grid;
    T.round = 0;
    B->wg_per_cu = loop_tuner::grid_wpc(T.grid);
    B->prof = T.start;
  } else {
    T.running = false;
    B->wg_per_cu = T.best_wpc;
    B->prof = T.best;
    DL_TRY(build_tables(B, B->live, gamma));
    out.rounds = T.rounds;
    out.pass_ms_tuned = T.best_ms;
    out.imbalance_tuned = T.best_imb;
    out.n_workgroups = B->n_wg;
    return DL_OK;
  }
  return trial_begin(B, T, gamma);
}

// Stops a tuning that the live set changed under: the best configuration
// timed so far (or the one running) serves on; build_tables follows.
static void tuner_abort(dl_batch* B, loop_tuner& T) {
  if (!T.running) return;
  T.running = false;
  if (T.best_ms < 1e300) {
    B->wg_per_cu = T.best_wpc;
    B->prof = T.best;
    B->tune.rounds = T.rounds;
    B->tune.pass_ms_tuned = T.best_ms;
    B->tune.imbalance_tuned = T.best_imb;
  }
}

// Certificates of every live member at once (the tables must be current): the
// scale pass at lam, one batched histogram + objective pass, the slot
// reduction, A x, the item part, one batched repair pass, the final sums, one
// copy to the host.  stats[i] of each live member i gets its certificate and
// status (DL_OK when it is finite; the gap test is the caller's).
static dl_status batch_certify(dl_batch* B, double gamma, dl_solve_stats* stats, std::vector<dl_status>& cs) {
  hipStream_t st = B->stream;
  const int nl = (int)B->live.size();
  const dl_problem* P0 = B->probs[B->live[0]];
  DL_TRY(dl_launch_qscale_batch(B->d_cargs, B->n, st));
  DL_TRY(dl_launch_grad_batch(P0, B->n_wg, B->d_cargs, B->d_wgs, B->lds, st, M_HIST | M_OBJ | (B->glob ? M_GLOB : 0)));
  if (B->n_red > 0) hipLaunchKernelGGL(reduce_batch, dim3(B->n_red), dim3(256), 0, st, B->d_upd, B->d_red);
  hipLaunchKernelGGL(cert_decode_batch, dim3(B->n_blk), dim3(256), 0, st, B->d_upd, B->d_blk);
  hipLaunchKernelGGL(cert_items_batch, dim3(nl), dim3(1024), 0, st, B->d_cert);
  DL_HIP_TRY(hipGetLastError());
  DL_TRY(dl_launch_grad_batch(P0, B->n_wg, B->d_rargs, B->d_wgs, B->lds_rep, st, M_REPAIR));
  hipLaunchKernelGGL(cert_final_batch, dim3(nl), dim3(1024), 0, st, B->d_cert, B->d_cres);
  DL_HIP_TRY(hipGetLastError());
  DL_HIP_TRY(hipMemcpyAsync(B->h_cres, B->d_cres, sizeof(double) * 5 * (size_t)nl, hipMemcpyDeviceToHost, st));
  DL_HIP_TRY(hipStreamSynchronize(st));
  cs.assign(B->n, DL_OK);
  for (int q = 0; q < nl; ++q) {
    const int i = B->live[q];
    memset(&stats[i], 0, sizeof(stats[i]));
    const double* c = B->h_cres + 5 * (size_t)q;
    cs[i] = dl_cert_stats(c, c[4] != 0.0, gamma, B->probs[i]->eq_mask, &stats[i]);
    stats[i].status = cs[i];
  }
  return DL_OK;
}

extern "C" dl_status dl_batch_create(int32_t n, dl_problem* const* probs, dl_batch** out) {
  DL_CHECK_ARG(out, "out is NULL");
  *out = nullptr;
  DL_CHECK_ARG(n >= 1 && probs, "need at least one problem");
  for (int i = 0; i < n; ++i) DL_CHECK_ARG(probs[i], "NULL problem in batch");
  for (int i = 0; i < n; ++i)
    if (probs[i]->tile_rows > 0) {
      dl_set_error("batch members must hold their whole histogram in one window (n_families * n_items <= 13000)");
      return DL_EUNSUPPORTED;
    }
  // each member keeps per-pass state (fixed-point scales, partial slots) in its problem
  for (int i = 0; i < n; ++i)
    for (int k = i + 1; k < n; ++k) DL_CHECK_ARG(probs[i] != probs[k], "a problem appears twice in the batch");
  const dl_problem* P0 = probs[0];
  for (int i = 1; i < n; ++i) {
    const dl_problem* P = probs[i];
    if (P->device != P0->device || P->stream != P0->stream || P->mf != P0->mf || P->has_a != P0->has_a ||
        P->storage != P0->storage || P->kmax != P0->kmax) {
      dl_set_error("batch members must share device, stream, storage and kernel variant (families, stored a)");
      return DL_EUNSUPPORTED;
    }
  }
  dl_batch* B = new (std::nothrow) dl_batch();
  if (!B) {
    dl_set_error("host allocation failed");
    return DL_ENOMEM;
  }
  B->n = n;
  B->probs.assign(probs, probs + n);
  B->stream = P0->stream;
  B->prof.assign((size_t)n, dl_inst_profile());
  B->model_tot.assign((size_t)n, 0.0);
  B->cmodel.assign((size_t)n, std::vector<double>());
  for (int i = 0; i < n; ++i) {
    const std::vector<float>& tc = probs[i]->task_cost;
    std::vector<double>& c = B->cmodel[(size_t)i];
    c.assign(tc.size() + 1, 0.0);
    for (size_t t = 0; t < tc.size(); ++t) c[t + 1] = c[t] + tc[t];
    B->model_tot[(size_t)i] = c.back();
  }
  memset(&B->tune, 0, sizeof(B->tune));
  auto fail = [&](dl_status s) {
    free_batch(B);
    return s;
  };
  if (hipDeviceGetAttribute(&B->n_cu, hipDeviceAttributeMultiprocessorCount, P0->device) != hipSuccess) {
    dl_set_error("hipDeviceGetAttribute failed");
    return fail(DL_EHIP);
  }
  if (hipMalloc((void**)&B->d_args, sizeof(dl_grad_args) * n) != hipSuccess ||
      hipMalloc((void**)&B->d_cargs, sizeof(dl_grad_args) * n) != hipSuccess ||
      hipMalloc((void**)&B->d_rargs, sizeof(dl_grad_args) * n) != hipSuccess ||
      hipMalloc((void**)&B->d_cert, sizeof(bcert) * n) != hipSuccess ||
      hipMalloc((void**)&B->d_cres, sizeof(double) * 5 * n) != hipSuccess ||
      hipHostMalloc((void**)&B->h_cres, sizeof(double) * 5 * n, hipHostMallocDefault) != hipSuccess) {
    dl_set_error("device or pinned host allocation failed");
    return fail(DL_ENOMEM);
  }
  *out = B;
  return DL_OK;
}

extern "C" void dl_batch_destroy(dl_batch* B) { free_batch(B); }

extern "C" dl_status dl_batch_get_tune(const dl_batch* B, dl_tune_result* out) {
  DL_CHECK_ARG(B && out, "NULL argument");
  *out = B->tune;
  return DL_OK;
}

extern "C" dl_status dl_batch_solve(dl_batch* B, const dl_solve_opts* o, const double* const* lambda0,
                                    double* const* lambda_out, dl_solve_stats* stats) {
  DL_CHECK_ARG(B && o && lambda_out && stats, "NULL argument");
  DL_CHECK_ARG(o->n_stages >= 1 && o->gammas && o->iters, "empty schedule");
  for (int s = 0; s < o->n_stages; ++s) {
    DL_CHECK_ARG(o->gammas[s] > 0.0 && isfinite(o->gammas[s]), "gamma must be positive and finite");
    DL_CHECK_ARG(o->iters[s] >= 0 || s == o->n_stages - 1, "only the last stage may run until tol");
  }
  for (int i = 0; i < B->n; ++i) DL_CHECK_ARG(lambda_out[i], "NULL lambda_out entry");
  DL_CHECK_ARG(o->max_iters >= 0 && o->check_every >= 0 && o->autotune_rounds >= 0, "negative limits");
  const double step_scale = o->step_scale > 0.0 ? o->step_scale : 1.0;
  auto t0 = std::chrono::steady_clock::now();
  // every solve starts from the cost-model split, 4 workgroups per compute unit
  B->prof.assign((size_t)B->n, dl_inst_profile());
  B->wg_per_cu = 4;
  memset(&B->tune, 0, sizeof(B->tune));
  for (dl_solver* s : B->solvers) dl_solver_destroy(s);
  B->solvers.assign(B->n, nullptr);
  for (int i = 0; i < B->n; ++i) memset(&stats[i], 0, sizeof(stats[i]));
  for (int i = 0; i < B->n; ++i) {
    const dl_status cs = dl_solver_create(B->probs[i], lambda0 ? lambda0[i] : nullptr, &B->solvers[i]);
    if (cs != DL_OK) {
      for (dl_solver* s : B->solvers) dl_solver_destroy(s);
      B->solvers.clear();
      return cs;
    }
  }
  // every member's accumulator starts at zero (each reader of a reduction clears it)
  for (int i = 0; i < B->n; ++i)
    if (hipMemsetAsync(B->probs[i]->acc, 0, sizeof(unsigned long long) * (size_t)B->probs[i]->nrow(), B->stream) !=
        hipSuccess) {
      for (dl_solver* s : B->solvers) dl_solver_destroy(s);
      B->solvers.clear();
      dl_set_error("hipMemsetAsync failed");
      return DL_EHIP;
    }
  std::vector<int> live(B->n);
  std::iota(live.begin(), live.end(), 0);
  std::vector<char> done(B->n, 0);
  std::vector<int64_t> iters(B->n, 0), checks(B->n, 0);
  std::vector<int> last_stage(B->n, 0);
  dl_status rc = DL_OK;
  int64_t total = 0;
  constexpr int64_t kTuneStart = 10;
  loop_tuner tuner;
  bool tuned = false;
  for (int stage = 0; stage < o->n_stages && rc == DL_OK && !live.empty(); ++stage) {
    const double gamma = o->gammas[stage];
    for (int i : live) {
      rc = dl_solver_set_stage(B->solvers[i], gamma, step_scale, stage == 0 ? 1 : o->reset_momentum);
      if (rc != DL_OK) break;
      last_stage[i] = stage;
    }
    if (rc != DL_OK) break;
    rc = build_tables(B, live, gamma);
    if (rc != DL_OK) break;
    const bool last = stage == o->n_stages - 1;
    const int64_t n_it = o->iters[stage];
    double tk = 1.0;
    int64_t k = 0;
    // the tuner runs once, from iteration 10 of the first stage long enough to hold it
    int64_t tune_at = -1;
    if (o->autotune_rounds > 0 && !tuned &&
        (n_it < 0 || n_it >= kTuneStart + loop_tuner::span(o->autotune_rounds))) {
      tune_at = kTuneStart;
      tuned = true;
    }
    while ((n_it < 0 || k < n_it) && total < o->max_iters && !live.empty()) {
      if (k == tune_at) {
        rc = tuner_start(B, tuner, gamma, o->autotune_rounds);
        if (rc != DL_OK) break;
      }
      rc = dl_launch_qscale_batch(B->d_args, B->n, B->stream);
      if (rc != DL_OK) break;
      rc = dl_launch_grad_batch(B->probs[live[0]], B->n_wg, B->d_args, B->d_wgs, B->lds, B->stream,
                                M_HIST | (B->glob ? M_GLOB : 0));
      if (rc != DL_OK) break;
      const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tk * tk));
      const double beta = (tk - 1.0) / tn;
      tk = tn;
      if (B->n_red > 0)
        hipLaunchKernelGGL(reduce_batch, dim3(B->n_red), dim3(256), 0, B->stream, B->d_upd, B->d_red);
      hipLaunchKernelGGL(update_batch, dim3(B->n_blk), dim3(256), 0, B->stream, B->d_upd, B->d_blk, gamma,
                         step_scale, beta);
      if (hipGetLastError() != hipSuccess) {
        dl_set_error("update_batch launch failed");
        rc = DL_EHIP;
        break;
      }
      ++k;
      ++total;
      for (int i : live) ++iters[i];
      if (tuner.running && --tuner.left == 0) {
        rc = trial_end(B, tuner, gamma);
        if (rc != DL_OK) break;
      }
      if (last && o->check_every > 0 && k % o->check_every == 0) {
        // every live member's certificate in batched launches, one synchronisation
        std::vector<dl_status> cst;
        rc = batch_certify(B, gamma, stats, cst);
        if (rc != DL_OK) break;
        std::vector<int> keep;
        for (int i : live) {
          const dl_status cs = cst[i];
          ++checks[i];
          if (cs != DL_OK) {
            stats[i].status = cs;
            done[i] = 1;
            continue;
          }
          if (stats[i].rel_gap <= o->tol) {
            stats[i].status = DL_OK;
            done[i] = 1;
          } else {
            keep.push_back(i);
          }
        }
        if (keep.size() != live.size()) {
          tuner_abort(B, tuner);
          live = keep;
          if (!live.empty()) {
            rc = build_tables(B, live, gamma);
            if (rc != DL_OK) break;
          }
        }
      }
      if (n_it < 0 && o->check_every == 0 && total >= o->max_iters) break;
    }
  }
  for (int i = 0; i < B->n && rc == DL_OK; ++i) {
    if (!done[i]) {
      dl_status cs = dl_solver_certificate(B->solvers[i], &stats[i]);
      ++checks[i];
      stats[i].status = (cs == DL_OK) ? (stats[i].rel_gap <= o->tol ? DL_OK : DL_NOT_CONVERGED) : cs;
    }
    dl_status ls = dl_solver_get_lambda(B->solvers[i], lambda_out[i]);
    if (ls != DL_OK) rc = ls;
  }
  if (rc == DL_OK && hipStreamSynchronize(B->stream) != hipSuccess) {
    dl_set_error("hipStreamSynchronize failed");
    rc = DL_EHIP;
  }
  const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  bool all_ok = true;
  for (int i = 0; i < B->n; ++i) {
    stats[i].iters = iters[i];
    stats[i].stage = last_stage[i];
    stats[i].n_checks = checks[i];
    stats[i].wall_ms = wall;
    if (stats[i].status != DL_OK) all_ok = false;
  }
  for (dl_solver* s : B->solvers) dl_solver_destroy(s);
  B->solvers.clear();
  if (rc != DL_OK) return rc;
  return all_ok ? DL_OK : DL_NOT_CONVERGED;
}
