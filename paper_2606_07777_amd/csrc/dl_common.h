// Internal declarations of the gfx950 dual-ascent library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dualip.h"

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void dl_set_error(const std::string& msg);

#define DL_HIP_TRY(expr)                                                              \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      dl_set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                \
      return (e_ == hipErrorOutOfMemory) ? DL_ENOMEM : DL_EHIP;                       \
    }                                                                                 \
  } while (0)

#define DL_CHECK_ARG(cond, msg)   \
  do {                            \
    if (!(cond)) {                \
      dl_set_error(msg);          \
      return DL_EINVAL;           \
    }                             \
  } while (0)

#define DL_TRY(expr)              \
  do {                            \
    dl_status s_ = (expr);        \
    if (s_ < 0) return s_;        \
  } while (0)

// ---------------------------------------------------------------------------
// Layout constants
// ---------------------------------------------------------------------------
constexpr int DL_WG = 1024;              // gradient-pass workgroup size (16 wavefronts)
constexpr int DL_WAVES = DL_WG / 64;
constexpr int DL_MAX_BUCKETS = 8;
constexpr int DL_LONG = 7;               // bucket code of rows longer than 64*KMAX
constexpr int DL_MAX_MJ = 13000;         // m*J that fits the LDS accumulation (12 B per entry)
// Larger coupling blocks keep every dual row in LDS and split the histogram
// rows into windows that fit beside them (the M_TILE mode): one launch per
// window, each pass recomputing x and keeping the contributions to its rows.
// Limits: DL_MAX_ITEMS items (16-bit item offsets) and LDS for the dual rows
// plus, in the certificate's repair pass, one factor per item.
constexpr int DL_MAX_ITEMS = 16383;
constexpr size_t DL_LDS_BYTES = 160 * 1024;
constexpr int DL_MAX_FAMILIES = 4;
static_assert(4 * DL_MAX_ITEMS <= 0xFFFF, "item byte offsets 4 j are stored in 16 bits");
// Elements per lane in the group path: the one-family kernel (a stored or not),
// and the multi-family kernels, whose coefficient registers need the room.
#ifndef DL_KMAX_PLAIN
#define DL_KMAX_PLAIN 12
#endif
constexpr int DL_KMAX_A = 8;
// Element loops of the group path step in chunks: loads in chunks of 4, the
// arithmetic in chunks of DL_CHUNK (a divisor of 4); a chunk runs when its
// first element is below the task's per-lane count.
#ifndef DL_CHUNK
#define DL_CHUNK 4
#endif
// Elements of zero padding after idx, c and every stored a family: a group of
// lanes may read up to 64*KMAX + 63 elements past a row start without
// predication, and masks what lies past the row.
constexpr int64_t DL_PAD = 4096;
// Register slots per lane a row of degree d needs when served by 2^glog lanes
// (chunks of four consecutive elements from the row start rounded down to a
// multiple of four, so up to three leading slots belong to the previous row).
__host__ __device__ inline int64_t dl_slots(int64_t d, int glog) {
  return 4 * ((d + 3 + (4LL << glog) - 1) >> (glog + 2));
}
// Element stride between stored a families (a multiple of 64, so every
// family's chunks stay as aligned as the c and idx arrays').
__host__ __device__ inline int64_t dl_astride(int64_t nnz) { return ((nnz + 63) & ~(int64_t)63) + DL_PAD; }

// A degree bucket: users [user_begin, user_end) of the reordered problem (sorted
// by degree, longest first) served by groups of 2^glog lanes, 64/2^glog users
// per wavefront task; glog == DL_LONG serves one user per task with a
// wavefront-wide loop over the row.
struct dl_bucket {
  int64_t task_begin;
  int64_t user_begin;
  int64_t user_end;
  int32_t glog;
  int32_t pad;
};

enum : int {
  M_HIST = 1,    // accumulate A x into the per-workgroup fixed-point histogram
  M_OBJ = 2,     // accumulate the per-user Lagrangian terms (FP64 per workgroup)
  M_REPAIR = 4,  // accumulate c.x~ + gamma/2 x~^2 with x~ = r_j x (certificate)
  M_VIN = 8,     // v given in caller order (ProjectionMap), no gather
  M_XOUT = 16,   // write x in the caller's order
  M_GLOB = 32,   // with M_HIST: also count sum x for the global-count row
  M_TILE = 64,   // with M_HIST: keep only the histogram rows of the launch's window (tile_b0, tile_bn)
};

struct dl_grad_args {
  // reordered instance
  const int64_t* rp;       // I_new + 1
  const uint16_t* idx;     // nnz item byte offsets 4 j (see dl_problem::idx)
  const void* cval;        // nnz, float or bf16
  const void* aval;        // n_stored * nnz
  const int64_t* orig_rp;  // per reordered user: row start in the caller's order
  int64_t nnz;
  int64_t astride;         // elements between stored a families (dl_astride(nnz))
  int32_t J, m;
  int32_t a_slot[DL_MAX_FAMILIES];  // stored slot of family k, -1: a == 1
  float qscale[DL_MAX_FAMILIES];    // coarsest fixed-point scale of family k (max|a_k| * radius)
  const float* qs_dev;              // m, device: this pass's scales (>= qscale), or NULL
  const unsigned* ext;              // per-item extremes, encoded: [max(0,-c)][max|c|][max a, max -a per stored slot], J each
  // tasks
  const int64_t* wg_task;           // n_wg + 1
  int32_t n_buckets;
  int32_t proj;                     // dl_proj_kind
  dl_bucket bk[DL_MAX_BUCKETS];
  float radius;
  float upper;                      // u of the box-cut set
  // iteration inputs
  float neg_inv_gamma;
  float gamma;
  int32_t glob;                     // 1: a global-count row (dual mu[m*J], count into part[.. + m*J])
  int32_t tile_b0, tile_bn;         // M_TILE: the window of histogram rows, in bytes (8 per row)
  const float* mu;                  // n_rows, lam in problem units (FP32)
  const float* rfac;                // J, repair factor (M_REPAIR)
  const float* v_in;                // nnz caller order (M_VIN)
  // outputs
  unsigned long long* part;         // n_wg * n_rows (n_rows = m*J + glob)
  double* obj_part;                 // n_wg
  float* x_out;                     // nnz caller order, nullable
  unsigned long long* wg_clock;     // nullable: per slot (start, end) steady-clock ticks
};

// Workgroup descriptor of a batched pass: tasks [t0, t1) of instance inst,
// histogram into that instance's partial slot.
struct dl_wg_desc {
  int32_t inst;
  int32_t slot;
  int64_t t0, t1;
};

struct dl_problem {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t I = 0, I_active = 0, nnz = 0;
  int32_t J = 0, m = 0, proj = 0, storage = 0, jacobi = 0;
  double radius = 1.0;
  double upper = 0.0;    // u of the box-cut set
  int32_t eq_mask = 0;   // bit k: family k holds equality rows (free duals)
  int32_t glob = 0;      // 1: one global-count row sum x <= gcap, dual coordinate m*J
  int32_t tile_rows = 0;  // m*J > DL_MAX_MJ: histogram rows per window (M_TILE), else 0
  int32_t n_tiles = 1;    // launches per histogram pass
  double gcap = 0.0;
  int64_t nrow() const { return (int64_t)m * J + glob; }
  int kmax = 16;
  int mf = 1;            // compiled family bound of the kernel variant (1, 2 or 4)
  bool has_a = false;    // at least one stored family
  int n_stored = 0;
  int a_slot[DL_MAX_FAMILIES] = {-1, -1, -1, -1};
  float qscale[DL_MAX_FAMILIES] = {0, 0, 0, 0};
  int32_t max_degree = 0;
  // per-item extremes of the stored values (order-preserving uint encoding):
  // [max(0, -c) over the item's users], [max |c|], then per stored slot [max a], [max -a]
  unsigned* ext = nullptr;
  float* qs_dev = nullptr;   // fixed-point scales of the last histogram pass: the families', then
                             // the global-count row's at index DL_MAX_FAMILIES
  unsigned* qs_words = nullptr;  // the scale kernel's pass-wide maxima (5 float bit patterns, zero between launches)
  unsigned* qs_cnt = nullptr;    // its arrival counter (zero between launches)

  // reordered device layout
  int64_t* rp = nullptr;
  uint16_t* idx = nullptr;   // item of every element as the byte offset 4 j (J <= DL_MAX_ITEMS)
  void* cval = nullptr;
  void* aval = nullptr;
  int64_t* orig_rp = nullptr;

  // task table
  std::vector<dl_bucket> buckets;
  int64_t n_tasks = 0;
  int n_wg = 0;          // workgroups of the current partition
  int n_wg_cap = 0;      // partial-sum slots allocated
  int n_cu = 0;
  int64_t* wg_task = nullptr;              // n_wg_cap + 1
  std::vector<float> task_cost;            // cost-model weight of every task
  unsigned long long* wg_clock = nullptr;  // 2 * n_wg_cap
  bool clocking = false;

  // item space (device)
  double* b = nullptr;       // n_rows (the global cap last)
  double* D = nullptr;       // n_rows Jacobi scaling (1 without Jacobi)
  double lhat = 1.0;
  std::vector<double> b_host, D_host;

  // per-pass scratch (device)
  unsigned long long* part = nullptr;  // n_wg * n_rows
  unsigned long long* acc = nullptr;   // n_rows reduced sums, zero between passes
  double* obj_part = nullptr;          // n_wg
  double* pobj_part = nullptr;         // n_wg
  float* mu = nullptr;                 // n_rows
  float* rfac = nullptr;               // J
  double* lam_tmp = nullptr;           // n_rows
  double* cert_out = nullptr;          // 8 doubles
  int* upd_flag = nullptr;             // dl_problem_update's non-finite flag
  double* cert_host = nullptr;         // pinned, 16 doubles: certificate values [0..3], its flag word at [8]
  double device_bytes = 0;
};

// Gradient pass and projection launches (dl_grad.hip).
// A histogram pass first sets its fixed-point scales (dl_launch_qscale) unless
// the caller has just done so for the same mu and gamma (scaled = true).
dl_status dl_launch_grad(const dl_problem* P, int mode, const float* mu, double gamma,
                         const float* rfac, const float* v_in, float* x_out, double* obj_part, bool scaled = false);
size_t dl_grad_lds_bytes(const dl_problem* P, int mode);
dl_grad_args dl_make_grad_args(const dl_problem* P, const float* mu, double gamma);
// Task ranges of n_wg workgroups with equal cost-model weight.
std::vector<int64_t> dl_model_partition(const dl_problem* P, int n_wg);
dl_status dl_set_partition(dl_problem* P, const std::vector<int64_t>& bounds);
// mode: M_HIST (| M_GLOB when some member has a global-count row) for an iteration,
// M_HIST | M_OBJ (| M_GLOB) and M_REPAIR for the certificate's two passes
dl_status dl_launch_grad_batch(const dl_problem* P, int n_wg, const dl_grad_args* d_args, const dl_wg_desc* d_wgs,
                               size_t lds, hipStream_t st, int mode);
dl_status dl_grad_prepare(const dl_problem* P);
// Fixed-point scales for a histogram pass at gather point mu (into P->qs_dev),
// and the same for every instance of a batched pass (one block per entry).
dl_status dl_launch_qscale(const dl_problem* P, const float* mu, double gamma);
dl_status dl_launch_qscale_batch(const dl_grad_args* d_args, int n, hipStream_t st);
// (Re)computes P->ext from the stored layout; c_only: only the two c columns.
dl_status dl_item_extremes(dl_problem* P, bool c_only);

// Order-preserving encoding of floats as unsigned (max of codes = code of max).
__host__ __device__ inline unsigned dl_ord_enc(float f) {
  unsigned u;
  __builtin_memcpy(&u, &f, 4);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float dl_ord_dec(unsigned e) {
  unsigned u = (e & 0x80000000u) ? (e & 0x7FFFFFFFu) : ~e;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}
constexpr unsigned DL_ORD_NEG_INF = 0x007FFFFFu;  // dl_ord_enc(-inf)

// BF16 helpers (storage form: c and a in bfloat16, FP32 arithmetic).
__host__ __device__ inline uint16_t dl_f32_to_bf16_rne(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}
