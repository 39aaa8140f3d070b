// Kernels of the gradient pass, as templates over the kernel variant: compiled
// once per variant (families class, stored a, storage type) by dl_grad_variant.hip.
#pragma once

#include <type_traits>

#include "dl_common.h"

// Gradient pass of the dual ascent on gfx950 (one launch per evaluation).
//
// Computes, for every user i, v_i = -(c_i + sum_k a_ki * lam_k[items of i]) / gamma
// and x_i = Pi_{C_i}(v_i) (eq. 3), then the per-item sums (A_k x)_j that give the
// gradient A x - b (eq. 4).  The paper evaluates these as two sparse products
// around a bucketed, fused simplex projection (Sections 4.1-4.3); here the three
// are one streaming pass over the user-major CSR:
//
//  * each workgroup (1024 lanes, one per CU) stages lam (m*J FP32, times
//    -1/gamma) in LDS once and gathers from there;
//  * users are reordered by degree, longest first, and served by groups of
//    G = 2^glog lanes holding up to KMAX elements each in registers; G is a
//    compile-time constant per degree bucket so every load of a row uses an
//    immediate offset, and the arrays carry zero padding so loads past a row
//    end need no predication (masked by select); rows longer than 64*KMAX use
//    a wavefront-wide loop over the row;
//  * each wavefront prefetches the next task's row pointers and row data while
//    it computes the current task (software pipelining);
//  * the simplex threshold: one pass keeps the three largest entries and the
//    positive sum; then the paper's early exit when the positive part already
//    fits, an exact exit when the largest entry leads the second by at least z,
//    an exact exit when the two largest carry z with the third at or below
//    their threshold, otherwise Newton steps from below on f(theta) =
//    sum max(v-theta,0) - z (each step is the exact threshold of the current
//    active set; the pass that forms it also checks whether the set survives
//    the step);
//  * a_k * x is rounded to a per-family fixed-point grid and added with 64-bit
//    integer LDS atomics into a per-workgroup histogram over items; integer
//    addition is associative, so the sums are bitwise reproducible for any
//    schedule and no float atomics are used; the histogram is written once per
//    workgroup and summed over workgroups by the update kernel.
namespace {

// Lane permutation within rows of 16 (every lane reads a valid source lane, so
// bound_ctrl is immaterial; it lets the compiler fold the move into the DPP
// form of the arithmetic instruction that consumes it).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ float swz_xor16(float v) {
  // ds_swizzle bit mode: and_mask 0x1F, or_mask 0, xor_mask 0x10 (within 32 lanes)
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}

// One butterfly step of an all-reduce over aligned groups of 2^(STEP+1) lanes.
template <int STEP>
__device__ __forceinline__ float xstep(float v) {
  if constexpr (STEP == 0) return dpp_f<0xB1>(v);   // quad_perm(1,0,3,2): lane ^ 1
  if constexpr (STEP == 1) return dpp_f<0x4E>(v);   // quad_perm(2,3,0,1): lane ^ 2
  if constexpr (STEP == 2) return dpp_f<0x141>(v);  // row_half_mirror: pairs the two quads of 8
  if constexpr (STEP == 3) return dpp_f<0x140>(v);  // row_mirror: pairs the two halves of 16
  if constexpr (STEP == 4) return swz_xor16(v);
  return __shfl_xor(v, 32, 64);
}

// All-reduce (sum / max / min) over aligned groups of 2^GLOG lanes.  Every lane
// of a group ends with the same bits (each step combines the same two operands).
template <int GLOG>
__device__ __forceinline__ float gsum(float v) {
  if constexpr (GLOG > 0) v += xstep<0>(v);
  if constexpr (GLOG > 1) v += xstep<1>(v);
  if constexpr (GLOG > 2) v += xstep<2>(v);
  if constexpr (GLOG > 3) v += xstep<3>(v);
  if constexpr (GLOG > 4) v += xstep<4>(v);
  if constexpr (GLOG > 5) v += xstep<5>(v);
  return v;
}
template <int GLOG>
__device__ __forceinline__ float gmax(float v) {
  if constexpr (GLOG > 0) v = fmaxf(v, xstep<0>(v));
  if constexpr (GLOG > 1) v = fmaxf(v, xstep<1>(v));
  if constexpr (GLOG > 2) v = fmaxf(v, xstep<2>(v));
  if constexpr (GLOG > 3) v = fmaxf(v, xstep<3>(v));
  if constexpr (GLOG > 4) v = fmaxf(v, xstep<4>(v));
  if constexpr (GLOG > 5) v = fmaxf(v, xstep<5>(v));
  return v;
}
template <int GLOG>
__device__ __forceinline__ float gmin(float v) {
  if constexpr (GLOG > 0) v = fminf(v, xstep<0>(v));
  if constexpr (GLOG > 1) v = fminf(v, xstep<1>(v));
  if constexpr (GLOG > 2) v = fminf(v, xstep<2>(v));
  if constexpr (GLOG > 3) v = fminf(v, xstep<3>(v));
  if constexpr (GLOG > 4) v = fminf(v, xstep<4>(v));
  if constexpr (GLOG > 5) v = fminf(v, xstep<5>(v));
  return v;
}
// (largest, second largest) over the group
template <int STEP>
__device__ __forceinline__ void top2_step(float& m1, float& m2) {
  const float o1 = xstep<STEP>(m1), o2 = xstep<STEP>(m2);
  const float hi = fmaxf(m1, o1), lo = fminf(m1, o1);
  m2 = fmaxf(lo, fmaxf(m2, o2));
  m1 = hi;
}
// (largest, second, third) over the group: the k-th largest of two sorted
// triples a, b is the largest min(a_i, b_j) over i + j = k (a_0 = b_0 = +inf)
template <int STEP>
__device__ __forceinline__ void top3_step(float& m1, float& m2, float& m3) {
  const float o1 = xstep<STEP>(m1), o2 = xstep<STEP>(m2), o3 = xstep<STEP>(m3);
  const float n3 = fmaxf(fmaxf(m3, o3), fmaxf(fminf(m1, o2), fminf(m2, o1)));
  const float n2 = fmaxf(fmaxf(m2, o2), fminf(m1, o1));
  m1 = fmaxf(m1, o1);
  m2 = n2;
  m3 = n3;
}
template <int GLOG>
__device__ __forceinline__ void gtop3(float& m1, float& m2, float& m3) {
  if constexpr (GLOG > 0) top3_step<0>(m1, m2, m3);
  if constexpr (GLOG > 1) top3_step<1>(m1, m2, m3);
  if constexpr (GLOG > 2) top3_step<2>(m1, m2, m3);
  if constexpr (GLOG > 3) top3_step<3>(m1, m2, m3);
  if constexpr (GLOG > 4) top3_step<4>(m1, m2, m3);
  if constexpr (GLOG > 5) top3_step<5>(m1, m2, m3);
}
template <int GLOG>
__device__ __forceinline__ void gtop2(float& m1, float& m2) {
  if constexpr (GLOG > 0) top2_step<0>(m1, m2);
  if constexpr (GLOG > 1) top2_step<1>(m1, m2);
  if constexpr (GLOG > 2) top2_step<2>(m1, m2);
  if constexpr (GLOG > 3) top2_step<3>(m1, m2);
  if constexpr (GLOG > 4) top2_step<4>(m1, m2);
  if constexpr (GLOG > 5) top2_step<5>(m1, m2);
}

template <typename TV>
__device__ __forceinline__ float ldv(const TV* p);
template <>
__device__ __forceinline__ float ldv<float>(const float* p) {
  return *p;
}
template <>
__device__ __forceinline__ float ldv<uint16_t>(const uint16_t* p) {
  return __uint_as_float((uint32_t)(*p) << 16);
}

// The library stores item indices as byte offsets jb = 4 j (the offset of item
// j's word in an LDS array of 4-byte words), so an item's word is addressed
// without a shift; its 8-byte histogram word sits at byte 2 jb.
__device__ __forceinline__ float lds_word(const float* base, int byte_off) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + byte_off);
}

// Adds w = a x on the fixed-point grid 1/qs to the histogram word at byte
// offset rb (round to nearest, ties to even).
__device__ __forceinline__ void hist_add(unsigned long long* h, int rb, float w, float qs) {
  int q = __float2int_rn(w * qs);
  if (q != 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(h) + rb), (unsigned long long)(long long)q);
}

// FP32 to u32, truncating, with the hardware convert's saturation: negative
// values (and -inf) give 0.
__device__ __forceinline__ uint32_t cvt_u32_sat(float f) {
  uint32_t q;
  asm("v_cvt_u32_f32 %0, %1" : "=v"(q) : "v"(f));
  return q;
}

// Families with a == 1: adds x = max(w, 0), rounded half up on the grid, with one
// fused multiply-add and a saturating convert (w <= 0 adds nothing, as x = 0
// would); the 64-bit addend has a zero high word.
__device__ __forceinline__ void hist_add_pos(unsigned long long* h, int rb, float w, float qs) {
  const uint32_t q = cvt_u32_sat(fmaf(w, qs, 0.5f));
  if (q != 0) atomicAdd(reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(h) + rb), (unsigned long long)q);
}

// One contribution to the histogram.  In the window mode only rows inside the
// launch's window [tile_b0, tile_b0 + tile_bn) (bytes) are kept, at their offset
// in the window.
template <bool HAS_A, int MODE>
__device__ __forceinline__ void hist_put(unsigned long long* h, int rb, float w, float qs, const dl_grad_args& A) {
  if constexpr ((MODE & M_TILE) != 0) {
    rb -= A.tile_b0;
    if ((unsigned)rb >= (unsigned)A.tile_bn) return;
  }
  if constexpr (HAS_A) hist_add(h, rb, w, qs);
  else hist_add_pos(h, rb, w, qs);
}

// Per-lane accumulators of one pass: the FP64 objective terms, and the
// fixed-point count of the global-count row (sum x on the grid 1/qs_g).
struct LaneAcc {
  double obj = 0.0;
  unsigned long long gcnt = 0ull;
};
// Fixed-point scales of a pass: the families', then the global-count row's.
constexpr int DL_NQS = DL_MAX_FAMILIES + 1;

// ---------------------------------------------------------------------------
// Group path: 2^GLOG lanes per user, up to KMAX elements per lane.
// ---------------------------------------------------------------------------
// Per-lane element loops run in chunks of 4: a chunk runs when its first
// element is below the task's K (uniform), elements past the row end inside a
// chunk are masked.  Whole chunks let the compiler batch loads and LDS reads.
#define DL_FOR_K(k, KMAX, K)                                   \
  _Pragma("unroll") for (int kc_ = 0; kc_ < (KMAX); kc_ += 4)  \
    if (kc_ < (K))                                             \
      _Pragma("unroll") for (int k = kc_; k < kc_ + 4; ++k)
// Arithmetic loops: chunks of DL_CHUNK, or of 2 with stored a (whose larger
// register set would otherwise spill in the batched kernel).
template <bool HAS_A>
constexpr int chunk_of() { return HAS_A ? 2 : DL_CHUNK; }
#define DL_FOR_KC(k, KMAX, K)                                                             \
  _Pragma("unroll") for (int kc_ = 0; kc_ < (KMAX); kc_ += chunk_of<HAS_A>())             \
    if (kc_ < (K))                                                                        \
      _Pragma("unroll") for (int k = kc_; k < kc_ + chunk_of<HAS_A>(); ++k)

struct TaskMeta {
  int64_t s;   // row start (0 for lanes without a user)
  int64_t e;   // row end (0 for lanes without a user); the length is taken late so
               // the row-pointer load is not waited on where it is issued
  int64_t os;  // row start in the caller's order
};

template <int GLOG>
__device__ __forceinline__ TaskMeta load_meta(const dl_grad_args& A, const dl_bucket& B, int64_t t, int lane,
                                              bool need_os) {
  const int64_t u = B.user_begin + (t - B.task_begin) * (int64_t)(64 >> GLOG) + (lane >> GLOG);
  TaskMeta m;
  m.s = 0;
  m.e = 0;
  m.os = 0;
  if (u < B.user_end) {
    m.s = A.rp[u];
    m.e = A.rp[u + 1];
    if (need_os) m.os = A.orig_rp[u];
  }
  return m;
}

template <int MF, bool HAS_A, int KMAX>
struct RowRegs {
  uint32_t jp[KMAX / 2];  // item byte offsets (4 j, 16 bits each), slots 2i and 2i+1 packed
  float c[KMAX];          // c, replaced in place by v
  float a[HAS_A ? MF : 1][KMAX];
};

// Item byte offset held in slot k.
template <int MF, bool HAS_A, int KMAX>
__device__ __forceinline__ int item_off(const RowRegs<MF, HAS_A, KMAX>& R, int k) {
  return (k & 1) ? (int)(R.jp[k >> 1] >> 16) : (int)(R.jp[k >> 1] & 0xFFFFu);
}

// Histogram byte offset (2 jb) of the item in slot k.  The low half-word is
// taken with a byte permute, so the offset is one permute and one shift-add with
// the histogram's base (an and-mask here becomes shift, mask and add).
template <int MF, bool HAS_A, int KMAX>
__device__ __forceinline__ int hist_off(const RowRegs<MF, HAS_A, KMAX>& R, int k) {
  const uint32_t w = R.jp[k >> 1];
  const uint32_t jb = (k & 1) ? (w >> 16) : __builtin_amdgcn_perm(0u, w, 0x0c0c0100u);
  return (int)(jb << 1);
}

// Which row element a lane's register slot k holds.  The G lanes of a group
// read the row in chunks of four consecutive elements starting at the row
// start rounded down to a multiple of four: slot k of lane lid holds window
// element 4 (lid + (k/4) G) + k%4, i.e. row element pos(k) = that - (s & 3).
// Every chunk is one aligned load per array (8 bytes of item offsets, 16 bytes
// of FP32 values or 8 of BF16) and the group's chunks of one step are
// contiguous.  Slots outside [0, d) are masked.
template <int GLOG>
__device__ __forceinline__ int slot_off(int k, int lid) {
  constexpr int G = 1 << GLOG;
  return 4 * (lid + (k >> 2) * G) + (k & 3);
}
// Row-start shift of the window (s mod 4).
__device__ __forceinline__ int row_shift(const TaskMeta& m) { return (int)(m.s & 3); }

// Wide loads of the row arrays.  (Plain loads: the nontemporal hint, which
// speeds up a pure streaming read, made this pass 12% slower.)
typedef int dl_v4i __attribute__((ext_vector_type(4)));
typedef float dl_v4f __attribute__((ext_vector_type(4)));
typedef unsigned dl_v2u __attribute__((ext_vector_type(2)));

// four 16-bit item offsets, kept packed in pairs
__device__ __forceinline__ void ld4_idx(const uint16_t* p, uint32_t* out) {
  const dl_v2u v = *reinterpret_cast<const dl_v2u*>(p);
  out[0] = v.x;
  out[1] = v.y;
}
template <typename TV>
__device__ __forceinline__ void ld4(const TV* p, float* out);
template <>
__device__ __forceinline__ void ld4<float>(const float* p, float* out) {
  const dl_v4f v = *reinterpret_cast<const dl_v4f*>(p);
  out[0] = v.x;
  out[1] = v.y;
  out[2] = v.z;
  out[3] = v.w;
}
template <>
__device__ __forceinline__ void ld4<uint16_t>(const uint16_t* p, float* out) {
  // four BF16 values as two packed words, parked in the chunk's upper two
  // registers; unpack_rows spreads them where they are first used (unpacking
  // here would make the wavefront wait for the loads of the task it prefetches)
  const dl_v2u v = *reinterpret_cast<const dl_v2u*>(p);
  out[2] = __uint_as_float(v.x);
  out[3] = __uint_as_float(v.y);
}

// The chunks of a row that ld4 loaded as packed BF16 words, as FP32 values
// (bit moves only).  Nothing to do for FP32 rows.
template <typename TV, int KMAX>
__device__ __forceinline__ void unpack_rows(float (&x)[KMAX], int K) {
  if constexpr (sizeof(TV) == 2) {
#pragma unroll
    for (int k4 = 0; k4 < KMAX / 4; ++k4) {
      if (4 * k4 < K) {
        const uint32_t w0 = __float_as_uint(x[4 * k4 + 2]);
        const uint32_t w1 = __float_as_uint(x[4 * k4 + 3]);
        x[4 * k4 + 0] = __uint_as_float(w0 << 16);
        x[4 * k4 + 1] = __uint_as_float(w0 & 0xFFFF0000u);
        x[4 * k4 + 2] = __uint_as_float(w1 << 16);
        x[4 * k4 + 3] = __uint_as_float(w1 & 0xFFFF0000u);
      }
    }
  }
}

// Issues the loads of one task's rows (slot k of lane lid: see slot_off).
// Reads past a row end stay inside the padded arrays and are masked later.
template <int GLOG, int MF, bool HAS_A, int KMAX, typename TV, int MODE>
__device__ __forceinline__ void load_rows(const dl_grad_args& A, const TaskMeta& m, int K, int lid,
                                          RowRegs<MF, HAS_A, KMAX>& R) {
  constexpr int G = 1 << GLOG;
  K = __builtin_amdgcn_readfirstlane(K);
  if constexpr ((MODE & M_VIN) != 0) {
    // the caller's v has no alignment relation to the library's layout: one element per load
    const int d = (int)(m.e - m.s);
    const int sh = row_shift(m);
    const float* vp = A.v_in + m.os;
    DL_FOR_K(k, KMAX, K) {
      const int p = slot_off<GLOG>(k, lid) - sh;
      R.c[k] = (p >= 0 && p < d) ? vp[p] : 0.f;
    }
    return;
  }
  const int64_t base = (m.s & ~(int64_t)3) + 4 * lid;
  const uint16_t* ip = A.idx + base;
  const TV* cp = reinterpret_cast<const TV*>(A.cval) + base;
#pragma unroll
  for (int k4 = 0; k4 < KMAX / 4; ++k4) {
    if (4 * k4 < K) {
      ld4_idx(ip + 4 * k4 * G, &R.jp[2 * k4]);
      ld4<TV>(cp + 4 * k4 * G, &R.c[4 * k4]);
    }
  }
  if constexpr (HAS_A) {
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if (f < A.m && A.a_slot[f] >= 0) {
        const TV* ap = reinterpret_cast<const TV*>(A.aval) + (int64_t)A.a_slot[f] * A.astride + base;
#pragma unroll
        for (int k4 = 0; k4 < KMAX / 4; ++k4)
          if (4 * k4 < K) ld4<TV>(ap + 4 * k4 * G, &R.a[f][4 * k4]);
      }
    }
  }
}

// v = (c + sum_k a_k mu_k[j]) * (-1/gamma) in place of c, computed as
// c (-1/gamma) + sum_k a_k mu'_k[j] from the staged mu' = mu (-1/gamma); -inf
// outside the row.  Slot k is inside the row when 0 <= slot_off(k, lid) - shift
// < d; with lo = shift - 4 lid that is lo <= c_k < d + lo on the compile-time
// part c_k = slot_off(k, 0) of the slot's offset.  lo <= 3 <= c_k for k >= 3,
// so those slots test the upper end only; slots 0..2 take the one unsigned
// compare (c_k - lo) < d.
template <int GLOG, int MF, bool HAS_A, int KMAX, typename TV, int MODE>
__device__ __forceinline__ void gather_v(const dl_grad_args& A, const TaskMeta& m, int K, int lid,
                                         RowRegs<MF, HAS_A, KMAX>& R, const float* s_mu,
                                         float (&cc)[(MODE & M_REPAIR) ? KMAX : 1]) {
  K = __builtin_amdgcn_readfirstlane(K);
  const unsigned d = (unsigned)(m.e - m.s);
  const int lo = row_shift(m) - slot_off<GLOG>(0, lid);
  const int hi = (int)d + lo;
  const int mm = A.m;
  if constexpr ((MODE & M_VIN) == 0) {
    unpack_rows<TV, KMAX>(R.c, K);
    if constexpr (HAS_A) {
#pragma unroll
      for (int f = 0; f < MF; ++f)
        if (f < mm && A.a_slot[f] >= 0) unpack_rows<TV, KMAX>(R.a[f], K);
    }
  }
  // the global-count row's dual: folded into the staged family-0 words when
  // family 0 has a == 1, added here when its a is stored
  float mug = 0.f;
  if constexpr (HAS_A) {
    if (A.glob && A.a_slot[0] >= 0) mug = lds_word(s_mu, 4 * mm * A.J);
  }
  DL_FOR_KC(k, KMAX, K) {
    {
      const bool in = k < 3 ? (unsigned)(slot_off<GLOG>(k, 0) - lo) < d : slot_off<GLOG>(k, 0) < hi;
      float val;
      if constexpr ((MODE & M_VIN) != 0) {
        val = R.c[k];
      } else {
        const int jb = item_off(R, k);
        // the family loop has a uniform trip count: every read is issued
        // unconditionally (rows of absent families read in-bounds LDS words
        // that the select discards), so the reads of a chunk batch up
        float sdot;
        const float mu0 = lds_word(s_mu, jb);
        if constexpr (HAS_A) {
          sdot = A.a_slot[0] >= 0 ? fmaf(R.a[0][k], mu0, mug) : mu0;
        } else {
          sdot = mu0;
        }
#pragma unroll
        for (int f = 1; f < MF; ++f) {
          const float muf = lds_word(s_mu, (f < mm ? f : 0) * 4 * A.J + jb);
          float af = 1.f;
          if constexpr (HAS_A) {
            if (A.a_slot[f] >= 0) af = R.a[f][k];
          }
          const float t = fmaf(af, muf, sdot);
          sdot = f < mm ? t : sdot;
        }
        if constexpr ((MODE & M_REPAIR) != 0) cc[k] = R.c[k];
        val = fmaf(R.c[k], A.neg_inv_gamma, sdot);  // eq. 3 argument
      }
      R.c[k] = in ? val : -INFINITY;
    }
  }
}

// Box-cut set {0 <= x <= u, sum x <= z} (Table 1's third projection kind):
// x = clamp(v - theta, 0, u), theta = 0 when clamp(v, 0, u) sums to at most
// z, else the root of f(theta) = sum clamp(v - theta, 0, u) - z, which is
// nonincreasing and linear between the breakpoints {v, v - u}.  Evaluation at
// theta: f, the count of coordinates free just right of theta (0 < v - theta
// <= u: one sitting at its cap starts to move) and the next breakpoint above
// theta.
template <int GLOG, int KMAX, bool HAS_A>
__device__ __forceinline__ void boxcut_eval(const float (&v)[KMAX], int K, float theta, float u, float& f,
                                            float& cnt, float& nb) {
  f = 0.f;
  cnt = 0.f;
  nb = INFINITY;
  DL_FOR_KC(k, KMAX, K) {
    {
      const float t = v[k] - theta;
      f += fminf(fmaxf(t, 0.f), u);
      cnt += (t > 0.f && t <= u) ? 1.f : 0.f;
      nb = fminf(nb, t > u ? v[k] - u : (t > 0.f ? v[k] : INFINITY));
    }
  }
  f = gsum<GLOG>(f);
  cnt = gsum<GLOG>(cnt);
  nb = gmin<GLOG>(nb);
}

// theta of every lane group of the wavefront: Newton steps from the left end
// of a bracket [lo, hi] (exact once the step stays inside the piece that
// starts at lo), the secant of the bracket once no breakpoint lies inside it
// (exact as well), bisection otherwise.  Every lane runs every round (the
// group reductions need the whole wavefront).
template <int GLOG, int KMAX, bool HAS_A>
__device__ __forceinline__ float boxcut_theta(const float (&v)[KMAX], int K, float z, float u) {
  float flo, clo, nblo;
  boxcut_eval<GLOG, KMAX, HAS_A>(v, K, 0.f, u, flo, clo, nblo);
  flo -= z;
  float m1 = -INFINITY;
  DL_FOR_KC(k, KMAX, K) m1 = fmaxf(m1, v[k]);
  m1 = gmax<GLOG>(m1);
  bool done = !(flo > 0.f);  // clamp(v, 0, u) already fits (or no user here)
  float theta = 0.f, lo = 0.f, hi = m1, fhi = -z;
  for (int it = 0; it < 64 && __any(!done); ++it) {
    float cand = 0.5f * (lo + hi);
    if (!done) {
      if (clo > 0.f) {
        const float tn = lo + flo * __builtin_amdgcn_rcpf(clo);
        if (tn <= nblo) {
          theta = tn;  // the linear piece at lo reaches z: exact
          done = true;
        }
        cand = tn;
      } else {
        cand = nblo;
      }
      if (!done && nblo >= hi) {
        theta = lo + (hi - lo) * (flo / (flo - fhi));  // f is linear on [lo, hi]
        done = true;
      }
      if (!(cand > lo && cand < hi)) cand = 0.5f * (lo + hi);
    }
    float f, c, nb;
    boxcut_eval<GLOG, KMAX, HAS_A>(v, K, cand, u, f, c, nb);
    f -= z;
    if (!done) {
      if (fabsf(f) <= z * 0x1p-22f) {
        theta = cand;
        done = true;
      } else if (f > 0.f) {
        lo = cand;
        flo = f;
        clo = c;
        nblo = nb;
      } else {
        hi = cand;
        fhi = f;
      }
    }
  }
  if (!done) theta = clo > 0.f ? lo + flo / clo : lo;
  return theta;
}

// Projects the task's rows (v in R.c) and accumulates what MODE asks.
template <int GLOG, int MF, bool HAS_A, int KMAX, typename TV, int MODE>
__device__ __forceinline__ void project_task(const dl_grad_args& A, const TaskMeta& m, int K, int lid,
                                             RowRegs<MF, HAS_A, KMAX>& R, const float* s_rf,
                                             unsigned long long* s_hist, LaneAcc& acc,
                                             const float (&cc)[(MODE & M_REPAIR) ? KMAX : 1],
                                             const float (&qs)[DL_NQS]) {
  K = __builtin_amdgcn_readfirstlane(K);
  float (&v)[KMAX] = R.c;
  const float z = A.radius;
  const bool box = (A.proj == DL_PROJ_BOX);
  const bool boxcut = (A.proj == DL_PROJ_BOXCUT);
  float theta = 0.f;
  if (boxcut) {
    theta = boxcut_theta<GLOG, KMAX, HAS_A>(v, K, z, A.upper);
  } else if (!box) {
    // one pass: the three largest entries and the positive part's sum.  These
    // settle most rows without a search: no user here; the positive part fits
    // (inequality form); the leader alone carries mass z (m1 - m2 >= z); or the two
    // leaders do, theta = (m1 + m2 - z) / 2, when the third lies at or below it.
    float m1 = -INFINITY, m2 = -INFINITY, m3 = -INFINITY, sp = 0.f;
    DL_FOR_KC(k, KMAX, K) {
      {
        m3 = __builtin_amdgcn_fmed3f(m2, m3, v[k]);  // third largest of {m1 >= m2 >= m3, v}
        m2 = __builtin_amdgcn_fmed3f(m1, m2, v[k]);
        m1 = fmaxf(m1, v[k]);
        sp += fmaxf(v[k], 0.f);
      }
    }
    gtop3<GLOG>(m1, m2, m3);
    sp = gsum<GLOG>(sp);
    const bool eq = A.proj == DL_PROJ_SIMPLEX_EQ;
    bool done = true;
    if (m1 == -INFINITY || (!eq && sp <= z)) {
      // theta = 0
    } else if (m1 - m2 >= z) {
      theta = m1 - z;
    } else {
      // m2 > theta2 since m1 - m2 < z; the top two are the active set when m3 <= theta2
      const float theta2 = 0.5f * (m1 + m2 - z);
      theta = theta2;
      if (!(m3 <= theta2)) {
        // start left of the root, as close as the sums allow: the root is at least
        // (sum of any k entries - z) / k, here for the top two and the top three
        theta = fmaxf(theta2, (m1 + m2 + m3 - z) * (1.f / 3.f));
        done = false;
      }
    }
    if (__any(!done)) {
      // only in wavefronts with a row left: the positive count (an integer: one
      // compare and one add-with-carry per element) for the bound with k = #positive
      unsigned cpi = 0;
      DL_FOR_KC(k, KMAX, K) cpi += v[k] > 0.f;
      const float cp = gsum<GLOG>((float)cpi);
      if (!done && sp > z) theta = fmaxf(theta, (sp - z) * __builtin_amdgcn_rcpf(cp));  // Newton step from 0
    }
    for (int it = 0; it < 64 && __any(!done); ++it) {
      float f = 0.f, mina = INFINITY;
      unsigned ci = 0;
      DL_FOR_KC(k, KMAX, K) {
        {
          const float t = v[k] - theta;
          f += fmaxf(t, 0.f);
          const bool act = t > 0.f;
          ci += act;
          mina = fminf(mina, act ? v[k] : INFINITY);
        }
      }
      f = gsum<GLOG>(f);
      const float cnt = gsum<GLOG>((float)ci);
      mina = gmin<GLOG>(mina);
      if (!done) {
        // Newton step: the exact threshold of the active set {v > theta}; the
        // set survives the step when its smallest member stays above it
        const float nt = theta + (f - z) * __builtin_amdgcn_rcpf(cnt);
        done = (mina > nt) || (fabsf(f - z) <= z * 0x1p-22f);
        theta = nt;
      }
    }
  }

  float lobj = 0.f;
  // t is the element's value before the clamp at 0: x = max(t, 0).  The
  // histogram of a family with a == 1 and the global count convert t itself
  // with a saturating convert, which maps t <= 0 to 0 as x would.
  auto emit = [&](int k, float t) {
    {
      const float x = fmaxf(t, 0.f);
      (void)x;  // unused in the histogram-only modes of families with a == 1
      if constexpr ((MODE & M_XOUT) != 0) {
        const int p = slot_off<GLOG>(k, lid) - row_shift(m);
        if (p >= 0 && p < (int)(m.e - m.s)) A.x_out[m.os + p] = x;
      }
      if constexpr ((MODE & M_HIST) != 0) {
#pragma unroll
        for (int f = 0; f < MF; ++f) {
          if (f < A.m) {
            float w = t;
            if constexpr (HAS_A) w = A.a_slot[f] >= 0 ? R.a[f][k] * x : x;
            hist_put<HAS_A, MODE>(s_hist, f * 8 * A.J + hist_off(R, k), w, qs[f], A);
          }
        }
        // global-count row: x >= 0 on its own grid, summed per lane in 64 bits
        if constexpr ((MODE & M_GLOB) != 0) acc.gcnt += cvt_u32_sat(fmaf(t, qs[DL_MAX_FAMILIES], 0.5f));
      }
      if constexpr ((MODE & M_OBJ) != 0) {
        // (c + A^T lam) x + gamma/2 x^2, with c + A^T lam = -gamma v; 0 when x = 0
        // (padding lanes hold v = -inf and x = 0: the clamp keeps their term an exact 0
        // rather than 0 * inf, whatever the compiler does with the select)
        const float term = x * fmaf(0.5f * A.gamma, x, -A.gamma * fmaxf(v[k], -0x1p100f));
        lobj += x > 0.f ? term : 0.f;
      }
      if constexpr ((MODE & M_REPAIR) != 0) {
        const float xt = lds_word(s_rf, item_off(R, k)) * x;
        lobj += xt * fmaf(0.5f * A.gamma, xt, cc[k]);
      }
    }
  };
  // one loop per projection kind, so the kind is not re-tested per element
  if (box) {
    DL_FOR_KC(k, KMAX, K) emit(k, fminf(v[k], z));
  } else if (boxcut) {
    const float u = A.upper;
    DL_FOR_KC(k, KMAX, K) emit(k, fminf(v[k] - theta, u));
  } else {
    DL_FOR_KC(k, KMAX, K) emit(k, v[k] - theta);
  }
  if (MODE & (M_OBJ | M_REPAIR)) acc.obj += (double)lobj;
}

// The tasks t0, t0 + DL_WAVES, ... < t1 of one bucket.  With PF the next
// task's rows load while the current one is projected: gather (waits for this
// task's rows), issue the next task's loads, then project and accumulate.
template <int GLOG, int MF, bool HAS_A, int KMAX, typename TV, int MODE>
__device__ __forceinline__ void run_bucket(const dl_grad_args& A, const dl_bucket& B, int64_t t0, int64_t t1,
                                           int lane, const float* s_mu, const float* s_rf,
                                           unsigned long long* s_hist, LaneAcc& acc,
                                           const float (&qs)[DL_NQS]) {
  if (t0 >= t1) return;
  // keeps per-bucket lane arithmetic inside this bucket's code (otherwise it is
  // hoisted out of the kernel's bucket loop for every bucket at once and spills)
  asm volatile("" : "+v"(lane));
  // software pipelining needs two tasks' rows in registers: with four families'
  // coefficients that spills within the 128 registers of 16 waves per CU
  constexpr bool PF = (MF <= 2) && !(MODE & M_REPAIR);
  constexpr int G = 1 << GLOG;
  const int lid = lane & (G - 1);
  constexpr bool need_os = (MODE & (M_VIN | M_XOUT)) != 0;
  auto kof = [&](const TaskMeta& m) {
    // users are sorted longest first: lane 0 holds the task's longest row;
    // slots per lane, whole chunks of four with wide loads (window shift <= 3)
    const int d0 = __builtin_amdgcn_readfirstlane((int)(m.e - m.s));
    return 4 * ((d0 + 3 + 4 * G - 1) >> (GLOG + 2));
  };
  float cc[(MODE & M_REPAIR) ? KMAX : 1];
  if constexpr (!PF) {
    RowRegs<MF, HAS_A, KMAX> R;
    for (int64_t t = t0; t < t1; t += DL_WAVES) {
      TaskMeta m = load_meta<GLOG>(A, B, t, lane, need_os);
      const int K = kof(m);
      load_rows<GLOG, MF, HAS_A, KMAX, TV, MODE>(A, m, K, lid, R);
      gather_v<GLOG, MF, HAS_A, KMAX, TV, MODE>(A, m, K, lid, R, s_mu, cc);
      project_task<GLOG, MF, HAS_A, KMAX, TV, MODE>(A, m, K, lid, R, s_rf, s_hist, acc, cc, qs);
    }
    return;
  }
  RowRegs<MF, HAS_A, KMAX> RA, RB;
  TaskMeta ma = load_meta<GLOG>(A, B, t0, lane, need_os);
  TaskMeta mb = ma;
  int64_t t = t0;
  if (t + DL_WAVES < t1) mb = load_meta<GLOG>(A, B, t + DL_WAVES, lane, need_os);
  int ka = kof(ma), kb = 0;
  load_rows<GLOG, MF, HAS_A, KMAX, TV, MODE>(A, ma, ka, lid, RA);
  while (true) {
    gather_v<GLOG, MF, HAS_A, KMAX, TV, MODE>(A, ma, ka, lid, RA, s_mu, cc);
    TaskMeta mc = mb;
    if (t + DL_WAVES < t1) {
      kb = kof(mb);
      load_rows<GLOG, MF, HAS_A, KMAX, TV, MODE>(A, mb, kb, lid, RB);
      if (t + 2 * DL_WAVES < t1) mc = load_meta<GLOG>(A, B, t + 2 * DL_WAVES, lane, need_os);
    }
    project_task<GLOG, MF, HAS_A, KMAX, TV, MODE>(A, ma, ka, lid, RA, s_rf, s_hist, acc, cc, qs);
    t += DL_WAVES;
    if (t >= t1) break;
    gather_v<GLOG, MF, HAS_A, KMAX, TV, MODE>(A, mb, kb, lid, RB, s_mu, cc);
    TaskMeta md = mc;
    if (t + DL_WAVES < t1) {
      ka = kof(mc);
      load_rows<GLOG, MF, HAS_A, KMAX, TV, MODE>(A, mc, ka, lid, RA);
      if (t + 2 * DL_WAVES < t1) md = load_meta<GLOG>(A, B, t + 2 * DL_WAVES, lane, need_os);
    }
    project_task<GLOG, MF, HAS_A, KMAX, TV, MODE>(A, mb, kb, lid, RB, s_rf, s_hist, acc, cc, qs);
    t += DL_WAVES;
    if (t >= t1) break;
    ma = mc;
    mb = md;
  }
}

// ---------------------------------------------------------------------------
// Rows longer than 64*KMAX: one wavefront per user, re-reading the row per
// Newton step (the row stays in L1/L2, so HBM sees it once).
// ---------------------------------------------------------------------------
template <int MF, bool HAS_A, typename TV, int MODE>
__device__ __forceinline__ float long_v(const dl_grad_args& A, const float* s_mu, int64_t s, int64_t os, int e,
                                        int& j /* item byte offset */, float& c, float (&af)[HAS_A ? MF : 1]) {
  if constexpr ((MODE & M_VIN) != 0) return A.v_in[os + e];
  j = A.idx[s + e];
  c = ldv<TV>(reinterpret_cast<const TV*>(A.cval) + s + e);
  // the global-count dual is folded into family 0's staged words when its a == 1
  float sdot = (HAS_A && A.glob && A.a_slot[0] >= 0) ? lds_word(s_mu, 4 * A.m * A.J) : 0.f;
#pragma unroll
  for (int f = 0; f < MF; ++f) {
    if (f < A.m) {
      float a = 1.f;
      if (HAS_A && A.a_slot[f] >= 0)
        a = ldv<TV>(reinterpret_cast<const TV*>(A.aval) + (int64_t)A.a_slot[f] * A.astride + s + e);
      if (HAS_A) af[f] = a;
      sdot = fmaf(a, lds_word(s_mu, f * 4 * A.J + j), sdot);
    }
  }
  return fmaf(c, A.neg_inv_gamma, sdot);  // the staged duals carry -1/gamma
}

template <int MF, bool HAS_A, typename TV, int MODE>
__device__ __forceinline__ void long_task(const dl_grad_args& A, int64_t t, const dl_bucket& B, const float* s_mu,
                                          const float* s_rf, unsigned long long* s_hist, int lane, LaneAcc& acc,
                                          const float (&qs)[DL_NQS]) {
  const int64_t u = B.user_begin + (t - B.task_begin);
  const int64_t s = A.rp[u];
  const int d = (int)(A.rp[u + 1] - s);
  const int64_t os = (MODE & (M_VIN | M_XOUT)) ? A.orig_rp[u] : 0;
  const float z = A.radius;
  const bool box = (A.proj == DL_PROJ_BOX);
  const bool boxcut = (A.proj == DL_PROJ_BOXCUT);
  const float ucap = A.upper;
  int j = 0;
  float c = 0.f;
  float af[HAS_A ? MF : 1];
  float theta = 0.f;
  if (boxcut) {
    // same bracketed Newton iteration as the group path, one wavefront per row
    auto eval = [&](float th, float& f, float& cnt, float& nb) {
      f = 0.f;
      cnt = 0.f;
      nb = INFINITY;
      for (int e = lane; e < d; e += 64) {
        const float v = long_v<MF, HAS_A, TV, MODE>(A, s_mu, s, os, e, j, c, af);
        const float t = v - th;
        f += fminf(fmaxf(t, 0.f), ucap);
        cnt += (t > 0.f && t <= ucap) ? 1.f : 0.f;
        nb = fminf(nb, t > ucap ? v - ucap : (t > 0.f ? v : INFINITY));
      }
      f = gsum<6>(f);
      cnt = gsum<6>(cnt);
      nb = gmin<6>(nb);
    };
    float flo, clo, nblo;
    eval(0.f, flo, clo, nblo);
    flo -= z;
    if (flo > 0.f) {
      float vmax = -INFINITY;
      for (int e = lane; e < d; e += 64) vmax = fmaxf(vmax, long_v<MF, HAS_A, TV, MODE>(A, s_mu, s, os, e, j, c, af));
      float lo = 0.f, hi = gmax<6>(vmax), fhi = -z;
      bool done = false;
      for (int it = 0; it < 64 && !done; ++it) {
        float cand;
        if (clo > 0.f) {
          cand = lo + flo / clo;
          if (cand <= nblo) {
            theta = cand;
            done = true;
            break;
          }
        } else {
          cand = nblo;
        }
        if (nblo >= hi) {
          theta = lo + (hi - lo) * (flo / (flo - fhi));  // f is linear on [lo, hi]
          done = true;
          break;
        }
        if (!(cand > lo && cand < hi)) cand = 0.5f * (lo + hi);
        float f, cn, nb;
        eval(cand, f, cn, nb);
        f -= z;
        if (fabsf(f) <= z * 0x1p-22f) {
          theta = cand;
          done = true;
        } else if (f > 0.f) {
          lo = cand;
          flo = f;
          clo = cn;
          nblo = nb;
        } else {
          hi = cand;
          fhi = f;
        }
      }
      if (!done) theta = clo > 0.f ? lo + flo / clo : lo;
    }
  } else if (!box) {
    float vmax = -INFINITY, sp = 0.f, cp = 0.f;
    for (int e = lane; e < d; e += 64) {
      float v = long_v<MF, HAS_A, TV, MODE>(A, s_mu, s, os, e, j, c, af);
      vmax = fmaxf(vmax, v);
      sp += fmaxf(v, 0.f);
      cp += v > 0.f ? 1.f : 0.f;
    }
    vmax = gmax<6>(vmax);
    sp = gsum<6>(sp);
    cp = gsum<6>(cp);
    const bool eq = A.proj == DL_PROJ_SIMPLEX_EQ;
    if (eq || sp > z) {
      theta = vmax - z;
      if (sp > z && cp > 0.f) theta = fmaxf(theta, (sp - z) / cp);
      for (int it = 0; it < 64; ++it) {
        float f = 0.f, cnt = 0.f, mina = INFINITY;
        for (int e = lane; e < d; e += 64) {
          float v = long_v<MF, HAS_A, TV, MODE>(A, s_mu, s, os, e, j, c, af);
          float tt = v - theta;
          f += fmaxf(tt, 0.f);
          cnt += tt > 0.f ? 1.f : 0.f;
          mina = fminf(mina, tt > 0.f ? v : INFINITY);
        }
        f = gsum<6>(f);
        cnt = gsum<6>(cnt);
        mina = gmin<6>(mina);
        const float nt = theta + (f - z) / cnt;
        const bool stable = (mina > nt) || (fabsf(f - z) <= z * 0x1p-22f);
        theta = nt;
        if (stable) break;
      }
    }
  }
  float lobj = 0.f;
  for (int e = lane; e < d; e += 64) {
    float v = long_v<MF, HAS_A, TV, MODE>(A, s_mu, s, os, e, j, c, af);
    float x = box ? fminf(fmaxf(v, 0.f), z) : (boxcut ? fminf(fmaxf(v - theta, 0.f), ucap) : fmaxf(v - theta, 0.f));
    if constexpr ((MODE & M_XOUT) != 0) A.x_out[os + e] = x;
    if constexpr ((MODE & M_HIST) != 0) {
#pragma unroll
      for (int f = 0; f < MF; ++f) {
        if (f < A.m) {
          float w = (HAS_A && A.a_slot[f] >= 0) ? af[HAS_A ? f : 0] * x : x;
          hist_put<HAS_A, MODE>(s_hist, f * 8 * A.J + 2 * j, w, qs[f], A);
        }
      }
      if constexpr ((MODE & M_GLOB) != 0) acc.gcnt += __float2uint_rz(fmaf(x, qs[DL_MAX_FAMILIES], 0.5f));
    }
    if constexpr ((MODE & M_OBJ) != 0) lobj += x > 0.f ? x * fmaf(0.5f * A.gamma, x, -A.gamma * v) : 0.f;
    if constexpr ((MODE & M_REPAIR) != 0) {
      const float xt = lds_word(s_rf, j) * x;
      lobj += xt * fmaf(0.5f * A.gamma, xt, c);
    }
  }
  if (MODE & (M_OBJ | M_REPAIR)) acc.obj += (double)lobj;
}

// One workgroup's share of a pass: tasks [w0, w1) of the instance A describes;
// its histogram goes to partial slot `slot`.
template <int MF, bool HAS_A, int KMAX, typename TV, int MODE>
__device__ __forceinline__ void grad_body(const dl_grad_args& A, int64_t w0, int64_t w1, int slot) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int mJ = A.m * A.J;
  const int nrow = mJ + A.glob;
  const bool need_mu = !(MODE & M_VIN);
  float* s_mu = reinterpret_cast<float*>(smem);
  const int mu_n = need_mu ? nrow : 0;
  float* s_rf = s_mu + mu_n;
  const int rf_n = (MODE & M_REPAIR) ? A.J : 0;
  size_t off = ((size_t)(mu_n + rf_n) * 4 + 15) & ~(size_t)15;
  // the histogram: every item row, or (M_TILE) the rows of this launch's window
  unsigned long long* s_hist = reinterpret_cast<unsigned long long*>(smem + off);
  const int hist_n = (MODE & M_HIST) ? (((MODE & M_TILE) != 0) ? (A.tile_bn >> 3) : mJ) : 0;
  double* s_obj = reinterpret_cast<double*>(smem + off + (size_t)hist_n * 8);
  unsigned long long* s_gc = reinterpret_cast<unsigned long long*>(s_obj + DL_WAVES);

  const int tid = threadIdx.x;
  unsigned long long t_start = 0;
  if (A.wg_clock && tid == 0) t_start = (unsigned long long)wall_clock64();
  if (need_mu) {
    // family 0's words carry the global-count dual as well when its a == 1; every
    // word is staged times -1/gamma, so v = c (-1/gamma) + sum_k a_k mu'_k[j] is one
    // fused multiply-add per element past the coupling sum
    const float mug0 = (A.glob && A.a_slot[0] < 0) ? A.mu[mJ] : 0.f;
    const float ng = A.neg_inv_gamma;
    for (int r = tid; r < mu_n; r += DL_WG) s_mu[r] = (r < A.J ? A.mu[r] + mug0 : A.mu[r]) * ng;
  }
  for (int r = tid; r < rf_n; r += DL_WG) s_rf[r] = A.rfac[r];
  for (int r = tid; r < hist_n; r += DL_WG) s_hist[r] = 0ull;
  __syncthreads();

  const int wave = tid >> 6;
  const int lane = tid & 63;
  LaneAcc acc;
  // this pass's fixed-point scales (uniform); the global-count row's last
  float qs[DL_NQS];
#pragma unroll
  for (int f = 0; f < DL_MAX_FAMILIES; ++f)
    qs[f] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(A.qs_dev ? A.qs_dev[f] : A.qscale[f])));
  qs[DL_MAX_FAMILIES] = A.qs_dev ? __int_as_float(__builtin_amdgcn_readfirstlane(
                                       __float_as_int(A.qs_dev[DL_MAX_FAMILIES])))
                                 : 0x1p30f / fmaxf(A.radius, 0x1p-30f);
  for (int b = 0; b < A.n_buckets; ++b) {
    const dl_bucket& B = A.bk[b];
    const int64_t b1 = (b + 1 < A.n_buckets) ? A.bk[b + 1].task_begin : w1;
    const int64_t lo = w0 > B.task_begin ? w0 : B.task_begin;
    const int64_t hi = w1 < b1 ? w1 : b1;
    if (lo >= hi) continue;
    // this wavefront's tasks: w0 + wave + k*DL_WAVES inside [lo, hi)
    int64_t first = w0 + wave;
    if (first < lo) first += ((lo - first + DL_WAVES - 1) / DL_WAVES) * DL_WAVES;
    switch (B.glog) {
      case 0: run_bucket<0, MF, HAS_A, KMAX, TV, MODE>(A, B, first, hi, lane, s_mu, s_rf, s_hist, acc, qs); break;
      case 1: run_bucket<1, MF, HAS_A, KMAX, TV, MODE>(A, B, first, hi, lane, s_mu, s_rf, s_hist, acc, qs); break;
      case 2: run_bucket<2, MF, HAS_A, KMAX, TV, MODE>(A, B, first, hi, lane, s_mu, s_rf, s_hist, acc, qs); break;
      case 3: run_bucket<3, MF, HAS_A, KMAX, TV, MODE>(A, B, first, hi, lane, s_mu, s_rf, s_hist, acc, qs); break;
      case 4: run_bucket<4, MF, HAS_A, KMAX, TV, MODE>(A, B, first, hi, lane, s_mu, s_rf, s_hist, acc, qs); break;
      case 5: run_bucket<5, MF, HAS_A, KMAX, TV, MODE>(A, B, first, hi, lane, s_mu, s_rf, s_hist, acc, qs); break;
      case 6: run_bucket<6, MF, HAS_A, KMAX, TV, MODE>(A, B, first, hi, lane, s_mu, s_rf, s_hist, acc, qs); break;
      default:
        for (int64_t t = first; t < hi; t += DL_WAVES)
          long_task<MF, HAS_A, TV, MODE>(A, t, B, s_mu, s_rf, s_hist, lane, acc, qs);
        break;
    }
  }
  if (MODE & (M_OBJ | M_REPAIR)) {
    // fixed-order FP64 reduction: lanes of a wavefront, then wavefronts in order
    double o_ = acc.obj;
    for (int o = 32; o > 0; o >>= 1) o_ += __shfl_xor(o_, o, 64);
    if (lane == 0) s_obj[wave] = o_;
  }
  if ((MODE & M_GLOB) && A.glob) {
    // integer sums: exact in any order
    unsigned long long g_ = acc.gcnt;
    for (int o = 32; o > 0; o >>= 1) g_ += __shfl_xor(g_, o, 64);
    if (lane == 0) s_gc[wave] = g_;
  }
  __syncthreads();
  if (MODE & M_HIST) {
    unsigned long long* dst = A.part + (size_t)slot * nrow;
    const int r0 = ((MODE & M_TILE) != 0) ? (A.tile_b0 >> 3) : 0;
    for (int r = tid; r < hist_n; r += DL_WG) dst[r0 + r] = s_hist[r];
    if ((MODE & M_GLOB) && A.glob && tid == 0) {
      unsigned long long g_ = 0ull;
      for (int w = 0; w < DL_WAVES; ++w) g_ += s_gc[w];
      dst[mJ] = g_;
    }
  }
  if ((MODE & (M_OBJ | M_REPAIR)) && tid == 0) {
    double tot = 0.0;
    for (int w = 0; w < DL_WAVES; ++w) tot += s_obj[w];
    A.obj_part[slot] = tot;
  }
  if (A.wg_clock) {
    __syncthreads();
    if (tid == 0) {
      A.wg_clock[2 * slot] = t_start;
      A.wg_clock[2 * slot + 1] = (unsigned long long)wall_clock64();
    }
  }
}

template <int MF, bool HAS_A, int KMAX, typename TV, int MODE>
__global__ void __launch_bounds__(DL_WG) grad_pass(dl_grad_args A) {
  grad_body<MF, HAS_A, KMAX, TV, MODE>(A, A.wg_task[blockIdx.x], A.wg_task[blockIdx.x + 1], (int)blockIdx.x);
}

// Many instances in one launch: workgroup w serves tasks [t0, t1) of
// instance wgs[w].inst (per-instance arguments in device memory).
template <int MF, bool HAS_A, int KMAX, typename TV, int MODE>
__global__ void __launch_bounds__(DL_WG) grad_pass_batch(const dl_grad_args* __restrict__ args,
                                                         const dl_wg_desc* __restrict__ wgs) {
  const dl_wg_desc w = wgs[blockIdx.x];
  grad_body<MF, HAS_A, KMAX, TV, MODE>(args[w.inst], w.t0, w.t1, w.slot);
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
    case M_HIST | M_XOUT: return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_XOUT>(P, A, lds);
    case M_HIST | M_OBJ | M_XOUT: return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_XOUT>(P, A, lds);
    case M_HIST | M_GLOB: return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_GLOB>(P, A, lds);
    case M_HIST | M_OBJ | M_GLOB: return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_GLOB>(P, A, lds);
    case M_HIST | M_XOUT | M_GLOB: return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_XOUT | M_GLOB>(P, A, lds);
    case M_HIST | M_OBJ | M_XOUT | M_GLOB:
      return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_XOUT | M_GLOB>(P, A, lds);
    default: break;
  }
  // coupling blocks beyond one LDS histogram (row windows) run on the multi-family kernels only
  if constexpr (MF >= 2) {
    switch (mode) {
      case M_HIST | M_TILE: return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_TILE>(P, A, lds);
      case M_HIST | M_OBJ | M_TILE: return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_TILE>(P, A, lds);
      case M_HIST | M_XOUT | M_TILE: return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_XOUT | M_TILE>(P, A, lds);
      case M_HIST | M_OBJ | M_XOUT | M_TILE:
        return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_XOUT | M_TILE>(P, A, lds);
      case M_HIST | M_GLOB | M_TILE: return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_GLOB | M_TILE>(P, A, lds);
      case M_HIST | M_OBJ | M_GLOB | M_TILE:
        return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_GLOB | M_TILE>(P, A, lds);
      case M_HIST | M_XOUT | M_GLOB | M_TILE:
        return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_XOUT | M_GLOB | M_TILE>(P, A, lds);
      case M_HIST | M_OBJ | M_XOUT | M_GLOB | M_TILE:
        return launch_one<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_XOUT | M_GLOB | M_TILE>(P, A, lds);
      default: break;
    }
  }
  switch (mode) {
    case M_REPAIR: return launch_one<MF, HAS_A, KMAX, TV, M_REPAIR>(P, A, lds);
    case M_VIN | M_XOUT: return launch_one<MF, HAS_A, KMAX, TV, M_VIN | M_XOUT>(P, A, lds);
    default: dl_set_error("internal: unknown gradient-pass mode"); return DL_EINVAL;
  }
}

template <int MF, bool HAS_A, int KMAX, typename TV>
dl_status launch_batch_t(const dl_problem* P, int n_wg, const dl_grad_args* d_args, const dl_wg_desc* d_wgs,
                         size_t lds, hipStream_t st, int mode) {
  (void)P;
  // the iteration's histogram pass, and the certificate's two passes
  switch (mode) {
#define DL_BATCH_CASE(MD)                                                                                 \
  case MD:                                                                                                \
    hipLaunchKernelGGL((grad_pass_batch<MF, HAS_A, KMAX, TV, MD>), dim3(n_wg), dim3(DL_WG), lds, st, d_args, \
                       d_wgs);                                                                            \
    break;
    DL_BATCH_CASE(M_HIST)
    DL_BATCH_CASE(M_HIST | M_GLOB)
    DL_BATCH_CASE(M_HIST | M_OBJ)
    DL_BATCH_CASE(M_HIST | M_OBJ | M_GLOB)
    DL_BATCH_CASE(M_REPAIR)
#undef DL_BATCH_CASE
    default:
      dl_set_error("internal: unknown batched gradient-pass mode");
      return DL_EINVAL;
  }
  DL_HIP_TRY(hipGetLastError());
  return DL_OK;
}

template <int MF, bool HAS_A, int KMAX, typename TV>
void set_attr_all() {
  (void)hipFuncSetAttribute((const void*)grad_pass_batch<MF, HAS_A, KMAX, TV, M_HIST>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  const int big = 160 * 1024;
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_REPAIR>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_XOUT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_XOUT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass_batch<MF, HAS_A, KMAX, TV, M_HIST | M_GLOB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass_batch<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass_batch<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_GLOB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass_batch<MF, HAS_A, KMAX, TV, M_REPAIR>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_GLOB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_GLOB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_XOUT | M_GLOB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_XOUT | M_GLOB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if constexpr (MF >= 2) {
    const void* gk[] = {
        (const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_TILE>,
        (const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_TILE>,
        (const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_XOUT | M_TILE>,
        (const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_XOUT | M_TILE>,
        (const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_GLOB | M_TILE>,
        (const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_GLOB | M_TILE>,
        (const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_XOUT | M_GLOB | M_TILE>,
        (const void*)grad_pass<MF, HAS_A, KMAX, TV, M_HIST | M_OBJ | M_XOUT | M_GLOB | M_TILE>};
    for (const void* k : gk) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  }
}
}  // namespace
