// One kernel variant of the gradient pass: this file is compiled once per
// (family class, stored a, storage type), chosen by DL_GV_MF (1, 2 or 4),
// DL_GV_A (0: every a == 1, 1: some family stored) and DL_GV_BF16 (0: FP32
// values, 1: BF16), so the variants build in parallel.  Each build exports
// the three entry points that dl_grad.hip dispatches to.
#include "dl_grad_kernels.h"

#if !defined(DL_GV_MF) || !defined(DL_GV_A) || !defined(DL_GV_BF16)
#error "dl_grad_variant.hip needs DL_GV_MF, DL_GV_A and DL_GV_BF16"
#endif

#define DL_GV_CAT2(a, b, c, d) a##_##b##_##c##_##d
#define DL_GV_CAT(a, b, c, d) DL_GV_CAT2(a, b, c, d)
#define DL_GV_FN(base) DL_GV_CAT(base, DL_GV_MF, DL_GV_A, DL_GV_BF16)

namespace {
constexpr int GV_MF = DL_GV_MF;
constexpr bool GV_A = DL_GV_A != 0;
constexpr int GV_KMAX = (GV_A && GV_MF > 1) ? DL_KMAX_A : DL_KMAX_PLAIN;
using GV_TV = std::conditional_t<DL_GV_BF16 != 0, uint16_t, float>;
}  // namespace

dl_status DL_GV_FN(dl_grad_launch_v)(const dl_problem* P, int mode, const dl_grad_args& A, size_t lds) {
  return launch_mode<GV_MF, GV_A, GV_KMAX, GV_TV>(P, mode, A, lds);
}

dl_status DL_GV_FN(dl_grad_batch_v)(const dl_problem* P, int n_wg, const dl_grad_args* d_args,
                                    const dl_wg_desc* d_wgs, size_t lds, hipStream_t st, int mode) {
  return launch_batch_t<GV_MF, GV_A, GV_KMAX, GV_TV>(P, n_wg, d_args, d_wgs, lds, st, mode);
}

void DL_GV_FN(dl_grad_attr_v)() { set_attr_all<GV_MF, GV_A, GV_KMAX, GV_TV>(); }
