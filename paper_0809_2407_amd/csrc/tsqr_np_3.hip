// Explicit instantiations of the TSQR kernels for padded column counts 52, 56, 60, 64.
#include "tsqr_kernels.h"

namespace tsqr {

#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 52
template hipError_t leaf_factor_np<52>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<52>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<52>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<52>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<52>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<52>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 56
template hipError_t leaf_factor_np<56>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<56>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<56>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<56>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<56>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<56>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 60
template hipError_t leaf_factor_np<60>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<60>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<60>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<60>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<60>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<60>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 64
template hipError_t leaf_factor_np<64>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<64>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<64>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<64>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<64>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<64>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif

}  // namespace tsqr
