// Explicit instantiations of the TSQR kernels for padded column counts 4, 8, 12, 16.
#include "tsqr_kernels.h"

namespace tsqr {

#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 4
template hipError_t leaf_factor_np<4>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<4>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<4>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<4>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<4>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<4>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 8
template hipError_t leaf_factor_np<8>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<8>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<8>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<8>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<8>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<8>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 12
template hipError_t leaf_factor_np<12>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<12>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<12>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<12>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<12>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<12>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 16
template hipError_t leaf_factor_np<16>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<16>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<16>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<16>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<16>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<16>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif

}  // namespace tsqr
