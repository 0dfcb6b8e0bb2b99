// Explicit instantiations of the TSQR kernels for padded column counts 36, 40, 44, 48.
#include "tsqr_kernels.h"

namespace tsqr {

#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 36
template hipError_t leaf_factor_np<36>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<36>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<36>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<36>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<36>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<36>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 40
template hipError_t leaf_factor_np<40>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<40>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<40>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<40>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<40>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<40>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 44
template hipError_t leaf_factor_np<44>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<44>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<44>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<44>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<44>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<44>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 48
template hipError_t leaf_factor_np<48>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<48>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<48>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<48>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<48>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<48>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif

}  // namespace tsqr
