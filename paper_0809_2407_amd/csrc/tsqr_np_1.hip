// Explicit instantiations of the TSQR kernels for padded column counts 20, 24, 28, 32.
#include "tsqr_kernels.h"

namespace tsqr {

#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 20
template hipError_t leaf_factor_np<20>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<20>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<20>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<20>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<20>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<20>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 24
template hipError_t leaf_factor_np<24>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<24>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<24>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<24>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<24>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<24>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 28
template hipError_t leaf_factor_np<28>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<28>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<28>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<28>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<28>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<28>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 32
template hipError_t leaf_factor_np<32>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, hipStream_t);
template hipError_t tree_np<32>(const Layout&, double*, bool, hipStream_t);
template hipError_t root_np<32>(const Layout&, double*, double*, int64_t, hipStream_t);
template hipError_t seeds_np<32>(const Layout&, double*, hipStream_t);
template hipError_t form_q_np<32>(const Layout&, const double*, int64_t, double*, double*, int64_t, hipStream_t);
template hipError_t apply_qt_np<32>(const Layout&, const double*, int64_t, int64_t, double*, int64_t, double*, hipStream_t);
#endif

}  // namespace tsqr
