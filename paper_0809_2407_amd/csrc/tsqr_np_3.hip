// Explicit instantiations of the TSQR kernels for padded column counts 52, 56, 64
// (widths 57-60 run on the 64-column kernels: see padded_width).
#include "tsqr_kernels.h"

namespace tsqr {

#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 52
TSQR_INSTANTIATE(52)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 56
TSQR_INSTANTIATE(56)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 64
TSQR_INSTANTIATE(64)
#endif

}  // namespace tsqr
