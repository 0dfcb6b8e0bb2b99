// Explicit instantiations of the TSQR kernels for padded column counts 56, 64
// (widths 49-52 run on the 56-column kernels, 57-60 on the 64-column ones:
// see padded_width).
#include "tsqr_kernels.h"

namespace tsqr {

#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 56
TSQR_INSTANTIATE(56)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 64
TSQR_INSTANTIATE(64)
#endif

}  // namespace tsqr
