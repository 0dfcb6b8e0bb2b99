// Explicit instantiations of the TSQR kernels for padded column counts 4, 8, 12, 16.
#include "tsqr_kernels.h"

namespace tsqr {

#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 4
TSQR_INSTANTIATE(4)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 8
TSQR_INSTANTIATE(8)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 12
TSQR_INSTANTIATE(12)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 16
TSQR_INSTANTIATE(16)
#endif

}  // namespace tsqr
