// Explicit instantiations of the TSQR kernels for padded column counts 20, 24, 28, 32.
#include "tsqr_kernels.h"

namespace tsqr {

#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 20
TSQR_INSTANTIATE(20)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 24
TSQR_INSTANTIATE(24)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 28
TSQR_INSTANTIATE(28)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 32
TSQR_INSTANTIATE(32)
#endif

}  // namespace tsqr
