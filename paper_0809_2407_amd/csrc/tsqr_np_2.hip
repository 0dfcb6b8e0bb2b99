// Explicit instantiations of the TSQR kernels for padded column counts 36, 40, 44, 48.
#include "tsqr_kernels.h"

namespace tsqr {

#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 36
TSQR_INSTANTIATE(36)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 40
TSQR_INSTANTIATE(40)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 44
TSQR_INSTANTIATE(44)
#endif
#if !defined(TSQR_ONLY_NP) || TSQR_ONLY_NP == 48
TSQR_INSTANTIATE(48)
#endif

}  // namespace tsqr
