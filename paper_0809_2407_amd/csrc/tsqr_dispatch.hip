// tsqr_dispatch.hip -- selects the instantiation for the padded column count.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsqr_internal.h"

namespace tsqr {

#ifdef TSQR_ONLY_NP
// experiment builds: a single column count
#define TSQR_NP_SWITCH(np, CALL)                                                                      \
    switch (np) {                                                                                     \
    case TSQR_ONLY_NP: return CALL(TSQR_ONLY_NP);                                                     \
    default: return hipErrorInvalidValue;                                                             \
    }
#else
#define TSQR_NP_SWITCH(np, CALL)                                                                      \
    switch (np) {                                                                                     \
    case 4: return CALL(4);                                                                           \
    case 8: return CALL(8);                                                                           \
    case 12: return CALL(12);                                                                         \
    case 16: return CALL(16);                                                                         \
    case 20: return CALL(20);                                                                         \
    case 24: return CALL(24);                                                                         \
    case 28: return CALL(28);                                                                         \
    case 32: return CALL(32);                                                                         \
    case 36: return CALL(36);                                                                         \
    case 40: return CALL(40);                                                                         \
    case 44: return CALL(44);                                                                         \
    case 48: return CALL(48);                                                                         \
    case 56: return CALL(56);                                                                         \
    case 64: return CALL(64);                                                                         \
    default: return hipErrorInvalidValue;                                                             \
    }
#endif

hipError_t launch_leaf_factor(const Layout& L, const double* A, int64_t lda, double* V, int64_t ldv, double* ws,
                              bool want_q, hipStream_t s)
{
#define CALL(NP) leaf_factor_np<NP>(L, A, lda, V, ldv, ws, want_q, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

hipError_t launch_tree(const Layout& L, double* ws, bool want_q, hipStream_t s)
{
#define CALL(NP) tree_np<NP>(L, ws, want_q, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

hipError_t launch_root(const Layout& L, double* ws, double* R, int64_t ldr, hipStream_t s)
{
#define CALL(NP) root_np<NP>(L, ws, R, ldr, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

hipError_t launch_seeds(const Layout& L, double* ws, hipStream_t s)
{
#define CALL(NP) seeds_np<NP>(L, ws, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

hipError_t launch_form_q(const Layout& L, const double* A, int64_t lda, double* ws, double* Q, int64_t ldq,
                         hipStream_t s)
{
#define CALL(NP) form_q_np<NP>(L, A, lda, ws, Q, ldq, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

hipError_t launch_apply_qt(const Layout& L, const double* A, int64_t lda, int64_t k, double* B, int64_t ldb,
                           double* ws, hipStream_t s)
{
#define CALL(NP) apply_qt_np<NP>(L, A, lda, k, B, ldb, ws, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

hipError_t launch_mixed_leaf(const Layout& L, const double* A, int64_t lda, double* ws, bool want_q, hipStream_t s)
{
#define CALL(NP) mixed_leaf_np<NP>(L, A, lda, ws, want_q, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

hipError_t launch_build_T(const Layout& L, double* ws, hipStream_t s)
{
#define CALL(NP) build_T_np<NP>(L, ws, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

int leaf_lds_bytes(int np, bool mixed, bool want_q)
{
#if defined(TSQR_ONLY_NP)
    return np == TSQR_ONLY_NP ? leaf_lds_bytes_np<TSQR_ONLY_NP>(mixed, want_q) : 0;
#else
    switch (np) {
#define CASE(NP) \
    case NP: return leaf_lds_bytes_np<NP>(mixed, want_q);
        CASE(4) CASE(8) CASE(12) CASE(16) CASE(20) CASE(24) CASE(28) CASE(32)
        CASE(36) CASE(40) CASE(44) CASE(48) CASE(56) CASE(64)
#undef CASE
    default: return 0;
    }
#endif
}

hipError_t launch_form_q1(const Layout& L, double* ws, hipStream_t s)
{
#define CALL(NP) form_q1_np<NP>(L, ws, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

hipError_t launch_reorth(const Layout& L, double* ws, double* R, int64_t ldr, hipStream_t s)
{
#define CALL(NP) reorth_np<NP>(L, ws, R, ldr, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

hipError_t launch_reorth_q(const Layout& L, double* ws, double* Q, int64_t ldq, hipStream_t s)
{
#define CALL(NP) reorth_q_np<NP>(L, ws, Q, ldq, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

hipError_t launch_qtb_mixed(const Layout& L, double* ws, int64_t k, double* B, int64_t ldb, hipStream_t s)
{
#define CALL(NP) qtb_mixed_np<NP>(L, ws, k, B, ldb, s)
    TSQR_NP_SWITCH(L.np, CALL)
#undef CALL
}

hipError_t launch_batch_factor(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                               bool want_q, int waves, hipStream_t s)
{
#define CALL(NP) batch_factor_np<NP>(C, probs, args, ws, want_q, waves, s)
    TSQR_NP_SWITCH(C.np, CALL)
#undef CALL
}

hipError_t launch_batch_form_q(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                               int waves, bool alias, hipStream_t s)
{
#define CALL(NP) batch_form_q_np<NP>(C, probs, args, ws, waves, alias, s)
    TSQR_NP_SWITCH(C.np, CALL)
#undef CALL
}

hipError_t launch_batch_factor_mixed(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args,
                                     double* ws, bool want_q, int waves, hipStream_t s)
{
#define CALL(NP) batch_factor_mixed_np<NP>(C, probs, args, ws, want_q, waves, s)
    TSQR_NP_SWITCH(C.np, CALL)
#undef CALL
}

hipError_t launch_batch_form_q_mixed(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args,
                                     double* ws, hipStream_t s)
{
#define CALL(NP) batch_form_q_mixed_np<NP>(C, probs, args, ws, s)
    TSQR_NP_SWITCH(C.np, CALL)
#undef CALL
}

}  // namespace tsqr
