// tsqr_caqr.hip -- CAQR on one GPU (Sec. 6, Alg. 3): the QR factorization
// of a general m x n matrix (m >= n) by panels of b columns, each panel
// factored by TSQR and its Q^T -- the leaf updates and the updates up the
// reduction tree (D = C_0 + Y^T C_1, C_0 -= T^T D, C_1 -= Y T^T D, Sec. 3.2)
// -- applied to the trailing matrix (right-looking).
//
// Step j works on the active matrix A[jb:, jb:] of m_j = m - jb rows:
//   1. TSQR of the panel A[jb:, jb:jb+b] (reflectors in place, the panel's R
//      to R[jb:jb+b, jb:jb+b]);
//   2. the trailing columns A[jb:, jb+b:] <- Q_j^T A[jb:, jb+b:] (tsqr_apply_qt):
//      their top b rows become R[jb:jb+b, jb+b:], the rest is the next
//      active matrix, in the coordinates of the complement of the panel's
//      column space that the panel's tree defines.
// R is unique up to the signs of its rows (Sec. 2), which the panel TSQRs
// normalise (diag >= 0).  Q stays implicit: the panels' reflectors in A and
// the panels' trees in the plan; tsqr_caqr_apply_qt applies Q^T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "tsqr.h"
#include "tsqr_internal.h"

struct tsqr_caqr_plan_s {
    int64_t m = 0, n = 0, b = 0;
    hipStream_t stream = nullptr;
    std::vector<tsqr_plan> panels;  // TSQR plan of panel j: (m - jb) x min(b, n - jb)
    int state = 0;                  // 1 after a factorisation
};

namespace {

// The part of R below the diagonal blocks: zero (the panels write the rest).
__global__ void __launch_bounds__(256) k_caqr_zero_lower(double* R, int64_t ldr, int64_t n)
{
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % n, j = e / n;
        if (i > j) R[i + j * ldr] = 0.0;
    }
}

tsqr_status caqr_hip(hipError_t e) { return e == hipSuccess ? 0 : (e == hipErrorOutOfMemory ? 2 : 1); }

void release(tsqr_caqr_plan_s* p)
{
    for (tsqr_plan q : p->panels)
        if (q) tsqr_plan_destroy(q);
    delete p;
}

}  // namespace

extern "C" {

tsqr_status tsqr_caqr_plan_create(tsqr_caqr_plan* out, int64_t m, int64_t n, int64_t panel, void* hip_stream)
{
    if (!out) return -1;
    *out = nullptr;
    if (m < 0 || m < n) return -2;
    if (n < 0) return -3;  // n = 0: a plan with no panels
    if (panel < 0 || panel > tsqr::kMaxN) return -4;
    tsqr_caqr_plan_s* p = new (std::nothrow) tsqr_caqr_plan_s();
    if (!p) return 2;
    p->m = m;
    p->n = n;
    p->b = panel > 0 ? panel : std::max<int64_t>(1, std::min<int64_t>(32, n));
    p->stream = (hipStream_t)hip_stream;
    tsqr_opts o = {};
    o.want_q = 1;
    for (int64_t j0 = 0; j0 < n; j0 += p->b) {
        const int64_t w = std::min<int64_t>(p->b, n - j0);
        tsqr_plan q = nullptr;
        const tsqr_status st = tsqr_plan_create(&q, m - j0, w, TSQR_FP64, &o, hip_stream);
        if (st != 0) {
            release(p);
            return st;
        }
        p->panels.push_back(q);
    }
    *out = p;
    return 0;
}

}  // extern "C"

namespace {

// Alg. 3 on [A B]: the k columns after A's n (same array, same lda) are
// updated with the trailing matrix, panel by panel.
tsqr_status caqr_factor(tsqr_caqr_plan p, double* A, int64_t lda, double* R, int64_t ldr, int64_t k)
{
    p->state = 0;
    const int64_t n = p->n, b = p->b;
    if (n == 0) {  // no columns: nothing to factor, Q = I leaves the right-hand sides
        p->state = 1;
        return 0;
    }
    // the strictly lower part of R is zero; the panels fill the rest
    hipLaunchKernelGGL(k_caqr_zero_lower, dim3((unsigned)std::min<int64_t>(1024, (n * n + 255) / 256)), dim3(256), 0,
                       p->stream, R, ldr, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return caqr_hip(e);
    for (size_t j = 0; j < p->panels.size(); ++j) {
        const int64_t j0 = (int64_t)j * b, w = std::min<int64_t>(b, n - j0);
        double* Aj = A + j0 + j0 * lda;  // the active matrix
        tsqr_status st = tsqr_factor(p->panels[j], Aj, lda, R + j0 + j0 * ldr, ldr);
        if (st != 0) return st;
        const int64_t rest = n - j0 - w;
        if (rest + k == 0) break;
        // one pass of Q_j^T over the trailing columns and the right-hand sides
        double* C = Aj + w * lda;
        st = tsqr_apply_qt(p->panels[j], Aj, lda, rest + k, C, lda);
        if (st != 0) return st;
        if (rest == 0) continue;
        // the top w rows of the updated trailing columns are R's row block
        e = hipMemcpy2DAsync(R + j0 + (j0 + w) * ldr, (size_t)ldr * sizeof(double), C, (size_t)lda * sizeof(double),
                             (size_t)w * sizeof(double), (size_t)rest, hipMemcpyDeviceToDevice, p->stream);
        if (e != hipSuccess) return caqr_hip(e);
    }
    p->state = 1;
    return 0;
}

}  // namespace

extern "C" {

tsqr_status tsqr_caqr_factor(tsqr_caqr_plan p, double* A, int64_t lda, double* R, int64_t ldr)
{
    if (!p) return -1;
    if (!A && p->n > 0) return -2;  // an empty problem references no matrix
    if (lda < p->m) return -3;
    if (!R && p->n > 0) return -4;
    if (ldr < p->n) return -5;
    return caqr_factor(p, A, lda, R, ldr, 0);
}

tsqr_status tsqr_caqr_factor_rhs(tsqr_caqr_plan p, double* A, int64_t lda, double* R, int64_t ldr, int64_t k)
{
    if (!p) return -1;
    if (!A && p->n > 0) return -2;  // an empty problem references no matrix
    if (lda < p->m) return -3;
    if (!R && p->n > 0) return -4;
    if (ldr < p->n) return -5;
    if (k < 0) return -6;
    return caqr_factor(p, A, lda, R, ldr, k);
}

tsqr_status tsqr_caqr_apply_qt(tsqr_caqr_plan p, const double* A, int64_t lda, int64_t k, double* B, int64_t ldb)
{
    if (!p) return -1;
    if (!A && p->n > 0) return -2;
    if (lda < p->m) return -3;
    if (k < 0) return -4;
    if (k == 0) return 0;
    if (!B && p->m > 0) return -5;  // a 0 x k B is not referenced
    if (ldb < p->m) return -6;
    if (p->state != 1) return 4;
    // Q^T = ... Q_1^T Q_0^T: panel j acts on rows jb .. of B
    for (size_t j = 0; j < p->panels.size(); ++j) {
        const int64_t j0 = (int64_t)j * p->b;
        const tsqr_status st = tsqr_apply_qt(p->panels[j], A + j0 + j0 * lda, lda, k, B + j0, ldb);
        if (st != 0) return st;
    }
    return 0;
}

tsqr_status tsqr_caqr_plan_info(tsqr_caqr_plan p, int64_t* panel, int64_t* npanels)
{
    if (!p) return -1;
    if (!panel) return -2;
    if (!npanels) return -3;
    *panel = p->b;
    *npanels = (int64_t)p->panels.size();
    return 0;
}

tsqr_status tsqr_caqr_plan_destroy(tsqr_caqr_plan p)
{
    if (!p) return -1;
    // a plan with no panels (n = 0) never enqueued work
    hipError_t e = p->panels.empty() ? hipSuccess : hipStreamSynchronize(p->stream);
    release(p);
    return caqr_hip(e);
}

}  // extern "C"
