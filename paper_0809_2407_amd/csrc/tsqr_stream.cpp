// tsqr_stream.cpp -- out-of-HBM TSQR: a matrix in host memory, streamed
// through the GPU in row blocks (the out-of-DRAM sequential TSQR of Sec. 7.1,
// Alg. 2, moved one level up the memory hierarchy: HBM is the fast memory,
// host memory the slow one).
//
// A flat tree over the blocks: R_0 from [0; A_0], then R_k = qr([R_{k-1}; A_k]),
// each stacked block factored on the device by this library's TSQR (leaf
// chains, binary tree, R only).  The device holds two stacked-block buffers:
// while block k is factored on the plan's stream, block k + 1 is copied in on
// a copy stream of its own (events order the two), so the host-to-device
// transfer overlaps the factorisation -- the overlap the paper's out-of-DRAM
// code left out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>

#include "tsqr.h"
#include "tsqr_internal.h"

struct tsqr_stream_plan_s {
    int64_t m = 0, n = 0, b = 0;      // rows, columns, rows per block
    int64_t nblocks = 0, b_last = 0;  // blocks; rows of the last one
    hipStream_t stream = nullptr;     // the caller's (compute) stream
    hipStream_t copy = nullptr;       // host-to-device copies
    double* X[2] = {nullptr, nullptr};  // stacked blocks [R; A_k], (n + b) x n, ld n + b
    double* Rd = nullptr;             // running R, n x n, ld n
    double* zeros = nullptr;          // n x n zeros: the R above the first block
    tsqr_plan full = nullptr, last = nullptr;  // R-only TSQR plans of n + b and n + b_last rows
    hipEvent_t copied[2] = {nullptr, nullptr}, done[2] = {nullptr, nullptr};
};

namespace {

tsqr_status st_hip(hipError_t e) { return e == hipSuccess ? 0 : (e == hipErrorOutOfMemory ? 2 : 1); }

void release(tsqr_stream_plan_s* p)
{
    if (p->stream) hipStreamSynchronize(p->stream);
    if (p->copy) {
        hipStreamSynchronize(p->copy);
        hipStreamDestroy(p->copy);
    }
    for (int i = 0; i < 2; ++i) {
        if (p->X[i]) hipFree(p->X[i]);
        if (p->copied[i]) hipEventDestroy(p->copied[i]);
        if (p->done[i]) hipEventDestroy(p->done[i]);
    }
    if (p->Rd) hipFree(p->Rd);
    if (p->zeros) hipFree(p->zeros);
    if (p->full) tsqr_plan_destroy(p->full);
    if (p->last && p->last != p->full) tsqr_plan_destroy(p->last);
    delete p;
}

}  // namespace

extern "C" {

tsqr_status tsqr_stream_plan_create(tsqr_stream_plan* out, int64_t m, int64_t n, int64_t block_rows, void* hip_stream)
{
    if (!out) return -1;
    *out = nullptr;
    if (m < 1 || m < n) return -2;
    if (n < 1) return -3;
    if (n > tsqr::kMaxN) return 3;
    if (block_rows < 0 || (block_rows > 0 && block_rows < n)) return -4;
    tsqr_stream_plan_s* p = new (std::nothrow) tsqr_stream_plan_s();
    if (!p) return 2;
    p->m = m;
    p->n = n;
    // automatic: blocks of about 1 GiB
    const int64_t b = block_rows > 0 ? block_rows : std::max<int64_t>(n, ((int64_t)1 << 27) / n);
    p->b = std::min<int64_t>(b, m);
    p->nblocks = (m + p->b - 1) / p->b;
    p->b_last = m - (p->nblocks - 1) * p->b;
    if (p->b_last < n && p->nblocks > 1) {
        // a last block of fewer than n rows joins the one before it
        p->nblocks -= 1;
        p->b_last += p->b;
    }
    p->stream = (hipStream_t)hip_stream;
    const int64_t rows = n + std::max(p->b, p->b_last);
    tsqr_opts o = {};
    o.want_q = 0;
    hipError_t e = hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipMalloc((void**)&p->X[i], (size_t)rows * n * sizeof(double));
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->copied[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipMalloc((void**)&p->Rd, (size_t)n * n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&p->zeros, (size_t)n * n * sizeof(double));
    if (e == hipSuccess) e = hipMemset(p->zeros, 0, (size_t)n * n * sizeof(double));
    if (e != hipSuccess) {
        release(p);
        return st_hip(e);
    }
    tsqr_status st = tsqr_plan_create(&p->full, n + p->b, n, TSQR_FP64, &o, hip_stream);
    if (st == 0 && p->b_last != p->b) st = tsqr_plan_create(&p->last, n + p->b_last, n, TSQR_FP64, &o, hip_stream);
    else if (st == 0) p->last = p->full;
    if (st != 0) {
        release(p);
        return st;
    }
    *out = p;
    return 0;
}

tsqr_status tsqr_stream_factor(tsqr_stream_plan p, const double* A, int64_t lda, double* R, int64_t ldr)
{
    if (!p) return -1;
    if (!A) return -2;
    if (lda < p->m) return -3;
    if (!R) return -4;
    if (ldr < p->n) return -5;
    const int64_t n = p->n;
    hipError_t e = hipSuccess;
    // the copy stream starts after earlier work on the caller's stream (which
    // may still be reading the buffers)
    e = hipEventRecord(p->done[1], p->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->copy, p->done[1], 0);
    for (int64_t k = 0; k < p->nblocks && e == hipSuccess; ++k) {
        const int buf = (int)(k & 1);
        const bool last = k == p->nblocks - 1;
        const int64_t rows = last ? p->b_last : p->b, ldx = n + rows;
        double* X = p->X[buf];
        // copy stream: block k into rows n .. of its buffer, once the
        // factorisation of block k - 2 no longer reads the buffer
        if (k >= 2) e = hipStreamWaitEvent(p->copy, p->done[buf], 0);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(X + n, (size_t)ldx * sizeof(double), A + k * p->b, (size_t)lda * sizeof(double),
                                 (size_t)rows * sizeof(double), (size_t)n, hipMemcpyHostToDevice, p->copy);
        if (e == hipSuccess) e = hipEventRecord(p->copied[buf], p->copy);
        // compute stream: [R_{k-1}; A_k] (zeros above the first block), then its R
        if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->copied[buf], 0);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(X, (size_t)ldx * sizeof(double), k == 0 ? p->zeros : p->Rd, (size_t)n * sizeof(double),
                                 (size_t)n * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice, p->stream);
        if (e != hipSuccess) break;
        tsqr_status st = tsqr_factor(last ? p->last : p->full, X, ldx, p->Rd, n);
        if (st != 0) return st;
        e = hipEventRecord(p->done[buf], p->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(R, (size_t)ldr * sizeof(double), p->Rd, (size_t)n * sizeof(double),
                             (size_t)n * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice, p->stream);
    return st_hip(e);
}

tsqr_status tsqr_stream_plan_info(tsqr_stream_plan p, int64_t* block_rows, int64_t* nblocks)
{
    if (!p) return -1;
    if (!block_rows) return -2;
    if (!nblocks) return -3;
    *block_rows = p->b;
    *nblocks = p->nblocks;
    return 0;
}

tsqr_status tsqr_stream_plan_destroy(tsqr_stream_plan p)
{
    if (!p) return -1;
    hipError_t e = hipStreamSynchronize(p->stream);
    release(p);
    return st_hip(e);
}

}  // extern "C"
