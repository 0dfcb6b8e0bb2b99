// tsqr_cmp.hip -- TSQR's competitors of Sec. 5 on the GPU, for the stability
// and cost contrast the paper draws: CholeskyQR (G = A^T A = R^T R, Q =
// A R^{-1}), CholeskyQR applied twice, classical Gram-Schmidt (CGS) and
// modified Gram-Schmidt (MGS).  All in FP64.
//
// CholeskyQR: partial Gram matrices of row groups on the f64 matrix cores
// (k_cmp_gram), the two-stage pairwise sum of the mixed path's second pass,
// one wavefront for the Cholesky factor, its inverse and (second pass of
// CholeskyQR2) R = R2 R1 (k_cmp_chol), and Q = A R^{-1} on the matrix cores
// (reorth_q_blocks).  Reads A twice and writes Q once (24mn bytes; CholeskyQR2
// 48mn).
//
// Gram-Schmidt: one pass over the rows per reduction the method needs, each
// workgroup a chunk of rows with a fixed summation order, then a reduction of
// the per-workgroup partial sums (k_gs_reduce), so results are deterministic.
//   MGS, step j (one pass): finish q_{j-1} = v_{j-1} / r_{j-1,j-1}, update
//     v_k -= r_{j-1,k} q_{j-1} (k >= j), and sum v_j^T v_k (k >= j) -- the
//     norm of v_j and its products with the later columns in the same pass,
//     so r_jj = sqrt(v_j^T v_j) and r_jk = (v_j^T v_k) / r_jj: the
//     coefficients q_j^T v_k of MGS with the normalisation applied after the
//     sum instead of before it.
//   CGS, step j (two passes): finish q_{j-1} and sum q_i^T a_j (i < j, a_j the
//     column of A); then v_j = a_j - sum_i r_ij q_i and its squared norm.
// Traffic: about 8mn^2 bytes for either (one pass over the trailing or the
// leading columns per step).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>

#include "tsqr.h"
#include "tsqr_kernels.h"

namespace tsqr {
namespace detail {

// ---- CholeskyQR -------------------------------------------------------------

// Partial Gram matrices of an FP64 column-major m x n matrix: wavefront w sums
// rows [w rw, (w + 1) rw) (rw a multiple of 64) into the upper blocks of its
// NPB x NPB slot of Gp.  In k-step s of a 64-row group, lane (q, p) supplies
// row 16 q + s of column 16 b + p: a lane reads 16 consecutive doubles of one
// column per block.  Rows past m and columns past n count as zero.
template <int NPB>
__global__ void __launch_bounds__(256) k_cmp_gram(const double* __restrict__ A, int64_t lda, int64_t m, int n,
                                                  int64_t rw, int64_t nw, double* __restrict__ Gp)
{
    constexpr int JB = NPB / 16;
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (w >= nw) return;
    const int q = lane >> 4, p = lane & 15;
    dbl4 acc[JB][JB];
#pragma unroll
    for (int ib = 0; ib < JB; ++ib)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) acc[ib][jb] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int64_t r0 = w * rw, r1 = (r0 + rw) < m ? (r0 + rw) : m;
    for (int64_t g = r0; g < r1; g += 64) {
        double x[JB][16];
        const bool full = g + 64 <= m;
#pragma unroll
        for (int b = 0; b < JB; ++b) {
            const int c = 16 * b + p, cc = c < n ? c : n - 1;
            const double* src = A + g + 16 * q + (int64_t)cc * lda;
            if (full) {
#pragma unroll
                for (int v = 0; v < 16; ++v) x[b][v] = src[v];
            } else {
                // the ragged last group: a row past m reads row m - 1, then counts as zero
                const int64_t row0 = g + 16 * q;
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t rr = row0 + v < m ? row0 + v : m - 1;
                    const double y = A[rr + (int64_t)cc * lda];
                    x[b][v] = row0 + v < m ? y : 0.0;
                }
            }
            if (c >= n) {
#pragma unroll
                for (int v = 0; v < 16; ++v) x[b][v] = 0.0;
            }
        }
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int ib = 0; ib < JB; ++ib)
#pragma unroll
                for (int jb = ib; jb < JB; ++jb) acc[ib][jb] = mfma16x16x4(x[ib][s], x[jb][s], acc[ib][jb]);
    }
    double* G = Gp + w * NPB * NPB;
#pragma unroll
    for (int ib = 0; ib < JB; ++ib)
#pragma unroll
        for (int jb = ib; jb < JB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) G[(16 * ib + q + 4 * r) + (16 * jb + p) * NPB] = acc[ib][jb][r];
}

template <int NPB>
__host__ __device__ constexpr int chol_lds_doubles() { return 3 * NPB * (NPB + 1); }

// One wavefront: the Cholesky factor R of G (its upper triangle, NPB x NPB,
// n x n used), R^{-1} (NPB x NPB, zero past n) and the caller's R -- R itself,
// or R R1 when R1 is given (the second pass of CholeskyQR2).  A pivot that is
// not positive stops the factorisation: R^{-1} is then zero (so Q comes out
// zero), the caller's R zero, and info records column + 1 (the first pass
// overwrites info, later ones keep an earlier breakdown).  Rkeep (may be
// NULL) receives R (NPB x NPB).
template <int NPB>
__global__ void __launch_bounds__(64) k_cmp_chol(const double* __restrict__ G, int n, const double* __restrict__ R1,
                                                 double* __restrict__ R, int64_t ldr, double* __restrict__ Rkeep,
                                                 double* __restrict__ Rinv, int* __restrict__ info, int first)
{
    constexpr int LD = NPB + 1;
    extern __shared__ double smem[];
    double* Gs = smem;            // G, then R
    double* Xl = Gs + NPB * LD;   // R^{-1}
    double* Rl = Xl + NPB * LD;   // R1
    const int lane = threadIdx.x;
    for (int e = lane; e < NPB * NPB; e += 64) {
        const int i = e % NPB, j = e / NPB;
        if (i <= j) {
            const double g = (j < n) ? G[e] : (i == j ? 1.0 : 0.0);
            Gs[i + j * LD] = g;
            Gs[j + i * LD] = g;
        }
        Rl[i + j * LD] = (R1 && i < n && j < n) ? R1[i + j * NPB] : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    int bad = 0;
    for (int k = 0; k < n; ++k) {
        const double dkk = Gs[k + k * LD];  // the same LDS word for every lane: a uniform decision
        if (!(dkk > 0.0)) {
            bad = k + 1;
            break;
        }
        const double d = sqrt(dkk);
        __syncthreads();
        for (int j = lane; j < n; j += 64) {
            if (j > k) Gs[k + j * LD] /= d;
            if (j == k) Gs[k + k * LD] = d;
        }
        __syncthreads();
        for (int j = lane; j < n; j += 64)
            if (j > k) {
                const double rkj = Gs[k + j * LD];
                for (int i = k + 1; i <= j; ++i) Gs[i + j * LD] = fma(-Gs[k + i * LD], rkj, Gs[i + j * LD]);
            }
        __syncthreads();
    }
    // R^{-1} by back substitution, column j by lane j (it reads back only its own writes)
    for (int j = lane; j < NPB; j += 64) {
        for (int i = 0; i < NPB; ++i) Xl[i + j * LD] = 0.0;
        if (!bad && j < n) {
            Xl[j + j * LD] = 1.0 / Gs[j + j * LD];
            for (int i = j - 1; i >= 0; --i) {
                const double acc = lds_dot(Gs + i, LD, Xl + j * LD, i + 1, j + 1);
                Xl[i + j * LD] = -acc / Gs[i + i * LD];
            }
        }
    }
    __syncthreads();
    for (int e = lane; e < NPB * NPB; e += 64) {
        const int i = e % NPB, j = e / NPB;
        Rinv[e] = Xl[i + j * LD];
        if (Rkeep) Rkeep[e] = (!bad && i <= j && j < n) ? Gs[i + j * LD] : 0.0;
    }
    // the caller's R: R (R1 == NULL) or R R1, upper times upper; column j by lane j
    for (int j = lane; j < n; j += 64)
        for (int i = 0; i < n; ++i)
            R[i + (int64_t)j * ldr] = (!bad && i <= j) ? lds_dot(Gs + i, LD, Rl + j * LD, i, j + 1) : 0.0;
    if (lane == 0) {
        if (first) *info = bad;
        else if (*info == 0) *info = bad;
    }
}

template <int NPB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_cmp_apply_rinv(const double* A, int64_t lda, int64_t m, int n, const double* __restrict__ Rinv, double* Q,
                 int64_t ldq, int64_t nblocks)
{
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    reorth_q_blocks<NPB, double>(A, lda, m, n, Rinv, Q, ldq, (int64_t)blockIdx.x * (blockDim.x >> 6) + wave,
                                 nblocks, nwaves, lane);
}

// ---- Gram-Schmidt -----------------------------------------------------------

constexpr int kGsThreads = 256, kGsRows = 16;           // rows per thread
constexpr int64_t kGsChunk = (int64_t)kGsThreads * kGsRows;  // rows per workgroup
constexpr int kGsMaxCols = 64;

// Sum over the workgroup (fixed order: a butterfly inside each wavefront, then
// the four wavefront sums in order); the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    const int wave = threadIdx.x >> 6;
    __syncthreads();  // red is reused by the next call
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// The coefficients of MGS step j - 1 from its sums s_k = v_{j-1}^T v_k
// (k >= j - 1): r = sqrt(s_{j-1}), r_{j-1,k} = s_k / r; a zero norm gives
// inv = 0 (q_{j-1} = 0) and records the breakdown.
struct GsPrev {
    double inv = 0.0;
    bool valid = false;
};

// MGS step j (see the file head).  sums holds the previous step's sums
// (s_k at index k); workgroup 0 writes row j - 1 of R.
__global__ void __launch_bounds__(kGsThreads) k_mgs_pass(double* X, int64_t ldx, int64_t m, int n, int j,
                                                         const double* __restrict__ sums,
                                                         double* __restrict__ partials, double* __restrict__ R,
                                                         int64_t ldr, int* __restrict__ info)
{
    __shared__ double red[4];
    __shared__ double coef[kGsMaxCols];
    __shared__ double inv_s;
    const int t = threadIdx.x;
    if (j > 0) {
        if (t == 0) {
            const double r = sqrt(sums[j - 1]);
            inv_s = r > 0.0 ? 1.0 / r : 0.0;
            if (blockIdx.x == 0) {
                R[(j - 1) + (int64_t)(j - 1) * ldr] = r;
                if (!(r > 0.0) && *info == 0) *info = j;
            }
        }
        __syncthreads();
        for (int k = j + t; k < n; k += kGsThreads) {
            const double c = sums[k] * inv_s;
            coef[k] = c;
            if (blockIdx.x == 0) R[(j - 1) + (int64_t)k * ldr] = c;
        }
        __syncthreads();
    }
    const double inv = j > 0 ? inv_s : 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * kGsChunk + t;
    double qv[kGsRows], aj[kGsRows];
    if (j > 0) {
        double* col = X + (int64_t)(j - 1) * ldx;
#pragma unroll
        for (int i = 0; i < kGsRows; ++i) {
            const int64_t r = r0 + (int64_t)i * kGsThreads;
            qv[i] = r < m ? col[r] * inv : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kGsRows; ++i) {
            const int64_t r = r0 + (int64_t)i * kGsThreads;
            if (r < m) col[r] = qv[i];
        }
    }
    for (int k = j; k < n; ++k) {
        double* col = X + (int64_t)k * ldx;
        const double c = j > 0 ? coef[k] : 0.0;
        double x[kGsRows];
#pragma unroll
        for (int i = 0; i < kGsRows; ++i) {
            const int64_t r = r0 + (int64_t)i * kGsThreads;
            x[i] = r < m ? col[r] : 0.0;
        }
        if (j > 0) {
#pragma unroll
            for (int i = 0; i < kGsRows; ++i) {
                const int64_t r = r0 + (int64_t)i * kGsThreads;
                x[i] = fma(-c, qv[i], x[i]);
                if (r < m) col[r] = x[i];
            }
        }
        if (k == j) {
#pragma unroll
            for (int i = 0; i < kGsRows; ++i) aj[i] = x[i];
        }
        double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
        for (int i = 0; i < kGsRows; i += 2) {
            acc0 = fma(aj[i], x[i], acc0);
            acc1 = fma(aj[i + 1], x[i + 1], acc1);
        }
        const double tot = block_sum(acc0 + acc1, red);
        if (t == 0) partials[(int64_t)blockIdx.x * kGsMaxCols + k] = tot;
    }
}

// CGS step j, first pass: q_{j-1} = v_{j-1} / r_{j-1,j-1} (norm2 holds
// ||v_{j-1}||^2) and the sums q_i^T a_j, i < j.
__global__ void __launch_bounds__(kGsThreads) k_cgs_dots(double* X, int64_t ldx, int64_t m, int j,
                                                         const double* __restrict__ norm2,
                                                         double* __restrict__ partials, double* __restrict__ R,
                                                         int64_t ldr, int* __restrict__ info)
{
    __shared__ double red[4];
    __shared__ double inv_s;
    const int t = threadIdx.x;
    if (t == 0) {
        const double r = j > 0 ? sqrt(norm2[0]) : 0.0;
        inv_s = r > 0.0 ? 1.0 / r : 0.0;
        if (j > 0 && blockIdx.x == 0) {
            R[(j - 1) + (int64_t)(j - 1) * ldr] = r;
            if (!(r > 0.0) && *info == 0) *info = j;
        }
    }
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * kGsChunk + t;
    double qv[kGsRows], aj[kGsRows];
    {
        const double* cj = X + (int64_t)j * ldx;
#pragma unroll
        for (int i = 0; i < kGsRows; ++i) {
            const int64_t r = r0 + (int64_t)i * kGsThreads;
            aj[i] = r < m ? cj[r] : 0.0;
        }
    }
    if (j > 0) {
        double* col = X + (int64_t)(j - 1) * ldx;
        const double inv = inv_s;
#pragma unroll
        for (int i = 0; i < kGsRows; ++i) {
            const int64_t r = r0 + (int64_t)i * kGsThreads;
            qv[i] = r < m ? col[r] * inv : 0.0;
            if (r < m) col[r] = qv[i];
        }
    }
    for (int i0 = 0; i0 < j; ++i0) {
        double x[kGsRows];
        if (i0 == j - 1) {
#pragma unroll
            for (int i = 0; i < kGsRows; ++i) x[i] = qv[i];
        } else {
            const double* col = X + (int64_t)i0 * ldx;
#pragma unroll
            for (int i = 0; i < kGsRows; ++i) {
                const int64_t r = r0 + (int64_t)i * kGsThreads;
                x[i] = r < m ? col[r] : 0.0;
            }
        }
        double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
        for (int i = 0; i < kGsRows; i += 2) {
            acc0 = fma(x[i], aj[i], acc0);
            acc1 = fma(x[i + 1], aj[i + 1], acc1);
        }
        const double tot = block_sum(acc0 + acc1, red);
        if (t == 0) partials[(int64_t)blockIdx.x * kGsMaxCols + i0] = tot;
    }
}

// CGS step j, second pass: v_j = a_j - sum_{i<j} r_ij q_i in place of a_j, and
// the sum of v_j^2; workgroup 0 writes R(0:j-1, j).
__global__ void __launch_bounds__(kGsThreads) k_cgs_update(double* X, int64_t ldx, int64_t m, int j,
                                                           const double* __restrict__ dots,
                                                           double* __restrict__ partials, double* __restrict__ R,
                                                           int64_t ldr)
{
    __shared__ double red[4];
    const int t = threadIdx.x;
    if (blockIdx.x == 0)
        for (int i = t; i < j; i += kGsThreads) R[i + (int64_t)j * ldr] = dots[i];
    const int64_t r0 = (int64_t)blockIdx.x * kGsChunk + t;
    double v[kGsRows];
    double* cj = X + (int64_t)j * ldx;
#pragma unroll
    for (int i = 0; i < kGsRows; ++i) {
        const int64_t r = r0 + (int64_t)i * kGsThreads;
        v[i] = r < m ? cj[r] : 0.0;
    }
    for (int i0 = 0; i0 < j; ++i0) {
        const double c = dots[i0];
        const double* col = X + (int64_t)i0 * ldx;
#pragma unroll
        for (int i = 0; i < kGsRows; ++i) {
            const int64_t r = r0 + (int64_t)i * kGsThreads;
            const double x = r < m ? col[r] : 0.0;
            v[i] = fma(-c, x, v[i]);
        }
    }
    double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
    for (int i = 0; i < kGsRows; i += 2) {
        const int64_t ra = r0 + (int64_t)i * kGsThreads, rb = ra + kGsThreads;
        if (ra < m) cj[ra] = v[i];
        if (rb < m) cj[rb] = v[i + 1];
        acc0 = fma(v[i], v[i], acc0);
        acc1 = fma(v[i + 1], v[i + 1], acc1);
    }
    const double tot = block_sum(acc0 + acc1, red);
    if (t == 0) partials[(int64_t)blockIdx.x * kGsMaxCols] = tot;
}

// sums[k] = sum over workgroups of partials[.][k], k in [k0, k1): one
// workgroup per column, a fixed order (strided thread sums, then block_sum).
__global__ void __launch_bounds__(kGsThreads) k_gs_reduce(const double* __restrict__ partials, int64_t nblocks,
                                                          int k0, double* __restrict__ sums)
{
    __shared__ double red[4];
    const int k = k0 + blockIdx.x;
    double a0 = 0.0, a1 = 0.0;
    int64_t b = threadIdx.x;
    for (; b + kGsThreads < nblocks; b += 2 * kGsThreads) {
        a0 += partials[b * kGsMaxCols + k];
        a1 += partials[(b + kGsThreads) * kGsMaxCols + k];
    }
    if (b < nblocks) a0 += partials[b * kGsMaxCols + k];
    const double tot = block_sum(a0 + a1, red);
    if (threadIdx.x == 0) sums[k] = tot;
}

// The last column: q_{n-1} = v_{n-1} / r_{n-1,n-1} (norm2 = ||v_{n-1}||^2).
__global__ void __launch_bounds__(kGsThreads) k_gs_finish(double* X, int64_t ldx, int64_t m, int n,
                                                          const double* __restrict__ norm2, double* __restrict__ R,
                                                          int64_t ldr, int* __restrict__ info)
{
    const double r = sqrt(norm2[0]);
    const double inv = r > 0.0 ? 1.0 / r : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        R[(n - 1) + (int64_t)(n - 1) * ldr] = r;
        if (!(r > 0.0) && *info == 0) *info = n;
    }
    double* col = X + (int64_t)(n - 1) * ldx;
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < m; row += (int64_t)gridDim.x * blockDim.x)
        col[row] *= inv;
}

// R = 0 (n x n) and info = 0 at the start of a factorisation.
__global__ void __launch_bounds__(256) k_cmp_init(double* R, int64_t ldr, int n, int* info)
{
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) R[e % n + (int64_t)(e / n) * ldr] = 0.0;
    if (threadIdx.x == 0) *info = 0;
}

// Column-major copy X <- A (m x n), for Gram-Schmidt with Q distinct from A.
__global__ void __launch_bounds__(256) k_cmp_copy(const double* __restrict__ A, int64_t lda, double* __restrict__ X,
                                                  int64_t ldx, int64_t m, int n)
{
    const int64_t total = m * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e % m, c = e / m;
        X[r + c * ldx] = A[r + c * lda];
    }
}

}  // namespace detail
}  // namespace tsqr

// ---- plans ------------------------------------------------------------------

struct tsqr_cmp_plan_s {
    int64_t m = 0, n = 0;
    int npb = 0;
    tsqr_cmp_method method = TSQR_CMP_CHOLQR;
    hipStream_t stream = nullptr;
    double* ws = nullptr;
    // CholeskyQR: partial, group and summed Gram matrices, R^{-1}, R1
    int64_t gram_waves = 0, gram_rows = 0;
    double *Gp = nullptr, *Gq = nullptr, *G = nullptr, *Rinv = nullptr, *R1 = nullptr;
    // Gram-Schmidt: per-workgroup partial sums and their totals
    int64_t gs_blocks = 0;
    double *partials = nullptr, *sums = nullptr;
    int* info = nullptr;
};

namespace {

using namespace tsqr::detail;

tsqr_status cmp_hip(hipError_t e) { return e == hipSuccess ? 0 : (e == hipErrorOutOfMemory ? 2 : 1); }

// One CholeskyQR of X (m x n) into Q: Gram, Cholesky (R to the caller, or
// R R1 when R1prev is given), Q = X R^{-1}.
template <int NPB>
hipError_t cholqr_pass(tsqr_cmp_plan_s* p, const double* X, int64_t ldx, double* Q, int64_t ldq, double* R,
                       int64_t ldr, const double* R1prev, double* Rkeep, bool first)
{
    hipStream_t s = p->stream;
    hipLaunchKernelGGL((k_cmp_gram<NPB>), dim3((unsigned)((p->gram_waves + 3) / 4)), dim3(256), 0, s, X, ldx, p->m,
                       (int)p->n, p->gram_rows, p->gram_waves, p->Gp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t ng = (p->gram_waves + 63) / 64;
    hipLaunchKernelGGL((k_gram_sum64<NPB>), dim3((NPB * NPB + 255) / 256, (unsigned)ng), dim3(256), 0, s, p->Gp,
                       p->gram_waves, p->Gq);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_gram_sum<NPB>), dim3((NPB * NPB + 255) / 256), dim3(256), 0, s, p->Gq, ng, p->G);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t lds = (size_t)chol_lds_doubles<NPB>() * sizeof(double);
    allow_lds(k_cmp_chol<NPB>, lds);
    hipLaunchKernelGGL((k_cmp_chol<NPB>), dim3(1), dim3(64), lds, s, p->G, (int)p->n, R1prev, R, ldr, Rkeep, p->Rinv,
                       p->info, first ? 1 : 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t nblocks = (p->m + 15) / 16;
    const int64_t waves = nblocks < 8192 ? nblocks : 8192;
    hipLaunchKernelGGL((k_cmp_apply_rinv<NPB>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, X, ldx, p->m,
                       (int)p->n, p->Rinv, Q, ldq, nblocks);
    return hipGetLastError();
}

template <int NPB>
hipError_t cholqr_np(tsqr_cmp_plan_s* p, const double* A, int64_t lda, double* Q, int64_t ldq, double* R,
                     int64_t ldr)
{
    if (p->method == TSQR_CMP_CHOLQR) return cholqr_pass<NPB>(p, A, lda, Q, ldq, R, ldr, nullptr, nullptr, true);
    // CholeskyQR2: Q1 = A R1^{-1} into Q, then the same on Q1 in place, R = R2 R1
    hipError_t e = cholqr_pass<NPB>(p, A, lda, Q, ldq, R, ldr, nullptr, p->R1, true);
    if (e == hipSuccess) e = cholqr_pass<NPB>(p, Q, ldq, Q, ldq, R, ldr, p->R1, nullptr, false);
    return e;
}

hipError_t cholqr(tsqr_cmp_plan_s* p, const double* A, int64_t lda, double* Q, int64_t ldq, double* R, int64_t ldr)
{
    switch (p->npb) {
    case 16: return cholqr_np<16>(p, A, lda, Q, ldq, R, ldr);
    case 32: return cholqr_np<32>(p, A, lda, Q, ldq, R, ldr);
    case 48: return cholqr_np<48>(p, A, lda, Q, ldq, R, ldr);
    case 64: return cholqr_np<64>(p, A, lda, Q, ldq, R, ldr);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gram_schmidt(tsqr_cmp_plan_s* p, const double* A, int64_t lda, double* Q, int64_t ldq, double* R,
                        int64_t ldr)
{
    hipStream_t s = p->stream;
    const int n = (int)p->n;
    const unsigned nb = (unsigned)p->gs_blocks;
    hipError_t e = hipSuccess;
    if ((const double*)Q != A) {
        hipLaunchKernelGGL(k_cmp_copy, dim3(2048), dim3(256), 0, s, A, lda, Q, ldq, p->m, n);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (p->method == TSQR_CMP_MGS) {
        for (int j = 0; j < n; ++j) {
            hipLaunchKernelGGL(k_mgs_pass, dim3(nb), dim3(kGsThreads), 0, s, Q, ldq, p->m, n, j, p->sums,
                               p->partials, R, ldr, p->info);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_gs_reduce, dim3((unsigned)(n - j)), dim3(kGsThreads), 0, s, p->partials,
                               p->gs_blocks, j, p->sums);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        // the last column's norm is sums[n - 1]
        hipLaunchKernelGGL(k_gs_finish, dim3(1024), dim3(256), 0, s, Q, ldq, p->m, n, p->sums + (n - 1), R, ldr,
                           p->info);
        return hipGetLastError();
    }
    // CGS: sums[0] carries ||v_{j-1}||^2 into step j, sums[1 ..] the products of step j
    double* norm2 = p->sums;
    double* dots = p->sums + 1;
    for (int j = 0; j < n; ++j) {
        hipLaunchKernelGGL(k_cgs_dots, dim3(nb), dim3(kGsThreads), 0, s, Q, ldq, p->m, j, norm2, p->partials, R, ldr,
                           p->info);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (j > 0) {
            hipLaunchKernelGGL(k_gs_reduce, dim3((unsigned)j), dim3(kGsThreads), 0, s, p->partials, p->gs_blocks, 0,
                               dots);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_cgs_update, dim3(nb), dim3(kGsThreads), 0, s, Q, ldq, p->m, j, dots, p->partials, R,
                           ldr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_gs_reduce, dim3(1), dim3(kGsThreads), 0, s, p->partials, p->gs_blocks, 0, norm2);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_gs_finish, dim3(1024), dim3(256), 0, s, Q, ldq, p->m, n, norm2, R, ldr, p->info);
    return hipGetLastError();
}

}  // namespace

extern "C" {

tsqr_status tsqr_cmp_plan_create(tsqr_cmp_plan* out, int64_t m, int64_t n, tsqr_cmp_method method, void* hip_stream)
{
    if (!out) return -1;
    *out = nullptr;
    if (m < 1 || m < n) return -2;
    if (n < 1) return -3;
    if (n > tsqr::kMaxN) return 3;
    const int mv = tsqr::abi_int(method);
    if (mv < TSQR_CMP_CHOLQR || mv > TSQR_CMP_MGS) return -4;
    tsqr_cmp_plan_s* p = new (std::nothrow) tsqr_cmp_plan_s();
    if (!p) return 2;
    p->m = m;
    p->n = n;
    p->npb = (int)((n + 15) / 16 * 16);
    p->method = method;
    p->stream = (hipStream_t)hip_stream;
    const int64_t npb2 = (int64_t)p->npb * p->npb;
    const int64_t groups = (m + 63) / 64;
    p->gram_waves = std::min<int64_t>(4096, groups);
    p->gram_rows = (groups + p->gram_waves - 1) / p->gram_waves * 64;
    p->gs_blocks = (m + tsqr::detail::kGsChunk - 1) / tsqr::detail::kGsChunk;
    int64_t off = 0;
    auto take = [&](int64_t doubles) {
        const int64_t o = off;
        off += (doubles + 31) / 32 * 32;
        return o;
    };
    const bool chol = method == TSQR_CMP_CHOLQR || method == TSQR_CMP_CHOLQR2;
    const int64_t oGp = take(chol ? p->gram_waves * npb2 : 0);
    const int64_t oGq = take(chol ? (p->gram_waves + 63) / 64 * npb2 : 0);
    const int64_t oG = take(chol ? npb2 : 0), oRi = take(chol ? npb2 : 0), oR1 = take(chol ? npb2 : 0);
    const int64_t oP = take(chol ? 0 : p->gs_blocks * tsqr::detail::kGsMaxCols);
    const int64_t oS = take(chol ? 0 : tsqr::detail::kGsMaxCols + 1);
    const int64_t oI = take(1);
    hipError_t e = hipMalloc((void**)&p->ws, (size_t)off * sizeof(double));
    if (e != hipSuccess) {
        delete p;
        return cmp_hip(e);
    }
    p->Gp = p->ws + oGp;
    p->Gq = p->ws + oGq;
    p->G = p->ws + oG;
    p->Rinv = p->ws + oRi;
    p->R1 = p->ws + oR1;
    p->partials = p->ws + oP;
    p->sums = p->ws + oS;
    p->info = reinterpret_cast<int*>(p->ws + oI);
    *out = p;
    return 0;
}

tsqr_status tsqr_cmp_factor(tsqr_cmp_plan p, const double* A, int64_t lda, double* Q, int64_t ldq, double* R,
                            int64_t ldr)
{
    if (!p) return -1;
    if (!A) return -2;
    if (lda < p->m) return -3;
    if (!Q) return -4;
    if (ldq < p->m || ((const double*)Q == A && ldq != lda)) return -5;
    if (!R) return -6;
    if (ldr < p->n) return -7;
    hipLaunchKernelGGL(tsqr::detail::k_cmp_init, dim3(1), dim3(256), 0, p->stream, R, ldr, (int)p->n, p->info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cmp_hip(e);
    if (p->method == TSQR_CMP_CHOLQR || p->method == TSQR_CMP_CHOLQR2) e = cholqr(p, A, lda, Q, ldq, R, ldr);
    else e = gram_schmidt(p, A, lda, Q, ldq, R, ldr);
    return cmp_hip(e);
}

tsqr_status tsqr_cmp_breakdown(tsqr_cmp_plan p, int* column)
{
    if (!p) return -1;
    if (!column) return -2;
    hipError_t e = hipStreamSynchronize(p->stream);
    int h = 0;
    if (e == hipSuccess) e = hipMemcpy(&h, p->info, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return cmp_hip(e);
    *column = h;
    return 0;
}

tsqr_status tsqr_cmp_plan_destroy(tsqr_cmp_plan p)
{
    if (!p) return -1;
    hipError_t e = hipStreamSynchronize(p->stream);
    hipError_t e2 = hipFree(p->ws);
    delete p;
    return cmp_hip(e != hipSuccess ? e : e2);
}

}  // extern "C"
