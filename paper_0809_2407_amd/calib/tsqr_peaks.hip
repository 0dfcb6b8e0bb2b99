// Machine ceilings measured on the part: a streaming copy and a streaming read
// with 16-byte accesses (HBM), and loops of FP64 FMA (vector ALU) and FP64
// MFMA 16x16x4 (matrix cores).  Not part of the factorisation.
#include <hip/hip_runtime.h>

#include "tsqr_peaks.h"

namespace {

constexpr int kBlock = 256;
constexpr int kCopyU = 1;  // 16-byte elements per lane and chunk: copy
constexpr int kReadU = 4;  // and read
constexpr int kLoopBlocksPerCU = 8;
constexpr int kMaxGrid = 1 << 20;

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));

// Both streams walk chunks of 256 * U elements: workgroup g takes chunks
// g, g + G, g + 2G, ... (G = the grid), lane l of a chunk touches elements
// l, l + 256, ..., l + 256 (U - 1) of it.  The default grid covers the buffer
// in one pass.  Of the forms measured (grid-stride loops of fixed grids, one
// pass with 1 to 8 elements per lane, non-temporal loads and stores) these were
// the fastest: one element per lane with plain accesses for the copy, four with
// non-temporal loads for the read.
__global__ __launch_bounds__(kBlock) void k_copy16(const d2* __restrict__ src, d2* __restrict__ dst, size_t n)
{
    const size_t step = (size_t)gridDim.x * kBlock * kCopyU;
    for (size_t base = (size_t)blockIdx.x * kBlock * kCopyU; base < n; base += step) {
        d2 v[kCopyU];
#pragma unroll
        for (int u = 0; u < kCopyU; ++u) {
            const size_t i = base + (size_t)u * kBlock + threadIdx.x;
            if (i < n) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < kCopyU; ++u) {
            const size_t i = base + (size_t)u * kBlock + threadIdx.x;
            if (i < n) dst[i] = v[u];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_read16(const d2* __restrict__ src, size_t n, double* __restrict__ partial)
{
    __shared__ double red[kBlock];
    const size_t step = (size_t)gridDim.x * kBlock * kReadU;
    double acc = 0.0;
    for (size_t base = (size_t)blockIdx.x * kBlock * kReadU; base < n; base += step) {
#pragma unroll
        for (int u = 0; u < kReadU; ++u) {
            const size_t i = base + (size_t)u * kBlock + threadIdx.x;
            if (i < n) {
                const d2 v = __builtin_nontemporal_load(&src[i]);
                acc += v.x + v.y;
            }
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// A copy in the access pattern of the TSQR Q kernel: wavefront w owns the rows
// of leaf w (leaf_rows each, the last leaf takes the rest), walks its tiles of
// tile_rows rows from the last to the first and moves each 16 rows at a time;
// lane 16 g + r moves row r of those 16 in columns 4 k + g (k < NK).  All of a
// block's loads are issued before its stores, as there.
template <int NK>
__global__ __launch_bounds__(kBlock) void k_copy_leaf(const double* __restrict__ src, int64_t lds,
                                                      double* __restrict__ dst, int64_t ldd, int64_t m, int n,
                                                      int64_t leaf_rows, int tile_rows, int64_t leaves)
{
    const int64_t leaf = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (leaf >= leaves) return;
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int64_t row0 = leaf * leaf_rows;
    const int64_t rend = leaf == leaves - 1 ? m : row0 + leaf_rows;
    const int64_t ntl = (rend - row0 + tile_rows - 1) / tile_rows;
    for (int64_t t = ntl - 1; t >= 0; --t) {
        const int64_t t0 = row0 + t * tile_rows;
        const int64_t tend = t0 + tile_rows < rend ? t0 + tile_rows : rend;
        for (int64_t b = t0; b < tend; b += 16) {
            const int64_t row = b + r;
            double y[NK];
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const int c = 4 * k + g;
                y[k] = (row < tend && c < n) ? src[row + (int64_t)c * lds] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const int c = 4 * k + g;
                if (row < tend && c < n) dst[row + (int64_t)c * ldd] = y[k];
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_fma_loop(double* __restrict__ out, int iters, double c, double d) {
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = (double)j;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = fma(x[j], c, d);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j];
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_mfma_loop(double* __restrict__ out, int iters, double a, double b) {
    d4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
        }
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) s += (acc[j][0] + acc[j][1]) + (acc[j][2] + acc[j][3]);
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

int loop_grid()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    return cus * kLoopBlocksPerCU;
}

int stream_grid(int64_t bytes, int per_lane)
{
    const int64_t chunk = (int64_t)16 * kBlock * per_lane;
    const int64_t g = (bytes + chunk - 1) / chunk;
    return (int)(g < 1 ? 1 : (g > kMaxGrid ? kMaxGrid : g));
}

int pick_grid(int grid, int kind, int64_t bytes)
{
    if (grid > 0) return grid;
    if (kind == 0) return stream_grid(bytes, kCopyU);
    if (kind == 1) return stream_grid(bytes, kReadU);
    return loop_grid();
}

int launched() { return hipGetLastError() == hipSuccess ? 0 : 1; }

}  // namespace

extern "C" {

int tsqr_peak_grid(int kind, int64_t bytes)
{
    if (kind < 0 || kind > 2 || bytes < 0) return -1;
    return pick_grid(0, kind, bytes);
}

int tsqr_peak_copy(const void* src, void* dst, int64_t bytes, int grid, void* stream) {
    if (!src || ((uintptr_t)src & 15)) return -1;
    if (!dst || ((uintptr_t)dst & 15)) return -2;
    if (bytes <= 0 || (bytes & 15)) return -3;
    if (grid > kMaxGrid) return -4;
    const char* s = (const char*)src;
    const char* d = (const char*)dst;
    if (s < d + bytes && d < s + bytes) return -2;
    const int g = pick_grid(grid, 0, bytes);
    hipLaunchKernelGGL(k_copy16, dim3(g), dim3(kBlock), 0, (hipStream_t)stream, (const d2*)src, (d2*)dst,
                       (size_t)(bytes / 16));
    return launched();
}

int tsqr_peak_read(const void* src, int64_t bytes, double* partial, int grid, void* stream) {
    if (!src || ((uintptr_t)src & 15)) return -1;
    if (bytes <= 0 || (bytes & 15)) return -2;
    if (!partial) return -3;
    if (grid > kMaxGrid) return -4;
    const int g = pick_grid(grid, 1, bytes);
    hipLaunchKernelGGL(k_read16, dim3(g), dim3(kBlock), 0, (hipStream_t)stream, (const d2*)src,
                       (size_t)(bytes / 16), partial);
    return launched();
}

int tsqr_peak_copy_leaf(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t m, int n,
                        int64_t leaf_rows, int tile_rows, void* stream)
{
    if (!src) return -1;
    if (lds < m) return -2;
    if (!dst) return -3;
    if (ldd < m) return -4;
    if (m < 1) return -5;
    if (n < 1 || n > 64) return -6;
    if (tile_rows < 16 || tile_rows % 16 != 0) return -8;
    if (leaf_rows < tile_rows || leaf_rows % tile_rows != 0) return -7;
    const char* s0 = (const char*)src;
    const char* s1 = (const char*)(src + (n - 1) * lds + m);
    const char* d0 = (const char*)dst;
    const char* d1 = (const char*)(dst + (n - 1) * ldd + m);
    if (s0 < d1 && d0 < s1) return -3;
    const int64_t leaves = m / leaf_rows > 0 ? m / leaf_rows : 1;
    const int64_t grid = (leaves + kBlock / 64 - 1) / (kBlock / 64);
    if (grid > ((int64_t)1 << 31) - 1) return -7;
    const hipStream_t st = (hipStream_t)stream;
    const dim3 g((unsigned)grid), b(kBlock);
    if (n <= 8) hipLaunchKernelGGL(k_copy_leaf<2>, g, b, 0, st, src, lds, dst, ldd, m, n, leaf_rows, tile_rows, leaves);
    else if (n <= 16) hipLaunchKernelGGL(k_copy_leaf<4>, g, b, 0, st, src, lds, dst, ldd, m, n, leaf_rows, tile_rows, leaves);
    else if (n <= 32) hipLaunchKernelGGL(k_copy_leaf<8>, g, b, 0, st, src, lds, dst, ldd, m, n, leaf_rows, tile_rows, leaves);
    else hipLaunchKernelGGL(k_copy_leaf<16>, g, b, 0, st, src, lds, dst, ldd, m, n, leaf_rows, tile_rows, leaves);
    return launched();
}

int tsqr_peak_fma(double* out, int grid, int iters, double c, double d, void* stream) {
    if (!out) return -1;
    if (grid > kMaxGrid) return -2;
    if (iters < 0) return -3;
    const int g = pick_grid(grid, 2, 0);
    if (g <= 0) return 1;
    hipLaunchKernelGGL(k_fma_loop, dim3(g), dim3(kBlock), 0, (hipStream_t)stream, out, iters, c, d);
    return launched();
}

int tsqr_peak_mfma(double* out, int grid, int iters, double a, double b, void* stream) {
    if (!out) return -1;
    if (grid > kMaxGrid) return -2;
    if (iters < 0) return -3;
    const int g = pick_grid(grid, 2, 0);
    if (g <= 0) return 1;
    hipLaunchKernelGGL(k_mfma_loop, dim3(g), dim3(kBlock), 0, (hipStream_t)stream, out, iters, a, b);
    return launched();
}

}  // extern "C"
