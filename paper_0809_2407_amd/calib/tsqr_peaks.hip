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
