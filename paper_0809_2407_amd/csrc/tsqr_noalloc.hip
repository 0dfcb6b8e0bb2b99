// tsqr_noalloc.hip -- the allocation-free entry point tsqr_factor_r_noalloc:
// the FP64 R-only factorisation of tsqr_factor (leaf chains, binary tree,
// signs) with its workspace in a fixed file-scope device array instead of a
// plan's hipMalloc'd one, for callers that cannot allocate (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "tsqr.h"
#include "tsqr_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int64_t kMaxChain = 256;  // the autotuner's accuracy guard on chain length
constexpr int kMaxDevices = 64;

// Workspace of tsqr_factor_r_noalloc: the R factors of every tree level, the
// signs and the root seed.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code this name is a host-side stand-in, not
// a device address: host code uses only the per-device address that
// hipGetSymbolAddress returns (scratch_of).
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {nullptr};

// The device address of `scratch` on device dev (the current device), looked
// up once per device.
hipError_t scratch_of(int dev, double** out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

tsqr_status hip_status(hipError_t e) { return e == hipSuccess ? 0 : (e == hipErrorOutOfMemory ? 2 : 1); }

}  // namespace

extern "C" tsqr_status tsqr_factor_r_noalloc(int64_t m, int64_t n, const double* A, int64_t lda, double* R,
                                             int64_t ldr, void* hip_stream, tsqr_info* info)
{
    if (m < 0 || m < n) return -1;
    if (n < 0) return -2;
    if (n > tsqr::kMaxN) return 3;
    if (!A && n > 0) return -3;  // an empty problem references no matrix
    if (lda < m) return -4;
    if (!R && n > 0) return -5;
    if (ldr < n) return -6;
    if (n == 0) {  // the empty problem: nothing to compute
        if (info) {
            *info = tsqr_info{};
            info->m = m;
            info->tree = TSQR_TREE_FLAT;
            info->precision = TSQR_FP64;
        }
        return 0;
    }
    // geometry: as many short chains as the R-only plans use (16384 leaves),
    // fewer when their R factors would not fit the scratch array; chains are
    // capped at kMaxChain tiles, beyond which the size is rejected (status 6)
    const int np = tsqr::padded_width(n);
    const int64_t mt = tsqr::tile_rows_for(np);
    const int64_t tiles = (m + mt - 1) / mt;
    int64_t f = std::max<int64_t>(1, tiles / 16384);
    tsqr::Layout L;
    for (;;) {
        if (f > kMaxChain) return 6;
        if (!tsqr::make_layout_r_compact(L, m, n, f * mt)) return 3;
        if ((size_t)L.total * sizeof(double) <= kScratchBytes) break;
        f *= 2;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e);
    if (dev < 0 || dev >= kMaxDevices) return 3;
    double* ws = nullptr;
    e = scratch_of(dev, &ws);
    if (e != hipSuccess) return hip_status(e);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // every entry of the workspace is written before it is read: nothing to clear
    e = tsqr::launch_leaf_factor(L, A, lda, nullptr, lda, ws, false, s);
    if (e == hipSuccess && L.levels > 0) e = tsqr::launch_tree(L, ws, false, s);
    if (e == hipSuccess) e = tsqr::launch_root(L, ws, R, ldr, s);
    if (e != hipSuccess) return hip_status(e);
    if (info) {
        *info = tsqr_info{};
        info->m = L.m;
        info->n = L.n;
        info->n_padded = L.np;
        info->tile_rows = L.mt;
        info->leaf_rows = L.leaf_rows;
        info->num_leaves = L.P;
        info->num_tiles = L.ntiles;
        info->tree_levels = L.levels;
        info->tree = L.P == 1 ? TSQR_TREE_FLAT : (L.f == 1 ? TSQR_TREE_BINARY : TSQR_TREE_HYBRID);
        info->waves = L.waves;
        info->precision = TSQR_FP64;
        info->workspace_bytes = L.total * (int64_t)sizeof(double);
    }
    return 0;
}
