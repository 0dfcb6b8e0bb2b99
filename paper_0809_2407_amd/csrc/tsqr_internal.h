// Internal declarations shared by the C-ABI host code and the HIP kernels of
// libtsqr.  Not installed; the public interface is include/tsqr.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsqr {

constexpr int kMaxLevels = 48;
constexpr int kMaxN = 64;

// Rows per tile for a padded column count np: about 4096 tile elements per
// wavefront (64 doubles per lane, the register budget of the leaf kernel), a
// multiple of 16, at most 512.  This is the fast-memory constraint of
// sequential TSQR (tile rows * n + n(n+1)/2 <= W) with W a wavefront's
// registers; the triangle R itself lives in LDS.
__host__ __device__ constexpr int tile_rows_for(int np)
{
    return (4096 / np / 16 * 16) > 512 ? 512 : (4096 / np / 16 * 16);
}

// Geometry of one TSQR problem: tiles, leaves (flat chains of tiles) and the
// binary tree over the leaves, plus the offsets of every workspace buffer.
struct Layout {
    int64_t m = 0, n = 0;
    int np = 0;          // n rounded up to a multiple of 4 (kernel column granularity)
    int npb = 0;         // n rounded up to a multiple of 16 (matrix-core block)
    int64_t mt = 0;      // tile rows
    int waves = 0;       // wavefronts per workgroup of the leaf kernel
    int64_t f = 0;       // tiles per leaf chain (every leaf but the last)
    int64_t leaf_rows = 0;
    int64_t P = 0;       // leaves
    int64_t ntiles_last = 0;
    int64_t ntiles = 0;  // tiles over all leaves
    int levels = 0;      // binary-tree levels above the leaves
    int64_t count[kMaxLevels + 1] = {0};  // count[0] = P, count[l] = nodes at level l

    // workspace offsets, in doubles
    int64_t nt = 0;                         // packed upper-triangle size np(np+1)/2
    int64_t off_T = 0;                      // per-tile T (packed), ntiles * nt
    int64_t off_R[kMaxLevels + 1] = {0};    // R of every entry of a level, count[l] * np*np
    int64_t off_S[kMaxLevels + 1] = {0};    // seeds of every entry of a level, count[l] * np*np
    int64_t off_Y[kMaxLevels + 1] = {0};    // node reflectors Y1 (np x np), level >= 1
    int64_t off_TN[kMaxLevels + 1] = {0};   // node T (packed), level >= 1
    int64_t off_D = 0;                      // signs, np
    int64_t total = 0;                      // doubles
};

// Fills the geometry.  Returns false for an unsupported shape.
bool make_layout(Layout& L, int64_t m, int64_t n, int64_t leaf_rows_req, int flat_len, int tree, int waves);

// Kernel launchers (tsqr_kernels.hip).  All enqueue on `s` and return the
// launch status.
hipError_t launch_leaf_factor(const Layout& L, const double* A, int64_t lda, double* V, int64_t ldv, double* ws,
                              bool want_q, hipStream_t s);
hipError_t launch_tree(const Layout& L, double* ws, bool want_q, hipStream_t s);
hipError_t launch_root(const Layout& L, double* ws, double* R, int64_t ldr, hipStream_t s);
hipError_t launch_seeds(const Layout& L, double* ws, hipStream_t s);
hipError_t launch_form_q(const Layout& L, const double* A, int64_t lda, double* ws, double* Q, int64_t ldq,
                         hipStream_t s);
hipError_t launch_apply_qt(const Layout& L, const double* A, int64_t lda, int64_t k, double* B, int64_t ldb,
                           double* ws, hipStream_t s);

}  // namespace tsqr
