// Internal declarations shared by the C-ABI host code and the HIP kernels of
// libtsqr.  Not installed; the public interface is include/tsqr.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>

namespace tsqr {

// The int a caller passed for an enumeration-typed argument or field of the C
// ABI.  A C caller may pass any int there, and reading a value outside an
// enumeration's range as that enumeration is undefined in C++, so the entry
// points read the bytes as an int before they validate them.
template <typename En>
inline int abi_int(const En& e)
{
    static_assert(sizeof(En) == sizeof(int), "C enumerations have the size of int");
    int v;
    std::memcpy(&v, &e, sizeof v);
    return v;
}

constexpr int kMaxLevels = 48;
constexpr int kMaxN = 64;
// Mixed precision: the second pass corrects Q and R when ||Q1^T Q1 - I||_F
// exceeds this bound.
constexpr double kReorthBound = 1e-13;
// Mixed precision: longest automatic leaf chain (tiles) of FP32 tiles.
constexpr int64_t kMaxChainF32 = 64;

// Rows per tile for a padded column count np: about 4096 tile elements per
// wavefront (64 doubles per lane, the register budget of the leaf kernel), a
// multiple of 16, at most 512.  This is the fast-memory constraint of
// sequential TSQR (tile rows * n + n(n+1)/2 <= W) with W a wavefront's
// registers; the triangle R itself lives in LDS.
__host__ __device__ constexpr int tile_rows_for(int np)
{
    // at np = 8 a 512-row tile leaves the reflector-keeping kernel short of registers
    return (4096 / np / 16 * 16) > (np == 8 ? 384 : 512) ? (np == 8 ? 384 : 512) : (4096 / np / 16 * 16);
}

// Padded column count of the kernels for n columns: n rounded up to a multiple
// of 4, except that widths 49-52 run on the 56-column kernels and 57-60 on the
// 64-column ones.  At 52 and 60 columns the factor layout gives each lane an
// odd number of columns (13, 15), and the compiler leaves the column loops of
// those instantiations rolled, which puts the whole tile in scratch memory
// (432-528 bytes per lane with no spill reported); four more zero columns
// (tau = 0 reflectors) cost far less.
__host__ __device__ constexpr int padded_width(int64_t n)
{
    return (n > 56 && n <= 60) ? 64 : ((n > 48 && n <= 52) ? 56 : (int)((n + 3) / 4 * 4));
}
// Most zero columns padded_width adds at a padded count np.
__host__ __device__ constexpr int max_padding(int np) { return (np == 64 || np == 56) ? 7 : 3; }

// Rows per tile of the mixed-precision leaf kernel, whose tile is held in FP32:
// twice the FP64 tile in the same registers, at most 1024.
#ifndef TSQR_F32_TILE_SCALE
#define TSQR_F32_TILE_SCALE 2
#endif
__host__ __device__ constexpr int tile_rows_f32(int np) { return TSQR_F32_TILE_SCALE * tile_rows_for(np); }

// Geometry of one TSQR problem: tiles, leaves (flat chains of tiles) and the
// binary tree over the leaves, plus the offsets of every workspace buffer.
struct Layout {
    int64_t m = 0, n = 0;
    int np = 0;          // padded column count of the kernels (padded_width)
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
    int64_t off_TN[kMaxLevels + 1] = {0};   // node T (packed), level >= 1; one contiguous run over the levels
    int64_t tree_nodes = 0;                 // nodes of levels >= 1 (T slots from off_TN[1])
    int64_t off_D = 0;                      // signs, np

    // mixed precision (FP32 first pass, FP64 second pass)
    bool mixed = false;
    // FP64 with Q: each leaf tile's T is formed by the leaf kernel itself (the
    // recursive variant, widths 16 and 32) instead of a T kernel after it
    bool rec = false;
    int64_t ld32 = 0;                       // rows of V32 and Q1: whole tiles, rounded up to 64
    int64_t off_T32 = 0;                    // per-tile T in FP32 (packed), ntiles * nt floats
    int64_t off_V32 = 0, off_Q1 = 0;        // FP32, ld32 x npb, zero past m and past n
    int64_t gram_waves = 0, gram_rows = 0;  // partial Gram matrices: wavefronts, rows each
    int64_t off_Gp = 0, off_Gq = 0, off_G = 0;  // partial, group and summed Gram matrices, npb x npb
    int64_t off_R1 = 0;                     // first-pass R (np x np)
    int64_t off_R2inv = 0;                  // R2^{-1} (npb x npb)
    int64_t off_info = 0;                   // ||Q1^T Q1 - I||_F, correction flag
    int64_t total = 0;                      // doubles
};

// ---- batched problems -------------------------------------------------------
constexpr int kBatchLevels = 32;

// Static description of one problem of a batch (uploaded once per plan): its
// geometry and the offsets of its workspace inside the plan's buffer.
struct BatchProblem {
    int64_t m = 0;
    int n = 0, levels = 0;
    int64_t P = 0, leaf_rows = 0, f = 0;
    int64_t ws_off = 0;  // doubles
    int64_t off_T = 0, off_D = 0;
    int64_t off_R[kBatchLevels] = {0}, off_S[kBatchLevels] = {0};
    int64_t off_Y[kBatchLevels] = {0}, off_TN[kBatchLevels] = {0};
    int64_t count[kBatchLevels] = {0};
    // mixed precision (offsets in doubles inside the problem's workspace)
    int64_t ld32 = 0, off_V32 = 0, off_T32 = 0, off_Q1 = 0;
    int64_t off_Gp = 0, off_Gq = 0, off_G = 0, off_R1 = 0, off_R2inv = 0, off_info = 0;
    int64_t gram_waves = 0, gram_rows = 0;
};

// Per-call matrices of one problem: A (factored in place) and the output
// (R for the factorisation, Q for the explicit Q).
struct BatchArgs {
    double* A = nullptr;
    int64_t lda = 0;
    double* X = nullptr;
    int64_t ldx = 0;
};

// Work items of the batched kernels: problem index in the high 32 bits,
// leaf or node index in the low 32 bits.
__host__ __device__ inline int64_t batch_item(int64_t p, int64_t i) { return (p << 32) | i; }

// Device-side work lists of one width class (all problems with the same np).
struct BatchClass {
    int np = 0;
    int64_t nprob = 0;
    int max_levels = 0;
    const int64_t* leaf_items = nullptr;  // (problem, leaf)
    int64_t n_leaf = 0;
    const int64_t* root_items = nullptr;  // (problem, 0)
    const int64_t* level_items[kBatchLevels] = {nullptr};  // (problem, node) of level l >= 1
    int64_t n_level[kBatchLevels] = {0};
    // mixed precision: partial Gram matrices (problem, w), their groups of 64
    // (problem, g), and the 1024-row chunks of Q = Q1 R2^{-1} (problem, c)
    const int64_t* gram_items = nullptr;
    int64_t n_gram = 0;
    const int64_t* gsum_items = nullptr;
    int64_t n_gsum = 0;
    const int64_t* rq_items = nullptr;
    int64_t n_rq = 0;
};

// Fills the geometry.  Returns false for an unsupported shape.  in_batch: the
// problem is one of many run together (a batched plan), whose parallelism
// comes from the other problems, so the automatic leaf length keeps the
// per-leaf factors under a quarter of the data at every size.
bool make_layout(Layout& L, int64_t m, int64_t n, int64_t leaf_rows_req, int flat_len, int tree, int waves,
                 bool mixed, bool want_q, bool in_batch = false);
// The geometry of an FP64 R-only factorisation with leaves of leaf_rows_req
// rows and a workspace holding only the R factors of every tree level, the
// signs and the root seed (L.total doubles).
bool make_layout_r_compact(Layout& L, int64_t m, int64_t n, int64_t leaf_rows_req);

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
// mixed precision: FP32 leaf chains, FP32 Q1, FP64 second pass (Gram,
// Cholesky, check, R = R2 R1 to the caller's R) and the corrected Q
hipError_t launch_mixed_leaf(const Layout& L, const double* A, int64_t lda, double* ws, bool want_q, hipStream_t s);
// T of every leaf tile from the tau and Gram entries the leaf kernel left in
// the tile's T slot (plans with Q, both precisions).
hipError_t launch_build_T(const Layout& L, double* ws, hipStream_t s);
// LDS bytes per wavefront of the single-problem leaf kernel for a padded width.
int leaf_lds_bytes(int np, bool mixed, bool want_q);
hipError_t launch_form_q1(const Layout& L, double* ws, hipStream_t s);
hipError_t launch_reorth(const Layout& L, double* ws, double* R, int64_t ldr, hipStream_t s);
hipError_t launch_reorth_q(const Layout& L, double* ws, double* Q, int64_t ldq, hipStream_t s);
// Q^T B on a mixed plan: the top n rows of B become R2^{-T} Q1^T B
hipError_t launch_qtb_mixed(const Layout& L, double* ws, int64_t k, double* B, int64_t ldb, hipStream_t s);

// batched FP64: every problem of a width class in one launch per phase
hipError_t launch_batch_factor(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                               bool want_q, int waves, hipStream_t s);
// alias: some problem's Q is its A (the graph then takes one wavefront per leaf)
hipError_t launch_batch_form_q(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                               int waves, bool alias, hipStream_t s);
hipError_t launch_batch_factor_mixed(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args,
                                     double* ws, bool want_q, int waves, hipStream_t s);
hipError_t launch_batch_form_q_mixed(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args,
                                     double* ws, hipStream_t s);

// Per-width launchers behind the dispatch (one instantiation per padded width).
template <int NP>
hipError_t leaf_factor_np(const Layout& L, const double* A, int64_t lda, double* V, int64_t ldv, double* ws,
                          bool want_q, hipStream_t s);
template <int NP>
hipError_t tree_np(const Layout& L, double* ws, bool want_q, hipStream_t s);
template <int NP>
hipError_t root_np(const Layout& L, double* ws, double* R, int64_t ldr, hipStream_t s);
template <int NP>
hipError_t seeds_np(const Layout& L, double* ws, hipStream_t s);
template <int NP>
hipError_t form_q_np(const Layout& L, const double* A, int64_t lda, double* ws, double* Q, int64_t ldq,
                     hipStream_t s);
template <int NP>
hipError_t apply_qt_np(const Layout& L, const double* A, int64_t lda, int64_t k, double* B, int64_t ldb,
                       double* ws, hipStream_t s);
template <int NP>
hipError_t mixed_leaf_np(const Layout& L, const double* A, int64_t lda, double* ws, bool want_q, hipStream_t s);
template <int NP>
hipError_t build_T_np(const Layout& L, double* ws, hipStream_t s);
template <int NP>
int leaf_lds_bytes_np(bool mixed, bool want_q);
template <int NP>
hipError_t form_q1_np(const Layout& L, double* ws, hipStream_t s);
template <int NP>
hipError_t reorth_np(const Layout& L, double* ws, double* R, int64_t ldr, hipStream_t s);
template <int NP>
hipError_t reorth_q_np(const Layout& L, double* ws, double* Q, int64_t ldq, hipStream_t s);
template <int NP>
hipError_t qtb_mixed_np(const Layout& L, double* ws, int64_t k, double* B, int64_t ldb, hipStream_t s);
template <int NP>
hipError_t batch_factor_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                           bool want_q, int waves, hipStream_t s);
template <int NP>
hipError_t batch_form_q_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                           int waves, bool alias, hipStream_t s);
template <int NP>
hipError_t batch_factor_mixed_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                                 bool want_q, int waves, hipStream_t s);
template <int NP>
hipError_t batch_form_q_mixed_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                                 hipStream_t s);

}  // namespace tsqr
