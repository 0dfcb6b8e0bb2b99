// tsqr_kernels.h -- gfx950 (CDNA4) kernels of TSQR (templates; instantiated
// per column count by the tsqr_np_*.hip units).
//
// Execution model.  One wavefront owns one leaf: a block row of the matrix
// reduced by a flat chain over its tiles, qr(A_0) then qr([R; A_k]) (the
// sequential TSQR of Alg. 2 with the wavefront's registers as fast memory).
// The leaf R factors are then combined on a binary tree, one launch per level,
// one wavefront per node (the parallel TSQR of Alg. 1, with the stacked pair
// [R_a; R_b] factored by the triangle-aware QR of Sec. 3.1).  The explicit Q is
// the tree replayed top-down (applying Q is a broadcast, Sec. 4.1).  Each
// tile's compact-WY T is formed by its own kernel (k_build_T) from the tau and
// Gram entries the leaf kernel leaves in the tile's T slot.
//
// Register layout of a tile ("L layout").  A tile has 16*RL rows and NP
// columns (NP = padded_width(n); padded columns are zero and
// stay zero).  Lane l = 16*cg + rg holds rows 16*i + rg (i < RL) and columns
// 4*k + cg (k < NP/4) in a[i][k].  Consequences:
//   - a sum over the rows of a column is a sum over the 16 lanes of one DPP row
//     (four DPP steps, every lane ends with the same bits);
//   - the f64 16x16x4 matrix-core op contracts over the lane-group index, so a
//     product that contracts over COLUMNS (Y Z, T S, Y1 Z) maps this layout onto
//     itself: the seed products and the Q expansion run on the matrix cores
//     with no data movement.
//
// Householder conventions: H_j = I - tau_j v_j v_j^T, v_j(j) = 1,
// beta = -sgn(alpha) ||x||, tau = (beta - alpha)/beta, tau = 0 when the part of
// the column below the pivot is zero.  Every tile stores T, the upper-triangular
// factor of H_0 ... H_{n-1} = I - V T V^T (the YT representation of Sec. 3.2).
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

#include "tsqr_internal.h"

namespace tsqr {
namespace detail {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma16x16x4(double a, double b, dbl4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over groups of LR consecutive lanes (LR = 8 or 16, inside one DPP row).
// Each step adds a partner whose own step adds the same two operands, so all
// lanes of a group end with identical bits.
template <int LR>
__device__ __forceinline__ double group_sum(double v)
{
    v += dpp_move<0xB1>(v);       // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);       // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);      // row_half_mirror: lane i <-> 7-i within 8
    if (LR == 16) v += dpp_move<0x140>(v);  // row_mirror: lane i <-> 15-i within 16
    return v;
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int LR>
__device__ __forceinline__ float group_sum(float v)
{
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x141>(v);
    if (LR == 16) v += dpp_move<0x140>(v);
    return v;
}

__device__ __forceinline__ float readlane_d(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// An opaque copy of a value: per-lane offsets derived from it inside a loop are
// recomputed there (a few integer ops) instead of being hoisted out of the
// loop and kept live, or spilled, across it.
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// The wavefront's index in its block, as a wave-uniform (scalar) value, so
// that addresses derived from it stay in scalar registers.
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Loads and stores at a wave-uniform base plus a 32-bit per-lane byte offset,
// the form that addresses through a scalar base register.
template <typename E, typename O>
__device__ __forceinline__ E ld_at(const E* base, O byte_off)
{
    return *reinterpret_cast<const E*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename E, typename O>
__device__ __forceinline__ void st_at(E* base, O byte_off, E v)
{
    *reinterpret_cast<E*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
// The same as a non-temporal store (output written once and not read again by
// the path: the explicit Q).
template <typename E, typename O>
__device__ __forceinline__ void st_nt(E* base, O byte_off, E v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<E*>(reinterpret_cast<char*>(base) + byte_off));
}

// True when the byte offset of element (15, 3) of a 16 x 4 block with leading
// dimension ld fits in 32 bits, so 32-bit per-lane offsets can be used.
inline bool lane_offsets_fit_32(int64_t ld) { return (uint64_t)(15 + 3 * ld) * 8u < (1ull << 32); }

// 1/p to about one ulp: hardware reciprocal and two Newton steps.
__device__ __forceinline__ double recip(double p)
{
    double r = __builtin_amdgcn_rcp(p);
    double e = fma(-p, r, 1.0);
    r = fma(r, e, r);
    e = fma(-p, r, 1.0);
    return fma(r, e, r);
}

// sqrt for positive normal arguments: hardware reciprocal square root and one
// Goldschmidt/Newton refinement of both the root and its half-reciprocal
// (no rescaling of subnormal or huge inputs).
__device__ __forceinline__ double sqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}

// The scalars of the Householder reflector of a column with pivot entry alpha
// and squared norm s of the part below the pivot (Sec. 4.2's local QR; LAPACK's
// convention): beta = -sgn(alpha) ||x||, tau = (beta - alpha)/beta = -d/beta and
// the scale 1/d of the part below the pivot, with d = alpha - beta (alpha and
// beta have opposite signs, so d has no cancellation); tau = 0 (H = I) when the
// part below the pivot is zero.  Branch-free: the selects discard the inf/NaN of
// s == 0.  alpha^2 + s must lie in the normal range (the caller rescales).
__device__ __forceinline__ void reflector_scalars(double alpha, double s, double& beta, double& scale, double& tau)
{
    const bool nz = s != 0.0;
    const double nrm = sqrt_pos(fma(alpha, alpha, s));
    const double bn = alpha < 0.0 ? nrm : -nrm;
    const double dd = alpha - bn;
    const double rr = recip(dd * bn);
    beta = nz ? bn : alpha;
    scale = nz ? bn * rr : 0.0;
    tau = nz ? -(dd * dd) * rr : 0.0;
}

// Maximum over groups of LR consecutive lanes (the pairing of group_sum).
template <int LR>
__device__ __forceinline__ double group_max(double v)
{
    v = fmax(v, dpp_move<0xB1>(v));
    v = fmax(v, dpp_move<0x4E>(v));
    v = fmax(v, dpp_move<0x141>(v));
    if (LR == 16) v = fmax(v, dpp_move<0x140>(v));
    return v;
}

__host__ __device__ constexpr int round16(int np) { return (np + 15) / 16 * 16; }
// The running triangle R lives in LDS packed by rows: R(r, c), r <= c, at
// r np - r(r+1)/2 + c (np(np+1)/2 doubles, rounded up to an even count).  The
// row index is the wave-uniform one in the factorisation, so the per-lane part
// of an address is the column alone.
template <int NP>
__host__ __device__ constexpr int rpk(int r, int c) { return r * NP - r * (r + 1) / 2 + c; }
__host__ __device__ constexpr int r_area(int np) { return (np * (np + 1) / 2 + 1) / 2 * 2; }
// Stride (doubles) between the per-lane segments of the reflector broadcast
// buffer: s = 2 mod 4, so that 8 or 16 segments read 16 bytes at a time hit
// disjoint banks, and 16-byte aligned.
__host__ __device__ constexpr int vb_stride(int rl) { return (rl % 4 == 2) ? rl : (rl % 4 == 3) ? rl + 3 : (rl % 4 == 1) ? rl + 1 : rl + 2; }
// The same byte stride rule (16 mod 32 bytes) for a broadcast buffer of floats.
__host__ __device__ constexpr int vb_stride_f(int rl) { return rl % 8 == 4 ? rl : rl + ((12 - rl % 8) % 8); }
template <typename E>
__host__ __device__ constexpr int vb_stride_e(int rl) { return sizeof(E) == 8 ? vb_stride(rl) : vb_stride_f(rl); }
__host__ __device__ constexpr int packed_size(int np) { return np * (np + 1) / 2; }
// Column groups of the factor layout: 8 when NP is a multiple of 8, else 4.
__host__ __device__ constexpr int col_groups(int np) { return np % 8 == 0 && np > 16 ? 8 : 4; }
// The Gram chunk buffer of the tree kernels with Q: 16 rows of np + 1 doubles
// (gram_out); R-only kernels have none.
__host__ __device__ constexpr int gram_area(int np) { return (16 * (np + 1) + 1) / 2 * 2; }
// per-wave LDS of the tree kernels: R, Gram chunk buffer (with Q), reflector broadcast, tau
template <typename E = double>
__host__ __device__ constexpr int factor_lds_doubles(int np, int tile_rows, bool want_q)
{
    return r_area(np) + (want_q ? gram_area(np) : 0) +
           ((64 / col_groups(np)) * vb_stride_e<E>(tile_rows / (64 / col_groups(np))) * (int)sizeof(E) + 7) / 8 +
           np;
}
// Widths whose FP64 leaf factors chained tiles in 16-column panels with the
// trailing update on the matrix cores (factor_tile_blocked), one bit per width
// np = 4 (bit + 1); they use the four-group layout.
#ifndef TSQR_BLOCKED_MASK
#define TSQR_BLOCKED_MASK 0x80ull  // np = 32
#endif
template <typename E = double>
__host__ __device__ constexpr bool leaf_blocked(int np)
{
    return sizeof(E) == 8 && np % 16 == 0 && ((TSQR_BLOCKED_MASK >> (np / 4 - 1)) & 1);
}
template <typename E = double>
__host__ __device__ constexpr int leaf_col_groups(int np) { return leaf_blocked<E>(np) ? 4 : col_groups(np); }
// The single-problem leaf kernel leaves T to k_build_T: with Q it keeps only a
// chunk buffer of the Gram (CH rows of np + 1 doubles).  CH = 16 where the
// per-wave LDS then stays within 20 KiB (two wavefronts per SIMD), else 4.
// Blocked widths also hold the chunk buffer without Q (the panel update uses
// it).
template <typename E = double>
__host__ __device__ constexpr int leaf_lds_doubles_ch(int np, int tile_rows, bool want_q, int ch)
{
    return r_area(np) + (want_q || leaf_blocked<E>(np) ? (ch * (np + 1) + 1) / 2 * 2 : 0) +
           ((64 / leaf_col_groups<E>(np)) * vb_stride_e<E>(tile_rows / (64 / leaf_col_groups<E>(np))) *
                (int)sizeof(E) + 7) / 8 +
           np;
}
constexpr int kLeafLdsBudget = 20480 / 8;  // doubles per wavefront for two wavefronts per SIMD
template <typename E = double>
__host__ __device__ constexpr int leaf_gram_chunk(int np, int tile_rows)
{
    return leaf_blocked<E>(np) || leaf_lds_doubles_ch<E>(np, tile_rows, true, 16) <= kLeafLdsBudget ? 16 : 4;
}
template <typename E = double>
__host__ __device__ constexpr int leaf_lds_doubles(int np, int tile_rows, bool want_q)
{
    return leaf_lds_doubles_ch<E>(np, tile_rows, want_q, leaf_gram_chunk<E>(np, tile_rows));
}
template <typename E>
__host__ __device__ constexpr int tile_rows_e(int np) { return sizeof(E) == 8 ? tile_rows_for(np) : tile_rows_f32(np); }

// --------------------------------------------------------------------------
// Householder QR of one tile held in registers.
//
// Layout: LC column groups of LR = 64/LC lanes; lane l = LR*cg + rg holds rows
// LR*i + rg (i < RL) and columns LC*k + cg (k < NP/LC) in a[i][k].  A sum over
// the rows of a column is a sum over the LR lanes of one group (DPP steps).
//
// FIRST:  the tile is A_0 of a chain; plain Householder on it (reflector j has
//         v(j) = 1, zeros above, y below).  Its top NP rows end up holding R.
// !FIRST: the tile is the rectangle under the running triangle R (kept in LDS
//         at Rs, column-major NP x NP): the QR of [R; A_k] with reflectors
//         [e_j; y_j] (Alg. 2; triangle on a rectangle, Sec. 3.1).  R is updated
//         in place, the tile is overwritten by the y_j.
// tau_j is recorded in taus for the compact-WY factor T (see gram_out and
// k_build_T).
//
// A reflector column is left unscaled in the registers while the tile is
// factored (y = x * sc, sc[k] holds the scale of the lane's column k, 1 for a
// column that is not a reflector yet); scale_tile applies it at the end.
// The magnitudes are assumed to keep (alpha - beta) * beta within the normal
// FP64 range (no scaling of the column norm).
// --------------------------------------------------------------------------
// KLO, KHI: factor only the columns held in slots [KLO, KHI) and update only
// those (a panel of the blocked factorization below); the default is the tile.
// TRI: the tile is upper triangular (the R_b of a tree node, Sec. 3.1): rows
// past a column are zero and stay zero, so reflector j = [e_j; y_j] has y_j
// nonzero in rows 0 .. j only, and the column steps of block kb skip the
// register slots of rows past its last column (eq. fact_2rs: the structured
// QR of two stacked triangles).
template <int NP, int RL, int LC, bool FIRST, typename E = double, int KLO = 0, int KHI = NP / LC, bool TRI = false>
__device__ __forceinline__ void factor_tile(E (&a)[RL][NP / LC], E (&sc)[NP / LC], double* Rs, E* vb,
                                            double* taus, int lane)
{
    constexpr int KC = NP / LC, LR = 64 / LC;
    const int cg = lane / LR, rg = lane % LR;
    E* my_vb = vb + rg * vb_stride_e<E>(RL);  // this lane's rows of the broadcast reflector
#pragma unroll
    for (int k = 0; k < KC; ++k) sc[k] = E(1);
#pragma unroll
    for (int kb = KLO; kb < KHI; ++kb) {
        const int ij = (LC * kb) / LR;   // register slot of the pivot rows of this block
        const int rg0 = (LC * kb) % LR;  // lane (within a group) of the block's first pivot row
        // TRI: the last register slot holding a row at or above this block's last column
        const int imax = TRI ? (LC * kb + LC - 1) / LR : RL - 1;
#pragma unroll 1
        for (int cgj = 0; cgj < LC; ++cgj) {
            const int j = LC * kb + cgj;
            const bool owner = cg == cgj;
            // row j of the running R (chained tiles) is written by reflector j
            // alone, so this step's entries can be read at its start, their LDS
            // latency hidden behind the norm (measured: 2% off the leaf, 3% off
            // the tree at n = 32)
            double rpre[KC];
            if constexpr (!FIRST) {
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    rpre[k] = 0.0;
                    if (k < kb || k >= KHI) continue;
                    rpre[k] = Rs[rpk<NP>(j, LC * k + cg)];
                }
            }
            // FP32 tile: column j is final here, so its owner lanes publish it
            // unscaled through LDS now and the round trip overlaps the norm and
            // the square root below; every lane scales its copy once the scale is
            // known (the same products, so the same bits).  Measured: 2.7% off the
            // FP32 leaf at n = 64; the FP64 tile was 0.5-1.5% slower with the copy
            // live across the square root, so it broadcasts the scaled reflector.
            constexpr bool EARLY = sizeof(E) == 4;
            E raw[RL];
            if constexpr (EARLY) {
                if (owner) {
#pragma unroll
                    for (int i = 0; i < RL; ++i) my_vb[i] = a[i][kb];
                }
                // the other lanes read what the owners wrote: the compiler reasons
                // per lane, so this barrier keeps their loads after the owners' stores
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int i = 0; i < RL; ++i) raw[i] = my_vb[i];
            }
            // squared norm of the part of column j below the pivot (two chains)
            double sp0 = 0.0, sp1 = 0.0;
#pragma unroll
            for (int i = 0; i < RL; ++i) {
                if (i > imax) continue;
                double x = (double)a[i][kb];
                if (FIRST && LR * i + rg <= j) x = 0.0;
                if (i & 1) sp1 = fma(x, x, sp1);
                else sp0 = fma(x, x, sp0);
            }
            const double s = readlane_d(group_sum<LR>(sp0 + sp1), cgj * LR);
            double alpha;
            if (FIRST) alpha = (double)readlane_d(a[ij][kb], cgj * LR + rg0 + cgj);
            else alpha = Rs[rpk<NP>(j, j)];
            double beta, scale, tau;
            if constexpr (sizeof(E) == 8) {
                // A column whose squared norm alpha^2 + s leaves [2^-960, 2^1002)
                // (it overflowed, lost bits to underflow, or is zero) gets its
                // scalars from its entries scaled by a power of two 2^-e that
                // brings the largest to [1, 2): beta scales back by 2^e and the
                // reflector's scale by 2^-e, both exactly; tau does not change.
                // FP32 tiles (norms summed in FP64 from FP32 entries) never get
                // there.  The test is on the exponent bits of alpha^2 + s in
                // scalar registers (zero, inf and NaN fall outside); the branch is
                // wave-uniform and never taken on ordinary data, but it costs the
                // leaf about 2% (measured at n = 32: the scalar chain can no
                // longer be scheduled across it; a branch to an empty block costs
                // the same).
                double ac = alpha, sc2 = s, up = 1.0, down = 1.0;
                const unsigned hw = (unsigned)__builtin_amdgcn_readfirstlane(__double2hiint(fma(alpha, alpha, s)));
                if (__builtin_expect(hw - 0x03F00000u > 0x7E8FFFFFu - 0x03F00000u, 0)) {
                    double mx = 0.0;
#pragma unroll
                    for (int i = 0; i < RL; ++i) {
                        if (i > imax) continue;
                        double x = fabs((double)a[i][kb]);
                        if (FIRST && LR * i + rg <= j) x = 0.0;
                        mx = fmax(mx, x);
                    }
                    mx = fmax(readlane_d(group_max<LR>(mx), cgj * LR), fabs(alpha));
                    const int e = mx > 0.0 ? ilogb(mx) : 0;
                    down = ldexp(1.0, -e);
                    up = ldexp(1.0, e);
                    double q0 = 0.0, q1 = 0.0;
#pragma unroll
                    for (int i = 0; i < RL; ++i) {
                        if (i > imax) continue;
                        double x = (double)a[i][kb] * down;
                        if (FIRST && LR * i + rg <= j) x = 0.0;
                        if (i & 1) q1 = fma(x, x, q1);
                        else q0 = fma(x, x, q0);
                    }
                    sc2 = readlane_d(group_sum<LR>(q0 + q1), cgj * LR);
                    ac = alpha * down;
                }
                reflector_scalars(ac, sc2, beta, scale, tau);
                beta *= up;
                scale *= down;
            } else {
                reflector_scalars(alpha, s, beta, scale, tau);
            }
            // the reflector v_j (the owners scale their own column at the end of the tile)
            if (owner) sc[kb] = (E)scale;
            E vr[RL];
            if constexpr (EARLY) {
#pragma unroll
                for (int i = 0; i < RL; ++i) {
                    const int row = LR * i + rg;
                    E v = raw[i] * (E)scale;
                    if (FIRST) v = row > j ? v : (row == j ? E(1) : E(0));
                    vr[i] = v;
                }
            } else {
                if (owner) {
#pragma unroll
                    for (int i = 0; i < RL; ++i) {
                        const int row = LR * i + rg;
                        E v = a[i][kb] * (E)scale;
                        if (FIRST) v = row > j ? v : (row == j ? E(1) : E(0));
                        my_vb[i] = v;
                    }
                }
                __builtin_amdgcn_wave_barrier();  // as above: loads after the owners' stores
#pragma unroll
                for (int i = 0; i < RL; ++i) vr[i] = my_vb[i];
            }
            // dot products of v_j with the trailing columns this lane holds (two chains)
            E d[KC];
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                d[k] = E(0);
                if (k < kb || k >= KHI) continue;
                E acc0 = E(0), acc1 = E(0);
#pragma unroll
                for (int i = 0; i < RL; ++i) {
                    if (i > imax) continue;
                    if (i & 1) acc1 = fma(vr[i], a[i][k], acc1);
                    else acc0 = fma(vr[i], a[i][k], acc0);
                }
                d[k] = group_sum<LR>(acc0 + acc1);
            }
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const int c = LC * k + cg;
                if (k < kb || k >= KHI) continue;
                // k == kb: only the columns right of the pivot are trailing
                const bool trailing = (k > kb) || (cg > cgj);
                double w = (double)d[k];
                double rjc = 0.0;
                if (!FIRST) {
                    rjc = rpre[k];
                    w += rjc;
                }
                const double tw = trailing ? tau * w : 0.0;
#pragma unroll
                for (int i = 0; i < RL; ++i)
                    if (i <= imax) a[i][k] = fma(-(E)tw, vr[i], a[i][k]);
                if (!FIRST && rg == 0 && trailing) Rs[rpk<NP>(j, c)] = rjc - tw;
            }
            if (FIRST) {
                if (owner && rg == rg0 + cgj) a[ij][kb] = (E)beta;
            } else {
                if (lane == 0) Rs[rpk<NP>(j, j)] = beta;
            }
            if (lane == 0) taus[j] = tau;
        }
    }
    // R and tau are read by other lanes after the tile
    __builtin_amdgcn_wave_barrier();
}

// --------------------------------------------------------------------------
// Blocked factorization of a chained tile ([R; A_k], reflectors [e_j; y_j]) in
// the four-group layout (LC = 4: lane 16 cg + rg holds rows 16 i + rg, columns
// 4 k + cg), in panels of 16 columns (four slots).  A panel is factored by
// factor_tile restricted to its slots; its reflectors are scaled in place; then
// every later 16-column block C (slots 4b .. 4b+3) takes the panel's compact-WY
// update at once (Sec. 3.2):
//   W = R(P, C) + Y_P^T A_C,   W' = T_P^T W,   R(P, C) -= W',   A_C -= Y_P W'.
// Y_P^T [Y_P | A_C] contracts over rows, which sit on the lanes of a group, so
// 16-row chunks go through LDS (cb) into the f64 16x16x4 operand layout, as in
// gram_accumulate; Y_P^T Y_P gives T_P by the recurrence of build_T (Gd: dense
// 16 x 16 Gram, Ts: T_P at stride 17, both in the chunk buffer once the chunks
// are done: 16 (NP + 1) >= 256 + 272).  A_C -= Y_P W' maps the register layout
// onto itself: the output rows 4r + q of the op are the columns 4r + cg of slot
// 4b + r, its columns p the rows 16 i + rg, and the B operand of K step s is
// slot 4P + s of the same rows.
// --------------------------------------------------------------------------
template <int NP, int RL, int P>
__device__ __forceinline__ void panel_update(double (&a)[RL][NP / 4], double* Rs, double* cb, const double* taus,
                                             double* Ts, int lane)
{
    constexpr int NB = NP / 16, LDP = NP + 1, NL = NB - P - 1;  // later 16-column blocks
    static_assert(16 * LDP >= 256 + 272, "the panel's Gram and T fit in the chunk buffer");
    double* Gd = cb;
    const int q = lane >> 4, p = lane & 15;
    dbl4 G = dbl4{0.0, 0.0, 0.0, 0.0};
    dbl4 Z[NL > 0 ? NL : 1];
#pragma unroll
    for (int b = 0; b < NL; ++b) Z[b] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < RL; ++i) {
        // chunk = rows 16 i .. 16 i + 15: lane (q, p) holds row p of it, columns 4 k + q
#pragma unroll
        for (int k = 4 * P; k < NP / 4; ++k) cb[p * LDP + 4 * k + q] = a[i][k];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const double y = cb[(4 * s + q) * LDP + 16 * P + p];  // Y_P(4s + q, p)
            G = mfma16x16x4(y, y, G);
#pragma unroll
            for (int b = 0; b < NL; ++b) Z[b] = mfma16x16x4(y, cb[(4 * s + q) * LDP + 16 * (P + 1 + b) + p], Z[b]);
        }
        __builtin_amdgcn_wave_barrier();
    }
    // T_P: lane (q, p) holds G(4r + q, p); the recurrence on row p (every group alike)
#pragma unroll
    for (int r = 0; r < 4; ++r) Gd[16 * p + 4 * r + q] = (4 * r + q < p) ? G[r] : 0.0;
    __builtin_amdgcn_wave_barrier();
    {
        const double* tb = taus + 16 * P;
        double tr[16];
#pragma unroll
        for (int jl = 0; jl < 16; ++jl) tr[jl] = 0.0;
#pragma unroll
        for (int jl = 0; jl < 16; ++jl) {
            const double tj = tb[jl];
            double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
            for (int kl = 0; kl < jl; ++kl) {
                if (kl & 1) acc1 = fma(tr[kl], Gd[16 * jl + kl], acc1);
                else acc0 = fma(tr[kl], Gd[16 * jl + kl], acc0);
            }
            const double v = (p < jl) ? -tj * (acc0 + acc1) : (p == jl ? tj : 0.0);
            tr[jl] = v;
            if (q == 0) Ts[p + 17 * jl] = v;
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int b = 0; b < NL; ++b) {
        const int c0 = 16 * (P + 1 + b);
        // W = R(16P + 4r + q, c0 + p) + Z[r];  W' = T_P^T W
        dbl4 Rv, Wv;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Rv[r] = Rs[rpk<NP>(16 * P + 4 * r + q, c0 + p)];
            Wv[r] = Rv[r] + Z[b][r];
        }
        dbl4 Wp = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) Wp = mfma16x16x4(Ts[(4 * s + q) + 17 * p], Wv[s], Wp);
#pragma unroll
        for (int r = 0; r < 4; ++r) Rs[rpk<NP>(16 * P + 4 * r + q, c0 + p)] = Rv[r] - Wp[r];
        // A_C -= Y_P W', one 16-row block at a time, in place
#pragma unroll
        for (int i = 0; i < RL; ++i) {
            dbl4 c = dbl4{a[i][4 * (P + 1 + b) + 0], a[i][4 * (P + 1 + b) + 1], a[i][4 * (P + 1 + b) + 2],
                          a[i][4 * (P + 1 + b) + 3]};
#pragma unroll
            for (int s = 0; s < 4; ++s) c = mfma16x16x4(-Wp[s], a[i][4 * P + s], c);
#pragma unroll
            for (int r = 0; r < 4; ++r) a[i][4 * (P + 1 + b) + r] = c[r];
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// The blocked chained factorization (FP64, LC = 4, NP a multiple of 16).
// On return every reflector is scaled (sc is all ones).  TK: the T_P of every
// panel but the last is kept at TA + 272 P (16 x 16 at stride 17), the diagonal
// blocks of the tile's T (the recursive leaf variant assembles the rest);
// otherwise it lives in the chunk buffer only while its panel update runs.
template <int NP, int RL, int P = 0, bool TK = false>
__device__ __forceinline__ void factor_tile_blocked(double (&a)[RL][NP / 4], double (&sc)[NP / 4], double* Rs,
                                                    double* vb, double* taus, double* cb, double* TA, int lane)
{
    factor_tile<NP, RL, 4, false, double, 4 * P, 4 * P + 4>(a, sc, Rs, vb, taus, lane);
#pragma unroll
    for (int k = 4 * P; k < 4 * P + 4; ++k) {
#pragma unroll
        for (int i = 0; i < RL; ++i) a[i][k] *= sc[k];
        sc[k] = 1.0;
    }
    if constexpr (P + 1 < NP / 16) {
        panel_update<NP, RL, P>(a, Rs, cb, taus, TK ? TA + 272 * P : cb + 256, lane);
        factor_tile_blocked<NP, RL, P + 1, TK>(a, sc, Rs, vb, taus, cb, TA, lane);
    }
}

// Applies the deferred reflector scales: y = x * sc below the diagonal (FIRST)
// or in every row (chained tiles).
template <int NP, int RL, int LC, bool FIRST, typename E = double>
__device__ __forceinline__ void scale_tile(E (&a)[RL][NP / LC], const E (&sc)[NP / LC], int lane)
{
    constexpr int KC = NP / LC, LR = 64 / LC;
    const int cg = lane / LR, rg = lane % LR;
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int i = 0; i < RL; ++i) {
            if (FIRST) a[i][k] = (LR * i + rg > LC * k + cg) ? a[i][k] * sc[k] : a[i][k];
            else a[i][k] *= sc[k];
        }
}

// Gram matrix G = V^T V of a factored tile on the matrix cores.  The tile sits
// in registers in the factor layout (rows on the lanes of a group), which the
// f64 16x16x4 op cannot contract over; so 16-row chunks go through LDS (cb,
// 16 x (NP+1) doubles) and are read back with rows on the lane-group index:
// lane (q, p) takes rows 4s + q and column 16b + p, the operand layout of both
// V^T (A) and V (B).  Reflectors: FIRST tiles have v_c(r) = 0 above the
// diagonal and 1 on it; chained tiles [e_c; y_c] contribute y_c^T y_d
// (c != d).  Writes the strictly upper part G(c, d), c < d, to Gs.
template <int NP, int RL, int LC, bool FIRST, int CH, typename E>
__device__ __forceinline__ void gram_accumulate(const E (&a)[RL][NP / LC], double* cb,
                                                dbl4 (&acc)[round16(NP) / 16][round16(NP) / 16], int lane)
{
    constexpr int KC = NP / LC, LR = 64 / LC, MT = LR * RL, LDP = NP + 1;
    constexpr int NPB = round16(NP), JB = NPB / 16;
    static_assert(MT % CH == 0 && CH % 4 == 0, "gram chunks are whole multiples of the K step");
    const int cg = lane / LR, rg = lane % LR;
    const int q = lane >> 4, p = lane & 15;
#pragma unroll
    for (int ib = 0; ib < JB; ++ib)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) acc[ib][jb] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c0 = 0; c0 < MT; c0 += CH) {
        // this lane's rows inside the chunk [c0, c0 + CH)
#pragma unroll
        for (int i = 0; i < RL; ++i) {
            const int row = LR * i + rg;
            if (LR * i + LR <= c0 || LR * i >= c0 + CH) continue;  // slot outside the chunk (compile-time test
            if (row < c0 || row >= c0 + CH) continue;               // on i, runtime on rg)
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const int col = LC * k + cg;
                double v = (double)a[i][k];  // products of FP32 entries are exact in FP64
                if (FIRST) v = row > col ? v : (row == col ? 1.0 : 0.0);
                cb[(row - c0) * LDP + col] = v;
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int s = 0; s < CH / 4; ++s) {
            double vv[JB];
#pragma unroll
            for (int b = 0; b < JB; ++b) {
                const int col = 16 * b + p;
                vv[b] = col < NP ? cb[(4 * s + q) * LDP + col] : 0.0;
            }
#pragma unroll
            for (int ib = 0; ib < JB; ++ib)
#pragma unroll
                for (int jb = ib; jb < JB; ++jb) acc[ib][jb] = mfma16x16x4(vv[ib], vv[jb], acc[ib][jb]);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Position of G(k, j), k < j, in the strictly upper Gram packed by rows.
__host__ __device__ constexpr int grow(int np, int k, int j) { return k * (np - 1) - k * (k - 1) / 2 + (j - k - 1); }

// The factors of a tile's T for a later construction (k_build_T): the tile's
// T slot of np(np+1)/2 entries receives tau (np entries) followed by the
// strictly upper Gram packed by rows (a row of a 16 x 16 output block is 16
// consecutive entries, so the stores coalesce).  CH: rows per LDS chunk of the
// Gram (4 where the leaf's LDS would otherwise cost occupancy).
template <int NP, int RL, int LC, bool FIRST, int CH, typename E>
__device__ __forceinline__ void gram_out(const E (&a)[RL][NP / LC], double* cb, const double* taus,
                                         E* __restrict__ slot, int lane)
{
    constexpr int JB = round16(NP) / 16;
    const int q = lane >> 4, p = lane & 15;
    dbl4 acc[JB][JB];
    gram_accumulate<NP, RL, LC, FIRST, CH, E>(a, cb, acc, lane);
    if (lane < NP) slot[lane] = (E)taus[lane];
    // uniform base plus a 32-bit per-lane byte offset (one address register)
    E* g = slot + NP;
    const int qo = opaque(q), po = opaque(p);
#pragma unroll
    for (int ib = 0; ib < JB; ++ib)
#pragma unroll
        for (int jb = ib; jb < JB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * ib + qo + 4 * r, col = 16 * jb + po;
                if (row < col && col < NP)
                    st_at(g, (uint32_t)(grow(NP, row, col) * (int)sizeof(E)), (E)acc[ib][jb][r]);
            }
}

// The recursive leaf variant (the recursive local QR of Elmroth and Gustavson
// that Sec. 3.1 and 7 bring into TSQR): the tile's compact-WY factor T is put
// together inside the leaf kernel from its 16-column blocks, T = [T_L, X; 0,
// T_R] with X = -T_L (Y_L^T Y_R) T_R (the product of two compact-WY blocks,
// Sec. 3.2), so no separate T kernel runs over the leaf tiles.  The recursion
// halves the columns down to the 16-column block of the matrix cores, where a
// panel is factored column by column (factor_tile); widths of one or two
// blocks, whose T blocks fit beside the leaf's LDS (NP = 16, 32), have it.
__host__ __device__ constexpr bool leaf_rec_ok(int np) { return np % 16 == 0 && np / 16 <= 2; }
// LDS of the T blocks (16 x 16 at stride 17): diagonal block b at 272 b, the
// block above the diagonal (two blocks) at 272 * 2.
__host__ __device__ constexpr int rec_ta_doubles(int np) { return (np / 16) * (np / 16 + 1) / 2 * 272; }

// T of a factored tile of the four-group layout (LC = 4: lane 16 cg + rg holds
// rows 16 i + rg, columns 4 k + cg), scaled reflectors in a, tau in taus,
// written packed by columns (column c at c (c + 1) / 2, rows 0 .. c) to slot.
// The diagonal blocks b >= D0 come from the tile's Gram by the column
// recurrence t_j = -tau_j T (V^T v_j) (earlier ones are already in TA: the
// panel updates of the blocked factorisation formed them); the block above the
// diagonal from G_01 = Y_0^T Y_1 on the matrix cores.  16-row chunks of the tile
// go through cb (16 x (NP+1) doubles) into the f64 16x16x4 operand layout, as in
// gram_accumulate.  FIRST: reflector c has 1 in row c and zeros above.
template <int NP, int RL, bool FIRST, int D0>
__device__ __forceinline__ void tile_T(const double (&a)[RL][NP / 4], double* cb, const double* taus, double* TA,
                                       double* __restrict__ slot, int lane)
{
    constexpr int KC = NP / 4, LDP = NP + 1, NB = NP / 16;
    static_assert(leaf_rec_ok(NP) && D0 >= 0 && D0 < NB, "one split at most");
    static_assert(16 * LDP >= 256 * NB, "the dense diagonal Gram blocks fit in the chunk buffer");
    const int cg = lane >> 4, rg = lane & 15;
    const int q = lane >> 4, p = lane & 15;
    dbl4 G[NB], H = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < NB; ++b) G[b] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < RL; ++i) {
        // chunk i = rows 16 i .. 16 i + 15: lane (cg, rg) holds row rg of it
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            double v = a[i][k];
            if (FIRST) {
                const int row = 16 * i + rg, col = 4 * k + cg;
                v = row > col ? v : (row == col ? 1.0 : 0.0);
            }
            cb[rg * LDP + 4 * k + cg] = v;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            double y[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) y[b] = cb[(4 * s + q) * LDP + 16 * b + p];
#pragma unroll
            for (int b = D0; b < NB; ++b) G[b] = mfma16x16x4(y[b], y[b], G[b]);
            // H(4r + q, p) = (Y_1^T Y_0)(4r + q, p) = G_01(p, 4r + q): the A operand of G_01
            if constexpr (NB == 2) H = mfma16x16x4(y[1], y[0], H);
        }
        __builtin_amdgcn_wave_barrier();
    }
    // dense strictly upper diagonal Gram blocks, G(k, j) at cb + 256 b + 16 j + k
#pragma unroll
    for (int b = D0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) cb[256 * b + 16 * p + 4 * r + q] = (4 * r + q < p) ? G[b][r] : 0.0;
    __builtin_amdgcn_wave_barrier();
    {
        // lane group q builds the rows p of block b (groups past the blocks
        // repeat the last one without writing it)
        const int b = q < D0 ? D0 : (q < NB ? q : NB - 1);
        const double* gb = cb + 256 * b;
        const double* tb = taus + 16 * b;
        double tr[16];
#pragma unroll
        for (int jl = 0; jl < 16; ++jl) tr[jl] = 0.0;
#pragma unroll
        for (int jl = 0; jl < 16; ++jl) {
            const double tj = tb[jl];
            double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
            for (int kl = 0; kl < jl; ++kl) {
                if (kl & 1) acc1 = fma(tr[kl], gb[16 * jl + kl], acc1);
                else acc0 = fma(tr[kl], gb[16 * jl + kl], acc0);
            }
            const double v = (p < jl) ? -tj * (acc0 + acc1) : (p == jl ? tj : 0.0);
            tr[jl] = v;
            if (q == b) TA[272 * b + p + 17 * jl] = v;
        }
    }
    __builtin_amdgcn_wave_barrier();
    if constexpr (NB == 2) {
        // X = G_01 T_11, then T_01 = -T_00 X
        dbl4 X = dbl4{0.0, 0.0, 0.0, 0.0}, Y = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) X = mfma16x16x4(H[s], TA[272 + (4 * s + q) + 17 * p], X);
#pragma unroll
        for (int s = 0; s < 4; ++s) Y = mfma16x16x4(TA[p + 17 * (4 * s + q)], X[s], Y);
#pragma unroll
        for (int r = 0; r < 4; ++r) TA[544 + (4 * r + q) + 17 * p] = -Y[r];
        __builtin_amdgcn_wave_barrier();
    }
    // packed by columns: lane r writes row r of column c
    const int bi = lane >> 4, rl = lane & 15;
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        const int cbk = c / 16;
        const int blk = bi == cbk ? cbk : (bi < cbk ? NB + cbk * (cbk - 1) / 2 + bi : cbk);
        const double v = TA[272 * blk + rl + 17 * (c % 16)];
        if (lane <= c) slot[c * (c + 1) / 2 + lane] = v;
    }
    __builtin_amdgcn_wave_barrier();  // the next tile rewrites cb and TA
}

// Tile load/store in the factor layout.  The per-lane part of the address
// (row rg, column cg) is one loop-invariant offset; the rest is uniform, so the
// compiler does not keep one address per element alive across the chain.
template <int NP, int RL, int LC, typename E = double>
__device__ __forceinline__ void load_tile(E (&a)[RL][NP / LC], const double* tb, int64_t lda,
                                          int64_t lane_off, int64_t valid, int n, int rg, int cg)
{
    constexpr int KC = NP / LC, LR = 64 / LC, MT = LR * RL;
    if (valid == MT && n == NP) {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const double* cb = tb + (int64_t)(LC * k) * lda + lane_off;
#pragma unroll
            for (int i = 0; i < RL; ++i) a[i][k] = (E)cb[LR * i];
        }
    } else {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const double* cb = tb + (int64_t)(LC * k) * lda + lane_off;
            const bool cv = LC * k + cg < n;
#pragma unroll
            for (int i = 0; i < RL; ++i) a[i][k] = (cv && LR * i + rg < valid) ? (E)cb[LR * i] : E(0);
        }
    }
}

template <int NP, int RL, int LC, typename E = double>
__device__ __forceinline__ void store_tile(const E (&a)[RL][NP / LC], E* tb, int64_t lda,
                                           int64_t lane_off, int64_t valid, int n, int rg, int cg)
{
    constexpr int KC = NP / LC, LR = 64 / LC, MT = LR * RL;
    if (valid == MT && n == NP) {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            E* cb = tb + (int64_t)(LC * k) * lda + lane_off;
#pragma unroll
            for (int i = 0; i < RL; ++i) cb[LR * i] = a[i][k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            E* cb = tb + (int64_t)(LC * k) * lda + lane_off;
            const bool cv = LC * k + cg < n;
#pragma unroll
            for (int i = 0; i < RL; ++i)
                if (cv && LR * i + rg < valid) cb[LR * i] = a[i][k];
        }
    }
}

// --------------------------------------------------------------------------
// Leaf kernel: one wavefront per leaf, the flat chain over its tiles.
// --------------------------------------------------------------------------
// E = float is the first pass of the mixed-precision path: the tile is held
// and updated in FP32 (FP32 dot products over at most 1024 rows, combined
// pairwise across lanes), while the reflector scalars (norm, beta, tau), the
// running triangle R and the Gram entries of T stay FP64.  V goes to a
// workspace of whole tiles (rows past m and columns past n are zeros) and T is
// rounded to FP32.
// With Q, each tile's T slot receives tau and the Gram entries (gram_out) and
// the T kernel (k_build_T, k_build_T_batch) forms T afterwards, so the leaf's
// LDS holds only a chunk buffer for the Gram.
// REC: the recursive variant (tile_T): each tile's T is written to its slot
// by the leaf itself; the LDS then also holds the T blocks (rec_ta_doubles).
template <int NP, bool WANT_Q, typename E, bool REC = false>
__device__ __forceinline__ void leaf_chain(const double* A, int64_t lda, E* V, int64_t ldv, int64_t m, int n,
                                           int64_t P, int64_t leaf_rows, int64_t f, E* __restrict__ Ttile,
                                           double* __restrict__ Rleaf, int64_t leaf, double* wsm, int lane)
{
    constexpr bool MIXED = sizeof(E) == 4;
    constexpr bool BLK = leaf_blocked<E>(NP);
    constexpr bool RT = REC && WANT_Q;
    static_assert(!REC || (!MIXED && leaf_rec_ok(NP) && leaf_col_groups<E>(NP) == 4),
                  "the recursive variant: FP64, one or two 16-column blocks, four column groups");
    constexpr int LC = leaf_col_groups<E>(NP), LR = 64 / LC, MT = tile_rows_e<E>(NP), RL = MT / LR, KC = NP / LC;
    constexpr int NT = packed_size(NP);
    constexpr int CH = leaf_gram_chunk<E>(NP, MT);
    constexpr int GA = (!WANT_Q && !BLK) ? 0 : (CH * (NP + 1) + 1) / 2 * 2;
    const int cg = lane / LR, rg = lane % LR;
    double* Rs = wsm;
    double* Gs = Rs + r_area(NP);
    E* vb = reinterpret_cast<E*>(Gs + GA);
    double* taus = Gs + GA + (LR * vb_stride_e<E>(RL) * (int)sizeof(E) + 7) / 8;
    double* TA = taus + NP;  // RT: the T blocks

    const int64_t row0 = leaf * leaf_rows;
    const int64_t rows = (leaf == P - 1) ? (m - row0) : leaf_rows;
    const int64_t ntl = (rows + MT - 1) / MT;
    const int64_t lane_off = rg + (int64_t)cg * lda;
    const int64_t lane_off_v = rg + (int64_t)cg * ldv;
    E a[RL][KC], sc[KC];
    // tile 0 (peeled: a branch between the two factor variants inside the
    // loop would make the register allocator keep two copies of the tile)
    {
        const int64_t valid = rows < MT ? rows : MT;
        load_tile<NP, RL, LC, E>(a, A + row0, lda, lane_off, valid, n, rg, cg);
        factor_tile<NP, RL, LC, true, E>(a, sc, Rs, vb, taus, lane);
        // the tile's top NP rows hold R on and above the diagonal
#pragma unroll
        for (int i = 0; i < (NP + LR - 1) / LR; ++i) {
            const int r = LR * i + rg;
            if (r < NP) {
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    const int c = LC * k + cg;
                    if (r <= c) Rs[rpk<NP>(r, c)] = (double)a[i][k];
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (WANT_Q) {
            scale_tile<NP, RL, LC, true, E>(a, sc, lane);
            // the mixed workspace takes whole tiles (zero rows and columns included)
            store_tile<NP, RL, LC, E>(a, V + row0, ldv, lane_off_v, MIXED ? MT : valid, MIXED ? NP : n, rg, cg);
            if constexpr (RT) tile_T<NP, RL, true, 0>(a, Gs, taus, TA, Ttile + (leaf * f) * NT, lane);
            else gram_out<NP, RL, LC, true, CH, E>(a, Gs, taus, Ttile + (leaf * f) * NT, lane);
        }
    }
    for (int64_t t = 1; t < ntl; ++t) {
        const int64_t t0 = row0 + t * MT;
        const int64_t valid = (rows - t * MT) < MT ? (rows - t * MT) : MT;
        load_tile<NP, RL, LC, E>(a, A + t0, lda, lane_off, valid, n, rg, cg);
        if constexpr (BLK) factor_tile_blocked<NP, RL, 0, RT>(a, sc, Rs, vb, taus, Gs, TA, lane);
        else factor_tile<NP, RL, LC, false, E>(a, sc, Rs, vb, taus, lane);
        if (WANT_Q) {
            scale_tile<NP, RL, LC, false, E>(a, sc, lane);
            store_tile<NP, RL, LC, E>(a, V + t0, ldv, lane_off_v, MIXED ? MT : valid, MIXED ? NP : n, rg, cg);
            if constexpr (RT)
                tile_T<NP, RL, false, BLK ? NP / 16 - 1 : 0>(a, Gs, taus, TA, Ttile + (leaf * f + t) * NT, lane);
            else gram_out<NP, RL, LC, false, CH, E>(a, Gs, taus, Ttile + (leaf * f + t) * NT, lane);
        }
    }
    __builtin_amdgcn_wave_barrier();
    double* Ro = Rleaf + leaf * NP * NP;
    for (int idx = lane; idx < NP * NP; idx += 64) {
        const int r = idx % NP, c = idx / NP;
        Ro[idx] = r <= c ? Rs[rpk<NP>(r, c)] : 0.0;
    }
}

// Per-wave LDS of the single-problem leaf kernel (REC: with the T blocks).
template <typename E = double>
__host__ __device__ constexpr int leaf_kernel_lds_doubles(int np, bool want_q, bool rec)
{
    return leaf_lds_doubles<E>(np, tile_rows_e<E>(np), want_q) + (rec && want_q ? rec_ta_doubles(np) : 0);
}

template <int NP, bool WANT_Q, typename E = double, bool REC = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_leaf_factor(const double* A, int64_t lda, E* V, int64_t ldv,
                                                     int64_t m, int n, int64_t P, int64_t leaf_rows, int64_t f,
                                                     E* __restrict__ Ttile, double* __restrict__ Rleaf)
{
    constexpr int WS = leaf_kernel_lds_doubles<E>(NP, WANT_Q, REC);
    extern __shared__ double smem[];
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t leaf = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (leaf >= P) return;
    leaf_chain<NP, WANT_Q, E, REC>(A, lda, V, ldv, m, n, P, leaf_rows, f, Ttile, Rleaf, leaf, smem + wave * WS,
                                   lane);
}

// T of every leaf tile (slots 0 .. ntiles-1, one wavefront each) from the tau
// and Gram entries the leaf kernel left in the slot (see gram_out), in place,
// in 16-column blocks (NB = ceil(NP / 16)):
//  - the diagonal blocks T_bb by the column recurrence of build_T, block b on
//    lanes 16b .. 16b+15 (lane 16b + r builds its row r), all blocks at once;
//  - then block column j = 1 .. NB-1 from the columns left of it on the matrix
//    cores, T(0:16j, blk j) = -T(0:16j, 0:16j) G(0:16j, blk j) T_jj (the
//    compact-WY product of two reflector blocks, Sec. 3.2): X_i = G_ij T_jj,
//    T_ij = -sum_{k=i}^{j-1} T_ik X_k.
// Each lane reads only its own operands (no broadcast of the whole Gram to
// every lane).  The blocks of T are staged in LDS at stride 17 (16 x 17
// doubles); the dense diagonal Gram blocks are staged in the space of the
// off-diagonal T blocks where it suffices (they are consumed before those are
// written).  Every read of the slot comes before the first write of T.
template <int NP>
struct BuildTLds {
    static constexpr int NB = round16(NP) / 16, NBLK = NB * (NB + 1) / 2;
    static constexpr bool GD_SHARED = (NBLK - NB) * 272 >= NB * 256;
    static constexpr int GD_OFF = GD_SHARED ? NB * 272 : NBLK * 272;
    static constexpr int TAU_OFF = GD_SHARED ? NBLK * 272 : NBLK * 272 + NB * 256;
    static constexpr int WS = TAU_OFF + 64;
};

template <int NP, typename E>
__device__ __forceinline__ void build_T_slot(E* __restrict__ slot, double* W, int lane)
{
    using S = BuildTLds<NP>;
    constexpr int NB = S::NB, NOFF = NB * (NB - 1) / 2;
    double* Gd = W + S::GD_OFF;
    double* taus = W + S::TAU_OFF;
    const int q = lane >> 4, p = lane & 15;

    // ---- reads: tau, the dense diagonal Gram blocks and the off-diagonal ones
    // as A operands (ga[o][s] = G(16 i + p, 16 j + 4 s + q) for the o-th pair
    // i < j).  FP32 slots are first copied, coalesced, into LDS as they stand
    // (the T-block area, not in use yet) and gathered there (per-lane gathers of
    // 4-byte entries waste most of each line); FP64 entries are gathered from
    // the slot directly, which measured faster.
    constexpr int NT = packed_size(NP), U = (NT + 63) / 64;
    constexpr bool STAGE = sizeof(E) == 4;
    static_assert(NT <= S::NBLK * 272, "the slot fits in the T-block area");
    if constexpr (STAGE) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = 64 * u + lane < NT ? (double)slot[64 * u + lane] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (64 * u + lane < NT) W[64 * u + lane] = v[u];
        __builtin_amdgcn_wave_barrier();
    }
    auto graw = [&](int e) { return STAGE ? W[NP + e] : (double)slot[NP + e]; };
    const double tau_l = lane < NP ? (STAGE ? W[lane] : (double)slot[lane]) : 0.0;
    double gdv[NB * 4];
#pragma unroll
    for (int u = 0; u < NB * 4; ++u) {
        const int e = 64 * u + lane, bb = e >> 8, jl = (e >> 4) & 15, kl = e & 15, j = 16 * bb + jl;
        gdv[u] = (kl < jl && j < NP) ? graw(grow(NP, 16 * bb + kl, j)) : 0.0;
    }
    double ga[NOFF > 0 ? NOFF : 1][4];
#pragma unroll
    for (int j = 1; j < NB; ++j)
#pragma unroll
        for (int i = 0; i < j; ++i)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int col = 16 * j + 4 * s + q;
                ga[j * (j - 1) / 2 + i][s] = col < NP ? graw(grow(NP, 16 * i + p, col)) : 0.0;
            }
    __builtin_amdgcn_wave_barrier();  // Gd and tau below overwrite the staged slot
    taus[lane] = tau_l;
#pragma unroll
    for (int u = 0; u < NB * 4; ++u) Gd[64 * u + lane] = gdv[u];
    __builtin_amdgcn_wave_barrier();

    // ---- diagonal blocks (columns past NP have tau = 0 and come out zero)
    {
        const int b = q < NB ? q : NB - 1, r = p;
        const double* gb = Gd + 256 * b;
        const double* tb = taus + 16 * b;
        double* td = W + 272 * b + r;
        double tr[16];
#pragma unroll
        for (int jl = 0; jl < 16; ++jl) tr[jl] = 0.0;
#pragma unroll
        for (int jl = 0; jl < 16; ++jl) {
            const double tj = tb[jl];
            double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
            for (int kl = 0; kl < jl; ++kl) {
                if (kl & 1) acc1 = fma(tr[kl], gb[16 * jl + kl], acc1);
                else acc0 = fma(tr[kl], gb[16 * jl + kl], acc0);
            }
            const double v = (r < jl) ? -tj * (acc0 + acc1) : (r == jl ? tj : 0.0);
            tr[jl] = v;
            if (q < NB) td[17 * jl] = v;
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    __builtin_amdgcn_wave_barrier();  // the diagonal blocks are read across lanes, Gd is dead

    // ---- block columns 1 .. NB-1
#pragma unroll
    for (int j = 1; j < NB; ++j) {
        const double* Tjj = W + 272 * j;
        dbl4 X[NB > 1 ? NB - 1 : 1];
#pragma unroll
        for (int i = 0; i < j; ++i) {
            X[i] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4; ++s)
                X[i] = mfma16x16x4(ga[j * (j - 1) / 2 + i][s], Tjj[(4 * s + q) + 17 * p], X[i]);
        }
#pragma unroll
        for (int i = 0; i < j; ++i) {
            dbl4 Y = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = i; k < j; ++k) {
                const double* Tik = W + 272 * (k == i ? i : NB + k * (k - 1) / 2 + i);
#pragma unroll
                for (int s = 0; s < 4; ++s) Y = mfma16x16x4(Tik[p + 17 * (4 * s + q)], X[k][s], Y);
            }
            double* Tij = W + 272 * (NB + j * (j - 1) / 2 + i);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) Tij[(4 * rr + q) + 17 * p] = -Y[rr];
        }
        __builtin_amdgcn_wave_barrier();  // block column j is an operand of the next ones
    }

    // ---- T packed by columns (column c at c(c+1)/2), lane r writes row r
    const int bi = lane >> 4, rl = lane & 15;
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        const int cb = c / 16;
        const int blk = bi == cb ? cb : NB + cb * (cb - 1) / 2 + (bi < cb ? bi : 0);
        const double v = W[272 * blk + rl + 17 * (c % 16)];
        if (lane <= c) slot[c * (c + 1) / 2 + lane] = (E)v;
    }
    __builtin_amdgcn_wave_barrier();  // a next slot rewrites this wave's LDS
}

template <int NP, typename E>
__global__ void __launch_bounds__(256) k_build_T(E* __restrict__ Ttile, int64_t ntiles)
{
    extern __shared__ double smem[];
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (g >= ntiles) return;
    build_T_slot<NP, E>(Ttile + g * packed_size(NP), smem + wave * BuildTLds<NP>::WS, lane);
}
// Visits the NP x NP doubles at src, lane-strided (element idx = 64 u + lane),
// with the global loads issued 16 at a time before their uses: a plain strided
// loop waits for every load in turn.
template <int NP, typename F>
__device__ __forceinline__ void visit_block(const double* __restrict__ src, int lane, F&& f)
{
    constexpr int U = (NP * NP + 63) / 64, CHUNK = 16;
#pragma unroll
    for (int u0 = 0; u0 < U; u0 += CHUNK) {
        double v[CHUNK];
#pragma unroll
        for (int u = 0; u < CHUNK; ++u) {
            const int idx = 64 * (u0 + u) + lane;
            v[u] = (u0 + u < U && idx < NP * NP) ? src[idx] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < CHUNK; ++u) {
            const int idx = 64 * (u0 + u) + lane;
            if (u0 + u < U && idx < NP * NP) f(idx, v[u]);
        }
    }
}

// --------------------------------------------------------------------------
// One level of the binary tree: node q stacks R_{2q} on R_{2q+1} (lower index
// on top) and factors the pair; an odd last entry is passed up unchanged
// (Alg. 1).  Y1 (upper triangular) and T of the node are kept for the
// broadcast of Q.
// --------------------------------------------------------------------------
template <int NP, bool WANT_Q>
__device__ __forceinline__ void tree_node(const double* __restrict__ Rin, int64_t cin, double* __restrict__ Rout,
                                          double* __restrict__ Ynode, double* __restrict__ Tnode, int64_t q,
                                          double* wsm, int lane)
{
    constexpr int LC = col_groups(NP), LR = 64 / LC, KC = NP / LC;
    // the node tile holds R_b (NP rows), padded with zero rows to whole 16-row
    // chunks of gram_out
    constexpr int RLN = round16(NP) / LR, NT = packed_size(NP);
    constexpr int GA = WANT_Q ? gram_area(NP) : 0;
    const int cg = lane / LR, rg = lane % LR;
    const int64_t ia = 2 * q, ib = 2 * q + 1;
    const double* Ra = Rin + ia * NP * NP;
    double* Ro = Rout + q * NP * NP;
    if (ib >= cin) {
        visit_block<NP>(Ra, lane, [&](int idx, double v) { Ro[idx] = v; });
        return;
    }
    double* Rs = wsm;
    double* Gs = Rs + r_area(NP);
    double* vb = Gs + GA;
    double* taus = vb + LR * vb_stride(RLN);
    visit_block<NP>(Ra, lane, [&](int idx, double v) {
        const int r = idx % NP, c = idx / NP;
        if (r <= c) Rs[rpk<NP>(r, c)] = v;
    });
    const double* Rb = Rin + ib * NP * NP;
    double a[RLN][KC], sc[KC];
#pragma unroll
    for (int i = 0; i < RLN; ++i) {
        const int r = LR * i + rg;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int c = LC * k + cg;
            a[i][k] = (r < NP) ? Rb[r + c * NP] : 0.0;
        }
    }
    __builtin_amdgcn_wave_barrier();
    factor_tile<NP, RLN, LC, false, double, 0, NP / LC, true>(a, sc, Rs, vb, taus, lane);
    if (WANT_Q) {
        scale_tile<NP, RLN, LC, false>(a, sc, lane);
        // tau and the Gram entries of Y1 to the node's T slot; the T kernel
        // forms T there once the tree is done (as for the leaf tiles)
        gram_out<NP, RLN, LC, false, 16, double>(a, Gs, taus, Tnode + q * NT, lane);
        double* Y = Ynode + q * NP * NP;
#pragma unroll
        for (int i = 0; i < RLN; ++i) {
            const int r = LR * i + rg;
            if (r < NP) {
#pragma unroll
                for (int k = 0; k < KC; ++k) Y[r + (LC * k + cg) * NP] = a[i][k];
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    for (int idx = lane; idx < NP * NP; idx += 64) {
        const int r = idx % NP, c = idx / NP;
        Ro[idx] = r <= c ? Rs[rpk<NP>(r, c)] : 0.0;
    }
}

template <int NP, bool WANT_Q>
__global__ void __launch_bounds__(256) k_tree_level(const double* __restrict__ Rin, int64_t cin,
                                                    double* __restrict__ Rout, double* __restrict__ Ynode,
                                                    double* __restrict__ Tnode, int64_t cout)
{
    constexpr int WS = factor_lds_doubles<double>(NP, round16(NP), WANT_Q);
    extern __shared__ double smem[];
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (q >= cout) return;
    tree_node<NP, WANT_Q>(Rin, cin, Rout, Ynode, Tnode, q, smem + wave * WS, lane);
}

// --------------------------------------------------------------------------
// Root: signs D = diag(sgn(R_jj)) (sgn(0) = +1), the user's R = D R with its
// strictly lower part zeroed, and the root seed diag(D) of the broadcast.
// --------------------------------------------------------------------------
template <int NP>
__device__ __forceinline__ void root_body(const double* __restrict__ Rroot, int n, double* __restrict__ R,
                                          int64_t ldr, double* __restrict__ Dsig, double* __restrict__ Sroot, int lane)
{
    for (int idx = lane; idx < NP * NP; idx += 64) {
        const int i = idx % NP, j = idx / NP;
        const double di = Rroot[i + i * NP] < 0.0 ? -1.0 : 1.0;
        if (i < n && j < n) R[i + (int64_t)j * ldr] = (i <= j) ? di * Rroot[idx] : 0.0;
        if (Sroot) Sroot[idx] = (i == j) ? di : 0.0;
    }
    if (lane < NP) Dsig[lane] = Rroot[lane + lane * NP] < 0.0 ? -1.0 : 1.0;
}

template <int NP>
__global__ void __launch_bounds__(64) k_root(const double* __restrict__ Rroot, int n, double* __restrict__ R,
                                             int64_t ldr, double* __restrict__ Dsig, double* __restrict__ Sroot)
{
    root_body<NP>(Rroot, n, R, ldr, Dsig, Sroot, threadIdx.x);
}

// The 16x16x4 matrix-core op in FP64 or FP32.  Both take A(i, k) from lane
// 16k + i and B(k, j) from lane 16k + j; the output rows differ: lane
// 16q + p, register r holds D(q + 4r, p) in FP64 and D(4q + r, p) in FP32.
// A block computed by one product and fed to the next as the B operand keeps
// the rows it came out with, so slot s of such a register block holds row
// krow(s, q) = 16 (s / 4) + out_row(q, s % 4), and the A operand of the next
// product is loaded with the same permutation of its k index.
template <typename E> struct Mfma;
template <> struct Mfma<double> {
    typedef dbl4 acc_t;
    __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
    __device__ static acc_t mma(double a, double b, acc_t c) { return mfma16x16x4(a, b, c); }
    __host__ __device__ static constexpr int out_row(int q, int r) { return q + 4 * r; }
};
template <> struct Mfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    __device__ static acc_t zero() { return acc_t{0.0f, 0.0f, 0.0f, 0.0f}; }
    __device__ static acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __host__ __device__ static constexpr int out_row(int q, int r) { return 4 * q + r; }
};
template <typename E>
__host__ __device__ constexpr int krow(int s, int q) { return 16 * (s / 4) + Mfma<E>::out_row(q, s % 4); }

// Z = T S with T upper triangular (packed by columns, column j at j(j+1)/2) in
// global memory, S in registers with Sr[s][jb] = S(krow(s, q), 16 jb + p).
// The result comes back in the same register layout.
template <int NP, int JW = round16(NP) / 16, typename E = double>
__device__ __forceinline__ void tri_times_regs(const E* __restrict__ T, const E (&Sr)[round16(NP) / 4][JW],
                                               E (&Zr)[round16(NP) / 4][JW], int lane)
{
    constexpr int NPB = round16(NP), JB = NPB / 16, KS = NPB / 4;
    const int ln = opaque(lane);
    const int cg = ln >> 4, rg = ln & 15;
#pragma unroll
    for (int ib = 0; ib < JB; ++ib) {
        // T(16 ib + p, c) vanishes for c < 16 ib: those k-steps are skipped
        E tv[KS];
#pragma unroll
        for (int s = 4 * ib; s < KS; ++s) {
            const int r = 16 * ib + rg, c = krow<E>(s, cg);
            const bool ok = r <= c && c < NP;
            // unconditional load, in bounds
            const E v = ld_at(T, (uint32_t)(ok ? c * (c + 1) / 2 + r : 0) * (uint32_t)sizeof(E));
            tv[s] = ok ? v : E(0);
        }
#pragma unroll
        for (int jb = 0; jb < JW; ++jb) {
            typename Mfma<E>::acc_t acc = Mfma<E>::zero();
#pragma unroll
            for (int s = 4 * ib; s < KS; ++s) acc = Mfma<E>::mma(tv[s], Sr[s][jb], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) Zr[4 * ib + r][jb] = acc[r];
        }
    }
}

// Columns 16 j0 .. 16 (j0 + JW) - 1 of an NP x NP FP64 seed (column-major,
// leading dimension NP) into / out of the register layout above.
template <int NP, int JW = round16(NP) / 16, typename E = double>
__device__ __forceinline__ void load_seed(const double* __restrict__ S, E (&Sr)[round16(NP) / 4][JW], int lane,
                                          int j0 = 0)
{
    constexpr int NPB = round16(NP), KS = NPB / 4;
    const int cg = lane >> 4, rg = lane & 15;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int jb = 0; jb < JW; ++jb) {
            const int r = krow<E>(s, cg), c = 16 * (j0 + jb) + rg;
            const bool ok = r < NP && c < NP;
            const double v = S[ok ? r + c * NP : 0];
            Sr[s][jb] = ok ? (E)v : E(0);
        }
}

template <int NP, int JW = round16(NP) / 16>
__device__ __forceinline__ void store_seed(double* __restrict__ S, const double (&Sr)[round16(NP) / 4][JW], int lane,
                                           int j0 = 0)
{
    constexpr int NPB = round16(NP), KS = NPB / 4;
    const int cg = lane >> 4, rg = lane & 15;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int jb = 0; jb < JW; ++jb) {
            const int r = krow<double>(s, cg), c = 16 * (j0 + jb) + rg;
            if (r < NP && c < NP) S[r + c * NP] = Sr[s][jb];
        }
}

// --------------------------------------------------------------------------
// One level of the top-down seed descent.  A node with seed S hands
// (I - T) S = S - Z to its top child and -Y1 Z to its bottom child, Z = T S
// (from (I - [I; Y1] T [I; Y1]^T) [S; 0]).  A pass-through node hands S down.
// --------------------------------------------------------------------------
template <int NP>
__device__ __forceinline__ void seed_node(const double* __restrict__ Sp, const double* __restrict__ Ynode,
                                          const double* __restrict__ Tnode, int64_t cin, double* __restrict__ Sc,
                                          int64_t q, int lane)
{
    constexpr int NPB = round16(NP), JB = NPB / 16, KS = NPB / 4, NT = packed_size(NP);
    const int cg = lane >> 4, rg = lane & 15;
    const int64_t ia = 2 * q, ib = 2 * q + 1;
    const double* S = Sp + q * NP * NP;
    if (ib >= cin) {
        visit_block<NP>(S, lane, [&](int idx, double v) { Sc[ia * NP * NP + idx] = v; });
        return;
    }
    double Sr[KS][JB], Zr[KS][JB];
    load_seed<NP>(S, Sr, lane);
    tri_times_regs<NP>(Tnode + q * NT, Sr, Zr, lane);
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) Sr[s][jb] -= Zr[s][jb];
    store_seed<NP>(Sc + ia * NP * NP, Sr, lane);
    // bottom child: -Y1 Z, Y1 read as the A operand straight from memory
    const double* Y = Ynode + q * NP * NP;
    double* Sb = Sc + ib * NP * NP;
#pragma unroll
    for (int ibk = 0; ibk < JB; ++ibk) {
        double yv[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int r = 16 * ibk + rg, c = 4 * s + cg;
            yv[s] = (r < NP && c < NP) ? Y[r + c * NP] : 0.0;
        }
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < KS; ++s) acc = mfma16x16x4(yv[s], Zr[s][jb], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * ibk + cg + 4 * r, col = 16 * jb + rg;
                if (row < NP && col < NP) Sb[row + col * NP] = -acc[r];
            }
        }
    }
}

template <int NP>
__global__ void __launch_bounds__(256) k_seed_level(const double* __restrict__ Sp, const double* __restrict__ Ynode,
                                                    const double* __restrict__ Tnode, int64_t cin,
                                                    double* __restrict__ Sc, int64_t cout)
{
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (q >= cout) return;
    seed_node<NP>(Sp, Ynode, Tnode, cin, Sc, q, lane);
}

// --------------------------------------------------------------------------
// Q kernel: a leaf's chain replayed from the last tile to the first.
// Tile k > 0: Z = T_k S_k, Q_k = -Y_k Z, S_{k-1} = S_k - Z.
// Tile 0: W = V_top^T S_0, Z = T_0 W, Q_0 = [S_0; 0] - V_0 Z.
// Every step acts on the seed's columns independently, so a leaf may be split
// over several wavefronts, each owning 16 JW of the seed's (and Q's) columns;
// they read the same V tiles at about the same time, the second read coming
// from L2.  The products run on the matrix cores; Q may alias V.
// --------------------------------------------------------------------------
// Column windows of 16 per wavefront: all of them up to 48 columns; above, two
// per wavefront in FP64 (a leaf on two wavefronts), all four in FP32 (one).
// Every wavefront of a leaf reads the leaf's V and T tiles, so fewer, wider
// windows cut that repeated traffic, as far as the registers allow.
#ifndef TSQR_FQ_F32_WINDOWS
#define TSQR_FQ_F32_WINDOWS 4
#endif
template <typename E = double>
constexpr int fq_col_blocks(int np)
{
    return round16(np) / 16 <= 3 ? round16(np) / 16 : (sizeof(E) == 8 ? 2 : TSQR_FQ_F32_WINDOWS);
}

// The seed windows in LDS: element (r, c) of a window at r + c ss_ld, the row
// stride padded past the padded width so that the 16 lanes of a group (which
// read 16 consecutive columns of one row) fall on different LDS banks (with a
// stride of round16(np) doubles they all hit the same banks).
template <typename E>
__host__ __device__ constexpr int ss_ld(int npb) { return sizeof(E) == 8 ? npb + 4 : npb + 1; }
// LDS elements (of E) per wavefront of the Q kernels: JW windows of 16 columns.
template <typename E>
__host__ __device__ constexpr int fq_lds_elems(int np, int jw) { return ss_ld<E>(round16(np)) * 16 * jw; }

// E = float is the first pass of the mixed-precision path: V and T in FP32
// from the mixed leaf kernel, the FP64 seeds rounded to FP32, products on the
// FP32 matrix cores, and Q1 written to a workspace of whole tiles and
// round16(NP) columns (rows past m hold values of zero rows of V; columns past
// n are zero).  Rows past m and columns past n of V are zeros there too, so
// no load or store needs a mask.
// NTQ: the FP64 Q is written with non-temporal stores (a single large problem:
// 1% off the Q kernel at n = 32; the batched plans' ragged small problems
// measured 8% slower with them).
// One step of a leaf's seed windows jofs .. jofs + JN - 1 (16 columns each,
// held in LDS at Ss in the register layout of the products): for a chained
// tile (first == false) Z = T S and the window becomes S - Z (the seed of the
// tile above); for the chain's first tile, Z = T (V_top^T S_0) with V_top the
// unit lower triangle of the tile's top rows, and S_0 stays (the [S_0; 0]
// term of the expansion).
template <int NP, int JN, typename E>
__device__ __forceinline__ void seed_windows(const E* __restrict__ T, const E* V, int64_t t0, int64_t lda,
                                             int64_t valid, int n, bool first, E* Ss, int jofs,
                                             E (&Zr)[round16(NP) / 4][JN], int lane)
{
    constexpr int NPB = round16(NP), JB = NPB / 16, KS = NPB / 4, SLD = ss_ld<E>(NPB);
    typedef Mfma<E> MM;
    const int cg = lane >> 4, rg = lane & 15;
    E Sr[KS][JN];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int jb = 0; jb < JN; ++jb) Sr[s][jb] = Ss[krow<E>(s, cg) + (16 * (jofs + jb) + rg) * SLD];
    if (!first) {
        tri_times_regs<NP, JN, E>(T, Sr, Zr, lane);
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int jb = 0; jb < JN; ++jb) Ss[krow<E>(s, cg) + (16 * (jofs + jb) + rg) * SLD] = Sr[s][jb] - Zr[s][jb];
    } else {
        E Wr[KS][JN];
#pragma unroll
        for (int ib = 0; ib < JB; ++ib) {
            // V_top(r, 16 ib + p) vanishes for r < 16 ib
            E vt[KS];
#pragma unroll
            for (int s = 4 * ib; s < KS; ++s) {
                const int r = krow<E>(s, cg), c = 16 * ib + rg;  // V_top(r, c)
                const bool ok = r > c && r < valid && c < n;
                const E v = V[t0 + (ok ? r + (int64_t)c * lda : 0)];
                vt[s] = ok ? v : (r == c && r < NP ? E(1) : E(0));
            }
#pragma unroll
            for (int jb = 0; jb < JN; ++jb) {
                typename MM::acc_t acc = MM::zero();
#pragma unroll
                for (int s = 4 * ib; s < KS; ++s) acc = MM::mma(vt[s], Sr[s][jb], acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) Wr[4 * ib + r][jb] = acc[r];
            }
        }
        tri_times_regs<NP, JN, E>(T, Wr, Zr, lane);
    }
}

template <int NP, bool WIDE, typename E, bool NTQ = false, int JWT = fq_col_blocks<E>(NP)>
__device__ __forceinline__ void form_q_leaf(const E* V, int64_t lda, int64_t m, int n, int64_t P, int64_t leaf_rows,
                                            int64_t f, const E* __restrict__ Ttile, const double* __restrict__ Sleaf,
                                            E* Q, int64_t ldq, int64_t leaf, int j0, E* Ss, int lane)
{
    constexpr bool MIXED = sizeof(E) == 4;
    constexpr int MT = tile_rows_e<E>(NP), RL = MT / 16, KC = NP / 4;
    constexpr int NPB = round16(NP), JB = NPB / 16, KS = NPB / 4, NT = packed_size(NP), SLD = ss_ld<E>(NPB);
    // k-steps of the expansion: the FP32 permutation of k mixes the columns of
    // a 16-block, so whole blocks are contracted (their padding is zero)
    constexpr int KX = MIXED ? KS : KC;
    constexpr int JW = JWT;
    constexpr int FQU = NP > 48 ? 1 : 2;  // row blocks in flight; more spills at the widest tiles
    // FP64 with more than two windows per wavefront: the seed step runs one
    // window at a time (a seed and its product for all four would not fit the registers)
    constexpr bool PERW = !MIXED && JW > 2;
    static_assert(JB % JW == 0, "column window must divide the padded width");
    typedef Mfma<E> MM;
    const int cg = lane >> 4, rg = lane & 15;
    // the seed window lives in LDS between tile steps (each lane owns the
    // elements of its register layout); at tile 0 it is S_0 for the [S_0; 0] term

    const int64_t row0 = leaf * leaf_rows;
    const int64_t rows = (leaf == P - 1) ? (m - row0) : leaf_rows;
    const int64_t ntl = (rows + MT - 1) / MT;
    {
        E Sr[KS][JW];
        load_seed<NP, JW, E>(Sleaf + leaf * NP * NP, Sr, lane, j0);
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int jb = 0; jb < JW; ++jb) Ss[krow<E>(s, cg) + (16 * jb + rg) * SLD] = Sr[s][jb];
    }
    for (int64_t t = ntl - 1; t >= 0; --t) {
        const int ln = opaque(lane);
        const int lcg = ln >> 4, lrg = ln & 15;
        // per-lane byte offsets within a 16 x 4 (FP64) or 16 x 16 (FP32) block
        // of V and of Q (64-bit only for leading dimensions past 32-bit reach)
        using off_t = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
        const int cstep = MIXED ? 4 : 1;  // column distance of the lane groups
        const off_t lane_v = (off_t)(lrg + cstep * lcg * lda) * (off_t)sizeof(E);
        const off_t lane_q = (off_t)(lrg + cstep * lcg * ldq) * (off_t)sizeof(E);
        // FP64: only the last TAIL groups of four columns can reach past n;
        // there a column past n reads column n - 1 instead (then zeroed)
        constexpr int TAIL = (max_padding(NP) + 3) / 4;
        int64_t tail_off[TAIL];
#pragma unroll
        for (int j = 0; j < TAIL; ++j) {
            const int c = 4 * (KX - TAIL + j) + lcg;
            tail_off[j] = lrg + (int64_t)(c < n ? c : n - 1) * lda;
        }
        const E* T = Ttile + (leaf * f + t) * NT;
        const int64_t t0 = row0 + t * MT;
        const int64_t valid = MIXED ? MT : ((rows - t * MT) < MT ? (rows - t * MT) : MT);
        E Zr[KS][JW];
        if constexpr (PERW) {
            // one window at a time: the seed and its product never share the registers
#pragma unroll
            for (int jb = 0; jb < JW; ++jb) {
                E Z1[KS][1];
                seed_windows<NP, 1, E>(T, V, t0, lda, valid, n, t == 0, Ss, jb, Z1, lane);
#pragma unroll
                for (int s = 0; s < KS; ++s) Zr[s][jb] = Z1[s][0];
            }
        } else {
            seed_windows<NP, JW, E>(T, V, t0, lda, valid, n, t == 0, Ss, 0, Zr, lane);
        }
        if (t == 0) __builtin_amdgcn_wave_barrier();  // S_0 is read across lanes below
        // expansion Q_t = [S_0; 0] (t == 0 only) - V_t Z, 16 rows at a time
        const bool full = valid == MT;  // every row of the tile exists
#pragma unroll FQU
        for (int i = 0; i < RL; ++i) {
            const int rl = 16 * i + lrg;
            const bool rv = rl < valid;
            const E* vb = V + t0 + 16 * i;
            E y[KX];
            if (MIXED) {
                // whole padded tiles: column krow(k, q) of V
#pragma unroll
                for (int k = 0; k < KX; ++k) y[k] = ld_at(vb + (int64_t)(16 * (k / 4) + k % 4) * lda, lane_v);
            } else if (full) {
#pragma unroll
                for (int k = 0; k < KX - TAIL; ++k) y[k] = ld_at(vb + (int64_t)(4 * k) * lda, lane_v);
#pragma unroll
                for (int j = 0; j < TAIL; ++j) {
                    const int k = KX - TAIL + j;
                    const E v = vb[tail_off[j]];
                    y[k] = 4 * k + lcg < n ? v : E(0);
                }
            } else {
                // ragged tile or padded columns: clamp to an element that exists, then zero
                const int rc = rv ? rl : (int)valid - 1;
#pragma unroll
                for (int k = 0; k < KX; ++k) {
                    const int c = 4 * k + lcg, cc = c < n ? c : n - 1;
                    const E v = V[t0 + rc + (int64_t)cc * lda];
                    y[k] = (rv && c < n) ? v : E(0);
                }
            }
            if (t == 0) {
#pragma unroll
                for (int k = 0; k < KX; ++k) {
                    const int c = krow<E>(k, lcg);
                    if (rl < NP) y[k] = (rl > c) ? y[k] : (rl == c ? E(1) : E(0));
                }
            }
            E* qb = Q + t0 + 16 * i + (int64_t)(16 * j0) * ldq;
#pragma unroll
            for (int jb = 0; jb < JW; ++jb) {
                typename MM::acc_t acc = MM::zero();
#pragma unroll
                for (int k = 0; k < KX; ++k) acc = MM::mma(Zr[k][jb], y[k], acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int cl = 16 * jb + MM::out_row(lcg, r), c = 16 * j0 + cl;
                    E v = -acc[r];
                    if (t == 0 && rl < NP) v += Ss[rl + cl * SLD];
                    if (MIXED) {
                        // every row and column of the workspace is written; zero past n
                        st_at(qb + (int64_t)(16 * jb + r) * ldq, lane_q, c < n ? v : E(0));
                    } else if (c < n && (full || rv)) {
                        // the window spans round16(NP) columns: those at or past n are never stored
                        if constexpr (NTQ) st_nt(qb + (int64_t)(16 * jb + 4 * r) * ldq, lane_q, v);
                        else st_at(qb + (int64_t)(16 * jb + 4 * r) * ldq, lane_q, v);
                    }
                }
            }
        }
    }
}

// JWT: 16-column windows per wavefront.  A leaf split over several
// wavefronts (JWT < round16(NP) / 16) must not have Q alias V: every
// wavefront reads all of V's columns for the rows whose Q window it writes, so
// one wavefront's stores could overwrite reflectors another has yet to read.
// Aliased calls take JWT = round16(NP) / 16 (one wavefront per leaf).
template <int NP, bool WIDE, typename E = double, int JWT = fq_col_blocks<E>(NP)>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_form_q(const E* V, int64_t lda, int64_t m, int n, int64_t P,
                                                int64_t leaf_rows, int64_t f, const E* __restrict__ Ttile,
                                                const double* __restrict__ Sleaf, E* Q, int64_t ldq)
{
    constexpr int NPB = round16(NP), JW = JWT, SPLIT = NPB / 16 / JW;
    extern __shared__ double smem_d[];
    E* smem = reinterpret_cast<E*>(smem_d);
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    const int64_t leaf = gw / SPLIT;
    const int j0 = (int)(gw % SPLIT) * JW;
    if (leaf >= P) return;
    form_q_leaf<NP, WIDE, E, true, JW>(V, lda, m, n, P, leaf_rows, f, Ttile, Sleaf, Q, ldq, leaf, j0,
                                       smem + wave * fq_lds_elems<E>(NP, JW), lane);
}

// --------------------------------------------------------------------------
// Second pass of the mixed-precision path.  Q1 (FP32, whole tiles, NPB =
// round16(NP) columns, zero past n) is re-orthogonalised in FP64:
//   G = Q1^T Q1 (products of FP32 values are exact in FP64), ||G - I||_F as
//   the check of ||Q1^T Q1 - I||_F, G = R2^T R2 (Cholesky; Q1 is orthonormal
//   to FP32 accuracy, so G is within about 1e-6 of I and the factorisation
//   cannot break down), and when the check exceeds its bound
//   Q = Q1 R2^{-1}, R = R2 R1.
// --------------------------------------------------------------------------

// Partial Gram matrices: wavefront w sums rows [w rw, (w + 1) rw) (rw a
// multiple of 64) into the upper blocks of its NPB x NPB slot of Gp.  In k-step
// s of a 64-row group, lane (q, p) supplies row 16 q + s of columns 16 b + p:
// the 16 rows a lane needs are consecutive, four 16-byte loads per block.
template <int NP>
__device__ __forceinline__ void gram_q1_wave(const float* __restrict__ Q1, int64_t ldq1, int64_t rows_total,
                                             int64_t rw, int64_t w, double* __restrict__ Gp, int lane)
{
    constexpr int NPB = round16(NP), JB = NPB / 16;
    const int q = lane >> 4, p = lane & 15;
    dbl4 acc[JB][JB];
#pragma unroll
    for (int ib = 0; ib < JB; ++ib)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) acc[ib][jb] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int64_t r0 = w * rw, r1 = (r0 + rw) < rows_total ? (r0 + rw) : rows_total;
    for (int64_t g = r0; g < r1; g += 64) {
        float x[JB][16];
#pragma unroll
        for (int b = 0; b < JB; ++b) {
            const float* src = Q1 + g + 16 * q + (int64_t)(16 * b + p) * ldq1;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float4 t = *reinterpret_cast<const float4*>(src + 4 * v);
                x[b][4 * v] = t.x;
                x[b][4 * v + 1] = t.y;
                x[b][4 * v + 2] = t.z;
                x[b][4 * v + 3] = t.w;
            }
        }
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int ib = 0; ib < JB; ++ib)
#pragma unroll
                for (int jb = ib; jb < JB; ++jb)
                    acc[ib][jb] = mfma16x16x4((double)x[ib][s], (double)x[jb][s], acc[ib][jb]);
    }
    double* G = Gp + w * NPB * NPB;
#pragma unroll
    for (int ib = 0; ib < JB; ++ib)
#pragma unroll
        for (int jb = ib; jb < JB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) G[(16 * ib + q + 4 * r) + (16 * jb + p) * NPB] = acc[ib][jb][r];
}

template <int NP>
__global__ void __launch_bounds__(256) k_gram_q1(const float* __restrict__ Q1, int64_t ldq1, int64_t rows_total,
                                                 int64_t rw, int64_t nw, double* __restrict__ Gp)
{
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (w >= nw) return;
    gram_q1_wave<NP>(Q1, ldq1, rows_total, rw, w, Gp, lane);
}

// Sum of the partial Gram matrices in two stages, both pairwise, so that every
// entry carries O(log nw) rounding steps (the check it feeds is 1e-13).
// Stage 1: block (x, g) adds partials [64 g, 64 g + 64) of 256 entries (eight
// interleaved accumulators, combined as a tree) into Gq[g].
template <int NP>
__device__ __forceinline__ double gram_sum64_entry(const double* __restrict__ Gp, int64_t nw, int64_t g, int e)
{
    constexpr int NPB = round16(NP);
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int64_t w0 = 64 * g, wn = (nw - w0) < 64 ? (nw - w0) : 64;
    if (wn == 64) {
#pragma unroll
        for (int u = 0; u < 64; ++u) a[u % 8] += Gp[(w0 + u) * NPB * NPB + e];
    } else {
        for (int64_t u = 0; u < wn; ++u) a[u % 8] += Gp[(w0 + u) * NPB * NPB + e];
    }
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

template <int NP>
__global__ void __launch_bounds__(256) k_gram_sum64(const double* __restrict__ Gp, int64_t nw, double* __restrict__ Gq)
{
    constexpr int NPB = round16(NP);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t g = blockIdx.y;
    if (e >= NPB * NPB) return;
    Gq[g * NPB * NPB + e] = gram_sum64_entry<NP>(Gp, nw, g, e);
}

// Stage 2: one thread per entry merges the ng group sums as a binary counter.
template <int NP>
__device__ __forceinline__ double gram_sum_entry(const double* __restrict__ Gq, int64_t ng, int e)
{
    constexpr int NPB = round16(NP);
    double stack[32];
    int64_t cnt = 0;
    for (int64_t g = 0; g < ng; ++g) {
        double cs = Gq[g * NPB * NPB + e];
        int lvl = 0;
        for (int64_t c = cnt; c & 1; c >>= 1) cs = stack[lvl++] + cs;
        stack[lvl] = cs;
        ++cnt;
    }
    double sum = 0.0;
    for (int lvl = 0; cnt >> lvl; ++lvl)
        if ((cnt >> lvl) & 1) sum = stack[lvl] + sum;
    return sum;
}

template <int NP>
__global__ void __launch_bounds__(256) k_gram_sum(const double* __restrict__ Gq, int64_t ng, double* __restrict__ G)
{
    constexpr int NPB = round16(NP);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NPB * NPB) return;
    G[e] = gram_sum_entry<NP>(Gq, ng, e);
}

// One wavefront: the check ||G - I||_F, the flag, the Cholesky factor R2 of
// G, R2^{-1}, and R = R2 R1 for the caller (R1 the sign-normalised first-pass
// R; diag(R2) > 0 keeps diag(R) >= 0).  Below the bound: R2^{-1} = I, R = R1.
// Everything the serial loops touch sits in LDS (reorth_lds_doubles): G and
// then R2, R2^{-1} and R1, each NPB x (NPB + 1) with column j owned by lane j;
// the inputs are read and R2^{-1} (NPB x NPB, zero past n) written with
// coalesced accesses.
// sum over k in [k0, k1) of a[k * lda] * b[k], four partial sums (the serial
// loops of the factorisation below are bound by the latency of one chain)
__device__ __forceinline__ double lds_dot(const double* a, int lda, const double* b, int k0, int k1)
{
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int k = k0;
    for (; k + 3 < k1; k += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] = fma(a[(k + u) * lda], b[k + u], s[u]);
    }
    for (; k < k1; ++k) s[0] = fma(a[k * lda], b[k], s[0]);
    return (s[0] + s[1]) + (s[2] + s[3]);
}

template <int NP>
__host__ __device__ constexpr int reorth_lds_doubles() { return 3 * round16(NP) * (round16(NP) + 1); }

template <int NP>
__device__ __forceinline__ void reorth_factor_body(const double* __restrict__ G, const double* __restrict__ R1,
                                                   int n, double bound, double* __restrict__ Xs,
                                                   double* __restrict__ info, double* __restrict__ R, int64_t ldr,
                                                   double* Gs, int lane)
{
    constexpr int NPB = round16(NP), LD = NPB + 1;
    double* Xl = Gs + NPB * LD;  // R2^{-1}
    double* Rl = Xl + NPB * LD;  // R1
    // symmetric G from its upper triangle, and R1; ||G - I||_F over the n x n block
    double dev = 0.0;
    for (int e = lane; e < NPB * NPB; e += 64) {
        const int i = e % NPB, j = e / NPB;
        if (i <= j) {
            const double g = G[e];
            Gs[i + j * LD] = g;
            Gs[j + i * LD] = g;
            if (j < n) {
                const double d = g - (i == j ? 1.0 : 0.0);
                dev = fma((i == j ? 1.0 : 2.0) * d, d, dev);
            }
        }
    }
    for (int e = lane; e < NP * NP; e += 64) Rl[e % NP + (e / NP) * LD] = R1[e];
    for (int off = 32; off >= 1; off >>= 1) dev += __shfl_xor(dev, off);
    const double orth = sqrt(dev);
    const bool apply = orth > bound;
    __syncthreads();
    if (apply) {
        // right-looking Cholesky G = R2^T R2, R2 upper, overwriting the upper triangle of Gs
        for (int k = 0; k < n; ++k) {
            const double d = sqrt(Gs[k + k * LD]);
            __syncthreads();
            for (int j = lane; j < n; j += 64) {
                if (j > k) Gs[k + j * LD] /= d;
                if (j == k) Gs[k + k * LD] = d;
            }
            __syncthreads();
            for (int j = lane; j < n; j += 64)
                if (j > k) {
                    // rows k + 1 .. j of column j; row k is only read, so four
                    // updates at a time load before they store
                    const double rkj = Gs[k + j * LD];
                    int i = k + 1;
                    for (; i + 3 <= j; i += 4) {
                        double a[4], g[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            a[u] = Gs[k + (i + u) * LD];
                            g[u] = Gs[i + u + j * LD];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) Gs[i + u + j * LD] = fma(-a[u], rkj, g[u]);
                    }
                    for (; i <= j; ++i) Gs[i + j * LD] = fma(-Gs[k + i * LD], rkj, Gs[i + j * LD]);
                }
            __syncthreads();
        }
        // column j of R2^{-1} by back substitution (the lane reads back only its own writes)
        for (int j = lane; j < NPB; j += 64) {
            for (int i = 0; i < NPB; ++i) Xl[i + j * LD] = 0.0;
            if (j < n) {
                Xl[j + j * LD] = 1.0 / Gs[j + j * LD];
                for (int i = j - 1; i >= 0; --i) {
                    const double acc = lds_dot(Gs + i, LD, Xl + j * LD, i + 1, j + 1);
                    Xl[i + j * LD] = -acc / Gs[i + i * LD];
                }
            }
        }
    } else {
        for (int j = lane; j < NPB; j += 64)
            for (int i = 0; i < NPB; ++i) {
                Xl[i + j * LD] = (i == j && j < n) ? 1.0 : 0.0;
                Gs[i + j * LD] = (i == j) ? 1.0 : 0.0;
            }
    }
    __syncthreads();
    for (int e = lane; e < NPB * NPB; e += 64) Xs[e] = Xl[e % NPB + (e / NPB) * LD];
    // R = R2 R1 (upper times upper), column j by lane j
    for (int j = lane; j < n; j += 64)
        for (int i = 0; i < n; ++i) {
            R[i + j * ldr] = i <= j ? lds_dot(Gs + i, LD, Rl + j * LD, i, j + 1) : 0.0;
        }
    if (lane == 0) {
        info[0] = orth;
        info[1] = apply ? 1.0 : 0.0;
    }
}

template <int NP>
__global__ void __launch_bounds__(64) k_reorth_factor(const double* __restrict__ G, const double* __restrict__ R1,
                                                      int n, double bound, double* __restrict__ Xs,
                                                      double* __restrict__ info, double* __restrict__ R, int64_t ldr)
{
    extern __shared__ double smem[];  // reorth_lds_doubles<NP>()
    reorth_factor_body<NP>(G, R1, n, bound, Xs, info, R, ldr, smem, threadIdx.x);
}

// Q = Q1 R2^{-1} in FP64 (R2^{-1} = I when the check passed), 16 rows at a
// time: D = R2^{-T} Q1^T on the matrix cores, so that a lane's outputs are 16
// consecutive rows of one column of Q.  R2^{-1} is upper triangular: output
// block ob needs k < 16 (ob + 1) only.
// Row blocks rb = rb0, rb0 + step, ... below rb1 of one problem.
// E: the element type of Q1 (float in the mixed path; double for the
// CholeskyQR comparison kernels, which form Q = A R^{-1} the same way).  Each
// 16-row block is read whole before any of its outputs is stored, so Q may be
// Q1 itself (FP64).
template <int NP, typename E = float>
__device__ __forceinline__ void reorth_q_blocks(const E* __restrict__ Q1, int64_t ldq1, int64_t m, int n,
                                                const double* __restrict__ R2inv, double* __restrict__ Q,
                                                int64_t ldq, int64_t rb0, int64_t rb1, int64_t step, int lane)
{
    constexpr int NPB = round16(NP), JB = NPB / 16, KS = NPB / 4;
    const int q = lane >> 4, p = lane & 15;
    // A operands R2^{-T}(16 ob + p, 4 s + q) = R2^{-1}(4 s + q, 16 ob + p), kept for the whole run
    double ra[JB][KS];
#pragma unroll
    for (int ob = 0; ob < JB; ++ob)
#pragma unroll
        for (int s = 0; s < KS; ++s) ra[ob][s] = (s < 4 * (ob + 1)) ? R2inv[(4 * s + q) + (16 * ob + p) * NPB] : 0.0;
    for (int64_t rb = rb0; rb < rb1; rb += step) {
        const int64_t row = 16 * rb + p;
        double x[KS];
        if constexpr (sizeof(E) == 4) {
            // the mixed workspace: whole tiles and round16 columns, zero-padded
#pragma unroll
            for (int s = 0; s < KS; ++s) x[s] = (double)Q1[row + (int64_t)(4 * s + q) * ldq1];
        } else {
            // a caller's m x n matrix: rows past m and columns past n read an
            // element that exists, then count as zero
            const int64_t rc = row < m ? row : m - 1;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int c = 4 * s + q, cc = c < n ? c : n - 1;
                const double v = (double)Q1[rc + (int64_t)cc * ldq1];
                x[s] = (row < m && c < n) ? v : 0.0;
            }
        }
#pragma unroll
        for (int ob = 0; ob < JB; ++ob) {
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4 * (ob + 1) && s < KS; ++s) acc = mfma16x16x4(ra[ob][s], x[s], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = 16 * ob + q + 4 * r;
                if (row < m && c < n) Q[row + (int64_t)c * ldq] = acc[r];
            }
        }
    }
}

template <int NP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_reorth_q(const float* __restrict__ Q1, int64_t ldq1, int64_t m, int n,
                                                  const double* __restrict__ R2inv, double* __restrict__ Q,
                                                  int64_t ldq, int64_t nblocks)
{
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    reorth_q_blocks<NP>(Q1, ldq1, m, n, R2inv, Q, ldq, (int64_t)blockIdx.x * (blockDim.x >> 6) + wave, nblocks, nwaves,
                        lane);
}

// --------------------------------------------------------------------------
// Q^T B, the reduction of Sec. 4.1, for up to kApplyCols right-hand sides per
// launch.  An NP x kApplyCols block X (C, W, D) lives in registers as
// Xr[s][jb] = X(4s + q, 16jb + p) with q = lane / 16, p = lane % 16: the
// B-operand layout of the f64 16x16x4 op, in which products with T^T and Y1
// come back.
// --------------------------------------------------------------------------
constexpr int kApplyCols = 32;

// X = T^T D, T packed upper triangular (T^T(r, c) = T(c, r), c <= r).
template <int NP>
__device__ __forceinline__ void trit_times_regs(const double* __restrict__ T,
                                                const double (&Dr)[round16(NP) / 4][kApplyCols / 16],
                                                double (&Xr)[round16(NP) / 4][kApplyCols / 16], int lane)
{
    constexpr int NPB = round16(NP), JB = NPB / 16, KS = NPB / 4, JK = kApplyCols / 16;
    const int q = lane >> 4, p = lane & 15;
#pragma unroll
    for (int ib = 0; ib < JB; ++ib) {
        double tv[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int r = 16 * ib + p, c = 4 * s + q;  // A(r, c) = T(c, r)
            tv[s] = (c <= r && r < NP) ? T[r * (r + 1) / 2 + c] : 0.0;
        }
#pragma unroll
        for (int jb = 0; jb < JK; ++jb) {
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < KS; ++s) acc = mfma16x16x4(tv[s], Dr[s][jb], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) Xr[4 * ib + r][jb] = acc[r];
        }
    }
}

// Leaf chain: tile 0 B_0 <- B_0 - V_0 T_0^T V_0^T B_0 and C = its top NP rows;
// tile k > 0: D = C + Y_k^T B_k, X = T_k^T D, C <- C - X, B_k <- B_k - Y_k X.
// C goes back to the leaf's top rows at the end.  W = Y^T B contracts over
// rows, so Y and B are read with rows on the lane-group index for it; the
// update reads Y with rows on the lanes of a group (the layout of the leaf
// kernel), which makes B^T - X^T Y^T land in B's own coalesced layout.
template <int NP>
__global__ void __launch_bounds__(256) k_apply_leaf(const double* __restrict__ V, int64_t lda, double* B,
                                                    int64_t ldb, int64_t k, int64_t m, int n, int64_t P,
                                                    int64_t leaf_rows, int64_t f, const double* __restrict__ Ttile)
{
    constexpr int MT = tile_rows_for(NP), NPB = round16(NP), JB = NPB / 16, KS = NPB / 4;
    constexpr int JK = kApplyCols / 16, KC4 = NP / 4, NT = packed_size(NP);
    extern __shared__ double smem[];
    // blockIdx.y picks the chunk of kApplyCols columns of B
    const int64_t c0 = (int64_t)blockIdx.y * kApplyCols;
    const int kc = (int)((k - c0) < kApplyCols ? (k - c0) : kApplyCols);
    B += c0 * ldb;
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int q = lane >> 4, p = lane & 15;
    const int64_t leaf = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (leaf >= P) return;
    double* cbuf = smem + wave * NP * kApplyCols;  // top NP rows of the updated tile 0

    const int64_t row0 = leaf * leaf_rows;
    const int64_t rows = (leaf == P - 1) ? (m - row0) : leaf_rows;
    const int64_t ntl = (rows + MT - 1) / MT;
    double Cr[KS][JK];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int jb = 0; jb < JK; ++jb) Cr[s][jb] = 0.0;
    for (int64_t t = 0; t < ntl; ++t) {
        const int64_t t0 = row0 + t * MT;
        const int64_t valid = (rows - t * MT) < MT ? (rows - t * MT) : MT;
        const bool first = t == 0;
        // W = Y^T B_t
        dbl4 wacc[JB][JK];
#pragma unroll
        for (int ib = 0; ib < JB; ++ib)
#pragma unroll
            for (int jb = 0; jb < JK; ++jb) wacc[ib][jb] = dbl4{0.0, 0.0, 0.0, 0.0};
        // 16 rows per block: lane group q takes rows 4q .. 4q + 3 of the block, so a
        // column's 16 rows (one 128-byte line) are requested together; the
        // contraction over rows takes them in this order
#pragma unroll 1
        for (int s = 0; s < MT / 16; ++s) {
            double yv[4][JB], bv[4][JK];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int r = 16 * s + 4 * q + u;
                const bool rv = r < valid;
#pragma unroll
                for (int b = 0; b < JB; ++b) {
                    const int c = 16 * b + p;
                    double y = (rv && c < n) ? V[t0 + r + (int64_t)c * lda] : 0.0;
                    if (first) y = c < NP ? (r > c ? y : (r == c ? 1.0 : 0.0)) : 0.0;
                    yv[u][b] = y;
                }
#pragma unroll
                for (int jb = 0; jb < JK; ++jb) {
                    const int c = 16 * jb + p;
                    bv[u][jb] = (rv && c < kc) ? B[t0 + r + (int64_t)c * ldb] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int ib = 0; ib < JB; ++ib)
#pragma unroll
                    for (int jb = 0; jb < JK; ++jb) wacc[ib][jb] = mfma16x16x4(yv[u][ib], bv[u][jb], wacc[ib][jb]);
        }
        double Dr[KS][JK], Xr[KS][JK];
#pragma unroll
        for (int ib = 0; ib < JB; ++ib)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int jb = 0; jb < JK; ++jb)
                    Dr[4 * ib + r][jb] = (first ? 0.0 : Cr[4 * ib + r][jb]) + wacc[ib][jb][r];
        trit_times_regs<NP>(Ttile + (leaf * f + t) * NT, Dr, Xr, lane);
        if (!first) {
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int jb = 0; jb < JK; ++jb) Cr[s][jb] -= Xr[s][jb];
        }
        // B_t <- B_t - Y X, 16 rows at a time (B^T - X^T Y^T on the matrix cores)
#pragma unroll 2
        for (int i = 0; i < MT / 16; ++i) {
            const int rl = 16 * i + p;
            const bool rv = rl < valid;
            const int64_t row = t0 + rl;
            double y[KC4];
#pragma unroll
            for (int s = 0; s < KC4; ++s) {
                const int c = 4 * s + q;
                double v = (rv && c < n) ? V[row + (int64_t)c * lda] : 0.0;
                if (first && rl < NP) v = rl > c ? v : (rl == c ? 1.0 : 0.0);
                y[s] = v;
            }
#pragma unroll
            for (int jb = 0; jb < JK; ++jb) {
                dbl4 acc;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = 16 * jb + q + 4 * r;
                    acc[r] = (rv && c < kc) ? B[row + (int64_t)c * ldb] : 0.0;
                }
#pragma unroll
                for (int s = 0; s < KC4; ++s) acc = mfma16x16x4(-Xr[s][jb], y[s], acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = 16 * jb + q + 4 * r;
                    if (rv && c < kc) B[row + (int64_t)c * ldb] = acc[r];
                    if (first && rl < NP) cbuf[rl * kApplyCols + c] = acc[r];
                }
            }
        }
        if (first) {
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int jb = 0; jb < JK; ++jb) {
                    const int r = 4 * s + q, c = 16 * jb + p;
                    Cr[s][jb] = r < NP ? cbuf[r * kApplyCols + c] : 0.0;
                }
            __builtin_amdgcn_wave_barrier();
        }
    }
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int jb = 0; jb < JK; ++jb) {
            const int r = 4 * s + q, c = 16 * jb + p;
            if (r < NP && r < rows && c < kc) B[row0 + r + (int64_t)c * ldb] = Cr[s][jb];
        }
}

// One tree level of Q^T B: node q stacks the tops C_a (first leaf of its top
// child) and C_b (first leaf of its bottom child): D = C_a + Y1^T C_b,
// X = T^T D, C_a <- C_a - X, C_b <- C_b - Y1 X.
template <int NP>
__global__ void __launch_bounds__(256) k_apply_tree(double* B, int64_t ldb, int64_t k, int64_t leaf_rows,
                                                    int64_t span, const double* __restrict__ Ynode,
                                                    const double* __restrict__ Tnode, int64_t cin, int64_t cout)
{
    constexpr int NPB = round16(NP), JB = NPB / 16, KS = NPB / 4, JK = kApplyCols / 16, NT = packed_size(NP);
    // blockIdx.y picks the chunk of kApplyCols columns of B
    const int64_t c0 = (int64_t)blockIdx.y * kApplyCols;
    const int kc = (int)((k - c0) < kApplyCols ? (k - c0) : kApplyCols);
    B += c0 * ldb;
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int q = lane >> 4, p = lane & 15;
    const int64_t nq = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (nq >= cout) return;
    const int64_t ia = 2 * nq, ib = 2 * nq + 1;
    if (ib >= cin) return;  // passes up unchanged
    double* Ba = B + ia * span * leaf_rows;
    double* Bb = B + ib * span * leaf_rows;
    double Car[KS][JK], Cbr[KS][JK], Dr[KS][JK], Xr[KS][JK];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int jb = 0; jb < JK; ++jb) {
            const int r = 4 * s + q, c = 16 * jb + p;
            const bool v = r < NP && c < kc;
            Car[s][jb] = v ? Ba[r + (int64_t)c * ldb] : 0.0;
            Cbr[s][jb] = v ? Bb[r + (int64_t)c * ldb] : 0.0;
        }
    const double* Y = Ynode + nq * NP * NP;
    // D = C_a + Y1^T C_b
#pragma unroll
    for (int ibk = 0; ibk < JB; ++ibk) {
        double yt[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int r = 4 * s + q, kk = 16 * ibk + p;  // A(kk, r) = Y1(r, kk)
            yt[s] = (r < NP && kk < NP) ? Y[r + kk * NP] : 0.0;
        }
#pragma unroll
        for (int jb = 0; jb < JK; ++jb) {
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < KS; ++s) acc = mfma16x16x4(yt[s], Cbr[s][jb], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) Dr[4 * ibk + r][jb] = Car[4 * ibk + r][jb] + acc[r];
        }
    }
    trit_times_regs<NP>(Tnode + nq * NT, Dr, Xr, lane);
    // C_b -= Y1 X
#pragma unroll
    for (int ibk = 0; ibk < JB; ++ibk) {
        double yv[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int r = 16 * ibk + p, kk = 4 * s + q;
            yv[s] = (r < NP && kk < NP) ? Y[r + kk * NP] : 0.0;
        }
#pragma unroll
        for (int jb = 0; jb < JK; ++jb) {
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < KS; ++s) acc = mfma16x16x4(yv[s], Xr[s][jb], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) Cbr[4 * ibk + r][jb] -= acc[r];
        }
    }
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int jb = 0; jb < JK; ++jb) {
            const int r = 4 * s + q, c = 16 * jb + p;
            if (r < NP && c < kc) {
                Ba[r + (int64_t)c * ldb] = Car[s][jb] - Xr[s][jb];
                Bb[r + (int64_t)c * ldb] = Cbr[s][jb];
            }
        }
}

// Root of Q^T B: rows 0..n-1 <- D rows 0..n-1.
template <int NP>
__global__ void __launch_bounds__(256) k_apply_signs(double* B, int64_t ldb, int n, int64_t k,
                                                     const double* __restrict__ Dsig)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * k) return;
    const int r = (int)(idx % n);
    const int64_t c = idx / n;
    B[r + c * ldb] *= Dsig[r];
}

template <typename K>
void allow_lds(K kernel, size_t bytes)
{
    if (bytes > 64 * 1024)
        hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bytes);
}

inline unsigned grid_for(int64_t items, int waves) { return (unsigned)((items + waves - 1) / waves); }

template <int NP>
hipError_t leaf_factor_np(const Layout& L, const double* A, int64_t lda, double* V, int64_t ldv, double* ws,
                          bool want_q, hipStream_t s)
{
    constexpr int MT = tile_rows_for(NP);
    const size_t lds = (size_t)L.waves * leaf_lds_doubles(NP, MT, want_q) * sizeof(double);
    const dim3 grid(grid_for(L.P, L.waves)), block(64 * L.waves);
    if (want_q && L.rec) {
        if constexpr (leaf_rec_ok(NP)) {
            const size_t lds_r = (size_t)L.waves * leaf_kernel_lds_doubles(NP, true, true) * sizeof(double);
            allow_lds(k_leaf_factor<NP, true, double, true>, lds_r);
            hipLaunchKernelGGL((k_leaf_factor<NP, true, double, true>), grid, block, lds_r, s, A, lda, V, ldv, L.m,
                               (int)L.n, L.P, L.leaf_rows, L.f, ws + L.off_T, ws + L.off_R[0]);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (want_q) {
        allow_lds(k_leaf_factor<NP, true>, lds);
        hipLaunchKernelGGL((k_leaf_factor<NP, true>), grid, block, lds, s, A, lda, V, ldv, L.m, (int)L.n, L.P,
                           L.leaf_rows, L.f, ws + L.off_T, ws + L.off_R[0]);
    } else {
        allow_lds(k_leaf_factor<NP, false>, lds);
        hipLaunchKernelGGL((k_leaf_factor<NP, false>), grid, block, lds, s, A, lda, V, ldv, L.m, (int)L.n, L.P,
                           L.leaf_rows, L.f, ws + L.off_T, ws + L.off_R[0]);
    }
    return hipGetLastError();
}

// T of every leaf tile from what the leaf kernel left in its slot (FP32 slots
// for the mixed path).
template <int NP>
hipError_t build_T_np(const Layout& L, double* ws, hipStream_t s)
{
    // FP64 above 48 columns: single-wavefront workgroups (7 fit a CU's LDS
    // instead of one 4-wavefront group).  The T kernel gets 1.6x faster and the
    // tree beside it slower; the step gained about 1% at n = 64.  The FP32 slots
    // and narrower widths measured better with 4-wavefront groups.
    constexpr int waves = 4, waves_d = NP > 48 ? 1 : 4;
    if (L.mixed) {
        const size_t lds = (size_t)waves * BuildTLds<NP>::WS * sizeof(double);
        allow_lds(k_build_T<NP, float>, lds);
        hipLaunchKernelGGL((k_build_T<NP, float>), dim3(grid_for(L.ntiles, waves)), dim3(64 * waves), lds, s,
                           reinterpret_cast<float*>(ws + L.off_T32), L.ntiles);
    } else {
        const size_t lds = (size_t)waves_d * BuildTLds<NP>::WS * sizeof(double);
        allow_lds(k_build_T<NP, double>, lds);
        hipLaunchKernelGGL((k_build_T<NP, double>), dim3(grid_for(L.ntiles, waves_d)), dim3(64 * waves_d), lds, s,
                           ws + L.off_T, L.ntiles);
    }
    return hipGetLastError();
}

// T in `count` consecutive FP64 slots holding tau and the Gram entries.
template <int NP>
hipError_t build_T_slots(double* slots, int64_t count, hipStream_t s)
{
    constexpr int waves = NP > 48 ? 1 : 4;
    const size_t lds = (size_t)waves * BuildTLds<NP>::WS * sizeof(double);
    allow_lds(k_build_T<NP, double>, lds);
    hipLaunchKernelGGL((k_build_T<NP, double>), dim3(grid_for(count, waves)), dim3(64 * waves), lds, s, slots, count);
    return hipGetLastError();
}

template <int NP>
hipError_t tree_np(const Layout& L, double* ws, bool want_q, hipStream_t s)
{
    constexpr int MTN = round16(NP);
    const int waves = NP <= 32 ? 4 : 2;  // per-wave LDS grows as NP^2
    const size_t lds = (size_t)waves * factor_lds_doubles(NP, MTN, want_q) * sizeof(double);
    for (int l = 1; l <= L.levels; ++l) {
        const dim3 grid(grid_for(L.count[l], waves)), block(64 * waves);
        if (want_q) {
            allow_lds(k_tree_level<NP, true>, lds);
            hipLaunchKernelGGL((k_tree_level<NP, true>), grid, block, lds, s, ws + L.off_R[l - 1], L.count[l - 1],
                               ws + L.off_R[l], ws + L.off_Y[l], ws + L.off_TN[l], L.count[l]);
        } else {
            allow_lds(k_tree_level<NP, false>, lds);
            hipLaunchKernelGGL((k_tree_level<NP, false>), grid, block, lds, s, ws + L.off_R[l - 1],
                               L.count[l - 1], ws + L.off_R[l], ws + L.off_Y[l], ws + L.off_TN[l], L.count[l]);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // T of every tree node (the seeds and Q^T B need them, the root does not)
    if (want_q && L.tree_nodes > 0) return build_T_slots<NP>(ws + L.off_TN[1], L.tree_nodes, s);
    return hipSuccess;
}

template <int NP>
hipError_t root_np(const Layout& L, double* ws, double* R, int64_t ldr, hipStream_t s)
{
    hipLaunchKernelGGL((k_root<NP>), dim3(1), dim3(64), 0, s, ws + L.off_R[L.levels], (int)L.n, R, ldr,
                       ws + L.off_D, ws + L.off_S[L.levels]);
    return hipGetLastError();
}

template <int NP>
hipError_t seeds_np(const Layout& L, double* ws, hipStream_t s)
{
    const int waves = 4;
    for (int l = L.levels; l >= 1; --l) {
        const dim3 grid(grid_for(L.count[l], waves)), block(64 * waves);
        hipLaunchKernelGGL((k_seed_level<NP>), grid, block, 0, s, ws + L.off_S[l], ws + L.off_Y[l],
                           ws + L.off_TN[l], L.count[l - 1], ws + L.off_S[l - 1], L.count[l]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int NP, int JW>
hipError_t form_q_launch(const Layout& L, const double* A, int64_t lda, double* ws, double* Q, int64_t ldq,
                         hipStream_t s)
{
    constexpr int NPB = round16(NP), SPLIT = NPB / 16 / JW;
    const size_t lds = (size_t)L.waves * fq_lds_elems<double>(NP, JW) * sizeof(double);
    const dim3 grid(grid_for(L.P * SPLIT, L.waves)), block(64 * L.waves);
    if (lane_offsets_fit_32(lda) && lane_offsets_fit_32(ldq)) {
        allow_lds(k_form_q<NP, false, double, JW>, lds);
        hipLaunchKernelGGL((k_form_q<NP, false, double, JW>), grid, block, lds, s, A, lda, L.m, (int)L.n, L.P,
                           L.leaf_rows, L.f, ws + L.off_T, ws + L.off_S[0], Q, ldq);
    } else {
        allow_lds(k_form_q<NP, true, double, JW>, lds);
        hipLaunchKernelGGL((k_form_q<NP, true, double, JW>), grid, block, lds, s, A, lda, L.m, (int)L.n, L.P,
                           L.leaf_rows, L.f, ws + L.off_T, ws + L.off_S[0], Q, ldq);
    }
    return hipGetLastError();
}

template <int NP>
hipError_t form_q_np(const Layout& L, const double* A, int64_t lda, double* ws, double* Q, int64_t ldq,
                     hipStream_t s)
{
    constexpr int NPB = round16(NP), JB = NPB / 16, JW = fq_col_blocks<double>(NP);
    // Q over V: one wavefront per leaf (see k_form_q)
    if ((const double*)Q == A && JW < JB) return form_q_launch<NP, JB>(L, A, lda, ws, Q, ldq, s);
    return form_q_launch<NP, JW>(L, A, lda, ws, Q, ldq, s);
}

template <int NP>
hipError_t apply_qt_np(const Layout& L, const double* A, int64_t lda, int64_t k, double* B, int64_t ldb, double* ws,
                       hipStream_t s)
{
    const size_t lds = (size_t)L.waves * NP * kApplyCols * sizeof(double);
    allow_lds(k_apply_leaf<NP>, lds);
    // every chunk of kApplyCols columns in the same launches (grid y), at most
    // kMaxChunks chunks per launch
    constexpr int64_t kMaxChunks = 65535;
    const int64_t nch = (k + kApplyCols - 1) / kApplyCols;
    for (int64_t g0 = 0; g0 < nch; g0 += kMaxChunks) {
        const int64_t ng = (nch - g0) < kMaxChunks ? (nch - g0) : kMaxChunks;
        const int64_t kg = (k - g0 * kApplyCols) < ng * kApplyCols ? (k - g0 * kApplyCols) : ng * kApplyCols;
        double* Bg = B + g0 * kApplyCols * ldb;
        hipLaunchKernelGGL((k_apply_leaf<NP>), dim3(grid_for(L.P, L.waves), (unsigned)ng), dim3(64 * L.waves), lds, s,
                           A, lda, Bg, ldb, kg, L.m, (int)L.n, L.P, L.leaf_rows, L.f, ws + L.off_T);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        int64_t span = 1;
        for (int l = 1; l <= L.levels; ++l) {
            hipLaunchKernelGGL((k_apply_tree<NP>), dim3(grid_for(L.count[l], 4), (unsigned)ng), dim3(256), 0, s, Bg,
                               ldb, kg, L.leaf_rows, span, ws + L.off_Y[l], ws + L.off_TN[l], L.count[l - 1],
                               L.count[l]);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            span *= 2;
        }
        const int64_t cnt = L.n * kg;
        hipLaunchKernelGGL((k_apply_signs<NP>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, Bg, ldb,
                           (int)L.n, kg, ws + L.off_D);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---- batched problems ------------------------------------------------------
// Persistent grids: every wavefront walks a device work list (grid stride), so
// one launch covers the leaves (or the nodes of one tree level) of every
// problem of a width class.  The per-item work is that of the single-problem
// kernels.

template <int NP, bool WANT_Q>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_leaf_batch(const BatchProblem* __restrict__ probs,
                                                    const BatchArgs* __restrict__ args, double* ws,
                                                    const int64_t* __restrict__ items, int64_t nitems)
{
    constexpr int WS = leaf_lds_doubles<double>(NP, tile_rows_for(NP), WANT_Q);
    extern __shared__ double smem[];
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems; it += nw) {
        const int64_t item = items[it];
        const int64_t p = item >> 32, leaf = item & 0xffffffff;
        const BatchProblem& B = probs[p];
        const BatchArgs X = args[p];
        double* w = ws + B.ws_off;
        leaf_chain<NP, WANT_Q, double>(X.A, X.lda, X.A, X.lda, B.m, B.n, B.P, B.leaf_rows, B.f, w + B.off_T,
                                       w + B.off_R[0], leaf, smem + wave * WS, lane);
        __builtin_amdgcn_wave_barrier();  // the next item rewrites this wave's LDS
    }
}

// T of every tile of every leaf item (the tiles of one leaf on one wavefront),
// from what k_leaf_batch left in the slots; the arithmetic of k_build_T.
template <int NP>
__global__ void __launch_bounds__(256) k_build_T_batch(const BatchProblem* __restrict__ probs, double* ws,
                                                       const int64_t* __restrict__ items, int64_t nitems)
{
    constexpr int MT = tile_rows_for(NP), NT = packed_size(NP);
    extern __shared__ double smem[];
    const int wave = wave_index(), lane = threadIdx.x & 63;
    double* W = smem + wave * BuildTLds<NP>::WS;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems; it += nw) {
        const int64_t item = items[it];
        const int64_t p = item >> 32, leaf = item & 0xffffffff;
        const BatchProblem& B = probs[p];
        const int64_t row0 = leaf * B.leaf_rows;
        const int64_t rows = (leaf == B.P - 1) ? (B.m - row0) : B.leaf_rows;
        const int64_t ntl = (rows + MT - 1) / MT;
        double* T = ws + B.ws_off + B.off_T + leaf * B.f * NT;
        for (int64_t t = 0; t < ntl; ++t) build_T_slot<NP, double>(T + t * NT, W, lane);
    }
}

template <int NP, bool WANT_Q>
__global__ void __launch_bounds__(256) k_tree_batch(const BatchProblem* __restrict__ probs, double* ws,
                                                    const int64_t* __restrict__ items, int64_t nitems, int l)
{
    constexpr int WS = factor_lds_doubles<double>(NP, round16(NP), WANT_Q);
    extern __shared__ double smem[];
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems; it += nw) {
        const int64_t item = items[it];
        const int64_t p = item >> 32, q = item & 0xffffffff;
        const BatchProblem& B = probs[p];
        double* w = ws + B.ws_off;
        tree_node<NP, WANT_Q>(w + B.off_R[l - 1], B.count[l - 1], w + B.off_R[l], w + B.off_Y[l], w + B.off_TN[l],
                              q, smem + wave * WS, lane);
        __builtin_amdgcn_wave_barrier();
    }
}

template <int NP>
__global__ void __launch_bounds__(256) k_root_batch(const BatchProblem* __restrict__ probs,
                                                    const BatchArgs* __restrict__ args, double* ws,
                                                    const int64_t* __restrict__ items, int64_t nitems, int want_q)
{
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems; it += nw) {
        const int64_t p = items[it] >> 32;
        const BatchProblem& B = probs[p];
        const BatchArgs X = args[p];
        double* w = ws + B.ws_off;
        root_body<NP>(w + B.off_R[B.levels], B.n, X.X, X.ldx, w + B.off_D, want_q ? w + B.off_S[B.levels] : nullptr,
                      lane);
    }
}

template <int NP>
__global__ void __launch_bounds__(256) k_seed_batch(const BatchProblem* __restrict__ probs, double* ws,
                                                    const int64_t* __restrict__ items, int64_t nitems, int l)
{
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems; it += nw) {
        const int64_t item = items[it];
        const int64_t p = item >> 32, q = item & 0xffffffff;
        const BatchProblem& B = probs[p];
        double* w = ws + B.ws_off;
        seed_node<NP>(w + B.off_S[l], w + B.off_Y[l], w + B.off_TN[l], B.count[l - 1], w + B.off_S[l - 1], q, lane);
    }
}

// JWT as for k_form_q: the graph of calls with some Q[i] aliasing A[i] takes
// one wavefront per leaf.
template <int NP, int JWT = fq_col_blocks<double>(NP)>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_form_q_batch(const BatchProblem* __restrict__ probs,
                                                    const BatchArgs* __restrict__ args, double* ws,
                                                    const int64_t* __restrict__ items, int64_t nitems)
{
    constexpr int NPB = round16(NP), JW = JWT, SPLIT = NPB / 16 / JW;
    extern __shared__ double smem[];
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems * SPLIT; it += nw) {
        const int64_t item = items[it / SPLIT];
        const int j0 = (int)(it % SPLIT) * JW;
        const int64_t p = item >> 32, leaf = item & 0xffffffff;
        const BatchProblem& B = probs[p];
        const BatchArgs X = args[p];
        double* w = ws + B.ws_off;
        form_q_leaf<NP, true, double, false, JW>(X.A, X.lda, B.m, B.n, B.P, B.leaf_rows, B.f, w + B.off_T,
                                                 w + B.off_S[0], X.X, X.ldx, leaf, j0,
                                                 smem + wave * fq_lds_elems<double>(NP, JW), lane);
        __builtin_amdgcn_wave_barrier();
    }
}

// T of the tree nodes of level l from the tau and Gram entries tree_node left
// in their slots (the arithmetic of k_build_T); one wavefront per (problem,
// node) item.  A pass-through node's slot holds nothing of use and its T is
// never read.
template <int NP>
__global__ void __launch_bounds__(256) k_build_T_nodes_batch(const BatchProblem* __restrict__ probs, double* ws,
                                                             const int64_t* __restrict__ items, int64_t nitems,
                                                             int l)
{
    constexpr int NT = packed_size(NP);
    extern __shared__ double smem[];
    const int wave = wave_index(), lane = threadIdx.x & 63;
    double* W = smem + wave * BuildTLds<NP>::WS;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems; it += nw) {
        const int64_t item = items[it];
        const int64_t p = item >> 32, q = item & 0xffffffff;
        const BatchProblem& B = probs[p];
        build_T_slot<NP, double>(ws + B.ws_off + B.off_TN[l] + q * NT, W, lane);
    }
}

// Grid of a persistent batched launch: enough waves to fill the device at two
// per SIMD, never more than there are items.
inline unsigned batch_grid(int64_t items, int waves)
{
    const int64_t cap = 256 * 8 / waves;  // 256 CUs, 8 waves each
    const int64_t need = (items + waves - 1) / waves;
    return (unsigned)(need < cap ? (need > 0 ? need : 1) : cap);
}

// T of every tree node of every problem of a class, level by level.
template <int NP>
hipError_t batch_node_T(const BatchClass& C, const BatchProblem* probs, double* ws, hipStream_t s)
{
    constexpr int waves = 4;
    const size_t lds = (size_t)waves * BuildTLds<NP>::WS * sizeof(double);
    allow_lds(k_build_T_nodes_batch<NP>, lds);
    for (int l = 1; l <= C.max_levels; ++l) {
        hipLaunchKernelGGL((k_build_T_nodes_batch<NP>), dim3(batch_grid(C.n_level[l], waves)), dim3(64 * waves), lds,
                           s, probs, ws, C.level_items[l], C.n_level[l], l);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int NP>
hipError_t batch_factor_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                           bool want_q, int waves, hipStream_t s)
{
    {
        const size_t lds = (size_t)waves * leaf_lds_doubles(NP, tile_rows_for(NP), want_q) * sizeof(double);
        const dim3 grid(batch_grid(C.n_leaf, waves)), block(64 * waves);
        if (want_q) {
            allow_lds(k_leaf_batch<NP, true>, lds);
            hipLaunchKernelGGL((k_leaf_batch<NP, true>), grid, block, lds, s, probs, args, ws, C.leaf_items, C.n_leaf);
        } else {
            allow_lds(k_leaf_batch<NP, false>, lds);
            hipLaunchKernelGGL((k_leaf_batch<NP, false>), grid, block, lds, s, probs, args, ws, C.leaf_items, C.n_leaf);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (want_q) {
            const size_t blds = (size_t)waves * BuildTLds<NP>::WS * sizeof(double);
            allow_lds(k_build_T_batch<NP>, blds);
            hipLaunchKernelGGL((k_build_T_batch<NP>), grid, block, blds, s, probs, ws, C.leaf_items, C.n_leaf);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    const int tw = NP <= 32 ? 4 : 2;
    const size_t tlds = (size_t)tw * factor_lds_doubles(NP, round16(NP), want_q) * sizeof(double);
    for (int l = 1; l <= C.max_levels; ++l) {
        const dim3 grid(batch_grid(C.n_level[l], tw)), block(64 * tw);
        if (want_q) {
            allow_lds(k_tree_batch<NP, true>, tlds);
            hipLaunchKernelGGL((k_tree_batch<NP, true>), grid, block, tlds, s, probs, ws, C.level_items[l], C.n_level[l], l);
        } else {
            allow_lds(k_tree_batch<NP, false>, tlds);
            hipLaunchKernelGGL((k_tree_batch<NP, false>), grid, block, tlds, s, probs, ws, C.level_items[l], C.n_level[l], l);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (want_q) {
        hipError_t e = batch_node_T<NP>(C, probs, ws, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_root_batch<NP>), dim3(batch_grid(C.nprob, 4)), dim3(256), 0, s, probs, args, ws,
                       C.root_items, C.nprob, want_q ? 1 : 0);
    return hipGetLastError();
}

template <int NP, int JW>
hipError_t batch_form_q_launch(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                               int waves, hipStream_t s)
{
    constexpr int NPB = round16(NP), SPLIT = NPB / 16 / JW;
    const size_t lds = (size_t)waves * fq_lds_elems<double>(NP, JW) * sizeof(double);
    allow_lds(k_form_q_batch<NP, JW>, lds);
    hipLaunchKernelGGL((k_form_q_batch<NP, JW>), dim3(batch_grid(C.n_leaf * SPLIT, waves)), dim3(64 * waves), lds,
                       s, probs, args, ws, C.leaf_items, C.n_leaf);
    return hipGetLastError();
}

template <int NP>
hipError_t batch_form_q_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                           int waves, bool alias, hipStream_t s)
{
    for (int l = C.max_levels; l >= 1; --l) {
        hipLaunchKernelGGL((k_seed_batch<NP>), dim3(batch_grid(C.n_level[l], 4)), dim3(256), 0, s, probs, ws,
                           C.level_items[l], C.n_level[l], l);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    constexpr int NPB = round16(NP), JB = NPB / 16, JWD = fq_col_blocks<double>(NP);
    // Q over A in some problem: one wavefront per leaf (see k_form_q)
    if (alias && JWD < JB) return batch_form_q_launch<NP, JB>(C, probs, args, ws, waves, s);
    return batch_form_q_launch<NP, JWD>(C, probs, args, ws, waves, s);
}

// ---- batched mixed precision ------------------------------------------------
// The single-problem mixed path per item: FP32 leaf chains into V32 / T32, T
// from the FP32 slots, the FP64 tree, R1 into the workspace, the seeds, Q1 in
// FP32, then the second pass (partial Gram matrices over row groups, the two
// pairwise sums, the check / Cholesky / R = R2 R1 per problem) and, for the
// explicit Q, Q = Q1 R2^{-1} over 16-row blocks.

template <int NP, bool WANT_Q>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_leaf_batch_mx(const BatchProblem* __restrict__ probs,
                                                    const BatchArgs* __restrict__ args, double* ws,
                                                    const int64_t* __restrict__ items, int64_t nitems)
{
    constexpr int WS = leaf_lds_doubles<float>(NP, tile_rows_f32(NP), WANT_Q);
    extern __shared__ double smem[];
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems; it += nw) {
        const int64_t item = items[it];
        const int64_t p = item >> 32, leaf = item & 0xffffffff;
        const BatchProblem& B = probs[p];
        const BatchArgs X = args[p];
        double* w = ws + B.ws_off;
        leaf_chain<NP, WANT_Q, float>(X.A, X.lda, reinterpret_cast<float*>(w + B.off_V32), B.ld32, B.m, B.n, B.P,
                                      B.leaf_rows, B.f, reinterpret_cast<float*>(w + B.off_T32), w + B.off_R[0],
                                      leaf, smem + wave * WS, lane);
        __builtin_amdgcn_wave_barrier();  // the next item rewrites this wave's LDS
    }
}

template <int NP>
__global__ void __launch_bounds__(256) k_build_T_batch_mx(const BatchProblem* __restrict__ probs, double* ws,
                                                          const int64_t* __restrict__ items, int64_t nitems)
{
    constexpr int MT = tile_rows_f32(NP), NT = packed_size(NP);
    extern __shared__ double smem[];
    const int wave = wave_index(), lane = threadIdx.x & 63;
    double* W = smem + wave * BuildTLds<NP>::WS;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems; it += nw) {
        const int64_t item = items[it];
        const int64_t p = item >> 32, leaf = item & 0xffffffff;
        const BatchProblem& B = probs[p];
        const int64_t row0 = leaf * B.leaf_rows;
        const int64_t rows = (leaf == B.P - 1) ? (B.m - row0) : B.leaf_rows;
        const int64_t ntl = (rows + MT - 1) / MT;
        float* T = reinterpret_cast<float*>(ws + B.ws_off + B.off_T32) + leaf * B.f * NT;
        for (int64_t t = 0; t < ntl; ++t) build_T_slot<NP, float>(T + t * NT, W, lane);
    }
}

// R (sign-normalised) of every problem into its R1 (leading dimension NP) and
// its root seed.
template <int NP>
__global__ void __launch_bounds__(256) k_root_batch_mx(const BatchProblem* __restrict__ probs, double* ws,
                                                       const int64_t* __restrict__ items, int64_t nitems)
{
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems; it += nw) {
        const BatchProblem& B = probs[items[it] >> 32];
        double* w = ws + B.ws_off;
        root_body<NP>(w + B.off_R[B.levels], B.n, w + B.off_R1, NP, w + B.off_D, w + B.off_S[B.levels], lane);
    }
}

template <int NP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_form_q1_batch(const BatchProblem* __restrict__ probs,
                                                    double* ws, const int64_t* __restrict__ items, int64_t nitems)
{
    constexpr int NPB = round16(NP), JW = fq_col_blocks<float>(NP), SPLIT = NPB / 16 / JW;
    extern __shared__ double smem_d[];
    float* smem = reinterpret_cast<float*>(smem_d);
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems * SPLIT; it += nw) {
        const int64_t item = items[it / SPLIT];
        const int j0 = (int)(it % SPLIT) * JW;
        const int64_t p = item >> 32, leaf = item & 0xffffffff;
        const BatchProblem& B = probs[p];
        double* w = ws + B.ws_off;
        const float* V32 = reinterpret_cast<const float*>(w + B.off_V32);
        form_q_leaf<NP, true, float>(V32, B.ld32, B.m, B.n, B.P, B.leaf_rows, B.f,
                                     reinterpret_cast<const float*>(w + B.off_T32), w + B.off_S[0],
                                     reinterpret_cast<float*>(w + B.off_Q1), B.ld32, leaf, j0,
                                     smem + wave * fq_lds_elems<float>(NP, JW), lane);
        __builtin_amdgcn_wave_barrier();
    }
}

// items: (problem, partial Gram index w)
template <int NP>
__global__ void __launch_bounds__(256) k_gram_q1_batch(const BatchProblem* __restrict__ probs, double* ws,
                                                       const int64_t* __restrict__ items, int64_t nitems)
{
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems; it += nw) {
        const int64_t item = items[it];
        const BatchProblem& B = probs[item >> 32];
        double* w = ws + B.ws_off;
        gram_q1_wave<NP>(reinterpret_cast<const float*>(w + B.off_Q1), B.ld32, B.ld32, B.gram_rows,
                         item & 0xffffffff, w + B.off_Gp, lane);
    }
}

// items: (problem, group g of 64 partials); one workgroup of 256 per item
template <int NP>
__global__ void __launch_bounds__(256) k_gram_sum64_batch(const BatchProblem* __restrict__ probs, double* ws,
                                                          const int64_t* __restrict__ items, int64_t nitems)
{
    constexpr int NPB = round16(NP);
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int64_t item = items[it];
        const BatchProblem& B = probs[item >> 32];
        double* w = ws + B.ws_off;
        const int64_t g = item & 0xffffffff;
        for (int e = threadIdx.x; e < NPB * NPB; e += blockDim.x)
            w[B.off_Gq + g * NPB * NPB + e] = gram_sum64_entry<NP>(w + B.off_Gp, B.gram_waves, g, e);
    }
}

// items: (problem, 0); one workgroup of 256 per item
template <int NP>
__global__ void __launch_bounds__(256) k_gram_sum_batch(const BatchProblem* __restrict__ probs, double* ws,
                                                        const int64_t* __restrict__ items, int64_t nitems)
{
    constexpr int NPB = round16(NP);
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BatchProblem& B = probs[items[it] >> 32];
        double* w = ws + B.ws_off;
        const int64_t ng = (B.gram_waves + 63) / 64;
        for (int e = threadIdx.x; e < NPB * NPB; e += blockDim.x)
            w[B.off_G + e] = gram_sum_entry<NP>(w + B.off_Gq, ng, e);
    }
}

// items: (problem, 0); one workgroup of one wavefront per item; R to the caller
template <int NP>
__global__ void __launch_bounds__(64) k_reorth_factor_batch(const BatchProblem* __restrict__ probs,
                                                            const BatchArgs* __restrict__ args, double* ws,
                                                            const int64_t* __restrict__ items, int64_t nitems,
                                                            double bound)
{
    extern __shared__ double Gs[];  // reorth_lds_doubles<NP>()
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int64_t p = items[it] >> 32;
        const BatchProblem& B = probs[p];
        const BatchArgs X = args[p];
        double* w = ws + B.ws_off;
        reorth_factor_body<NP>(w + B.off_G, w + B.off_R1, B.n, bound, w + B.off_R2inv, w + B.off_info, X.X, X.ldx,
                               Gs, threadIdx.x);
        __syncthreads();  // the next item rewrites the LDS buffers
    }
}

// items: (problem, chunk c): 16-row blocks [64 c, 64 c + 64) of the problem
template <int NP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_reorth_q_batch(const BatchProblem* __restrict__ probs,
                                                    const BatchArgs* __restrict__ args, double* ws,
                                                    const int64_t* __restrict__ items, int64_t nitems)
{
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < nitems; it += nw) {
        const int64_t item = items[it];
        const int64_t p = item >> 32, c = item & 0xffffffff;
        const BatchProblem& B = probs[p];
        const BatchArgs X = args[p];
        double* w = ws + B.ws_off;
        const int64_t nblocks = (B.m + 15) / 16;
        const int64_t rb1 = 64 * c + 64 < nblocks ? 64 * c + 64 : nblocks;
        reorth_q_blocks<NP>(reinterpret_cast<const float*>(w + B.off_Q1), B.ld32, B.m, B.n, w + B.off_R2inv, X.X,
                            X.ldx, 64 * c, rb1, 1, lane);
    }
}

template <int NP>
hipError_t batch_factor_mixed_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                                 bool want_q, int waves, hipStream_t s)
{
    hipError_t e;
    {
        const size_t lds = (size_t)waves * leaf_lds_doubles<float>(NP, tile_rows_f32(NP), want_q) * sizeof(double);
        const dim3 grid(batch_grid(C.n_leaf, waves)), block(64 * waves);
        if (want_q) {
            allow_lds(k_leaf_batch_mx<NP, true>, lds);
            hipLaunchKernelGGL((k_leaf_batch_mx<NP, true>), grid, block, lds, s, probs, args, ws, C.leaf_items,
                               C.n_leaf);
        } else {
            allow_lds(k_leaf_batch_mx<NP, false>, lds);
            hipLaunchKernelGGL((k_leaf_batch_mx<NP, false>), grid, block, lds, s, probs, args, ws, C.leaf_items,
                               C.n_leaf);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (want_q) {
            const size_t blds = (size_t)waves * BuildTLds<NP>::WS * sizeof(double);
            allow_lds(k_build_T_batch_mx<NP>, blds);
            hipLaunchKernelGGL((k_build_T_batch_mx<NP>), grid, block, blds, s, probs, ws, C.leaf_items, C.n_leaf);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    const int tw = NP <= 32 ? 4 : 2;
    const size_t tlds = (size_t)tw * factor_lds_doubles(NP, round16(NP), want_q) * sizeof(double);
    for (int l = 1; l <= C.max_levels; ++l) {
        const dim3 grid(batch_grid(C.n_level[l], tw)), block(64 * tw);
        if (want_q) {
            allow_lds(k_tree_batch<NP, true>, tlds);
            hipLaunchKernelGGL((k_tree_batch<NP, true>), grid, block, tlds, s, probs, ws, C.level_items[l], C.n_level[l], l);
        } else {
            allow_lds(k_tree_batch<NP, false>, tlds);
            hipLaunchKernelGGL((k_tree_batch<NP, false>), grid, block, tlds, s, probs, ws, C.level_items[l], C.n_level[l], l);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (want_q) {
        e = batch_node_T<NP>(C, probs, ws, s);
        if (e != hipSuccess) return e;
    }
    if (!want_q) {
        // R only: the first pass is the result
        hipLaunchKernelGGL((k_root_batch<NP>), dim3(batch_grid(C.nprob, 4)), dim3(256), 0, s, probs, args, ws,
                           C.root_items, C.nprob, 0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_root_batch_mx<NP>), dim3(batch_grid(C.nprob, 4)), dim3(256), 0, s, probs, ws, C.root_items,
                       C.nprob);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int l = C.max_levels; l >= 1; --l) {
        hipLaunchKernelGGL((k_seed_batch<NP>), dim3(batch_grid(C.n_level[l], 4)), dim3(256), 0, s, probs, ws,
                           C.level_items[l], C.n_level[l], l);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    {
        constexpr int NPB = round16(NP), JW = fq_col_blocks<float>(NP), SPLIT = NPB / 16 / JW;
        const size_t lds = (size_t)waves * fq_lds_elems<float>(NP, JW) * sizeof(float);
        allow_lds(k_form_q1_batch<NP>, lds);
        hipLaunchKernelGGL((k_form_q1_batch<NP>), dim3(batch_grid(C.n_leaf * SPLIT, waves)), dim3(64 * waves), lds,
                           s, probs, ws, C.leaf_items, C.n_leaf);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_gram_q1_batch<NP>), dim3(batch_grid(C.n_gram, 4)), dim3(256), 0, s, probs, ws, C.gram_items,
                       C.n_gram);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_gram_sum64_batch<NP>), dim3((unsigned)(C.n_gsum < 4096 ? C.n_gsum : 4096)), dim3(256), 0, s,
                       probs, ws, C.gsum_items, C.n_gsum);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_gram_sum_batch<NP>), dim3((unsigned)(C.nprob < 4096 ? C.nprob : 4096)), dim3(256), 0, s,
                       probs, ws, C.root_items, C.nprob);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t rlds = (size_t)reorth_lds_doubles<NP>() * sizeof(double);
    allow_lds(k_reorth_factor_batch<NP>, rlds);
    hipLaunchKernelGGL((k_reorth_factor_batch<NP>), dim3((unsigned)(C.nprob < 4096 ? C.nprob : 4096)), dim3(64),
                       rlds, s, probs, args, ws, C.root_items, C.nprob, kReorthBound);
    return hipGetLastError();
}

template <int NP>
hipError_t batch_form_q_mixed_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                                 hipStream_t s)
{
    hipLaunchKernelGGL((k_reorth_q_batch<NP>), dim3(batch_grid(C.n_rq, 4)), dim3(256), 0, s, probs, args, ws,
                       C.rq_items, C.n_rq);
    return hipGetLastError();
}

// ---- mixed precision -------------------------------------------------------

// True when the byte offset of element (15, 12) of a 16 x 16 FP32 block with
// leading dimension ld fits in 32 bits.
inline bool lane_offsets_fit_32_f32(int64_t ld) { return (uint64_t)(15 + 12 * ld) * 4u < (1ull << 32); }

template <int NP>
hipError_t mixed_leaf_np(const Layout& L, const double* A, int64_t lda, double* ws, bool want_q, hipStream_t s)
{
    constexpr int MT = tile_rows_f32(NP);
    const size_t lds = (size_t)L.waves * leaf_lds_doubles<float>(NP, MT, want_q) * sizeof(double);
    const dim3 grid(grid_for(L.P, L.waves)), block(64 * L.waves);
    float* V32 = reinterpret_cast<float*>(ws + L.off_V32);
    float* T32 = reinterpret_cast<float*>(ws + L.off_T32);
    if (want_q) {
        allow_lds(k_leaf_factor<NP, true, float>, lds);
        hipLaunchKernelGGL((k_leaf_factor<NP, true, float>), grid, block, lds, s, A, lda, V32, L.ld32, L.m,
                           (int)L.n, L.P, L.leaf_rows, L.f, T32, ws + L.off_R[0]);
    } else {
        allow_lds(k_leaf_factor<NP, false, float>, lds);
        hipLaunchKernelGGL((k_leaf_factor<NP, false, float>), grid, block, lds, s, A, lda, V32, L.ld32, L.m,
                           (int)L.n, L.P, L.leaf_rows, L.f, T32, ws + L.off_R[0]);
    }
    return hipGetLastError();
}

template <int NP>
hipError_t form_q1_np(const Layout& L, double* ws, hipStream_t s)
{
    constexpr int NPB = round16(NP), JW = fq_col_blocks<float>(NP), SPLIT = NPB / 16 / JW;
    const size_t lds = (size_t)L.waves * fq_lds_elems<float>(NP, JW) * sizeof(float);
    const dim3 grid(grid_for(L.P * SPLIT, L.waves)), block(64 * L.waves);
    const float* V32 = reinterpret_cast<const float*>(ws + L.off_V32);
    const float* T32 = reinterpret_cast<const float*>(ws + L.off_T32);
    float* Q1 = reinterpret_cast<float*>(ws + L.off_Q1);
    if (lane_offsets_fit_32_f32(L.ld32)) {
        allow_lds(k_form_q<NP, false, float>, lds);
        hipLaunchKernelGGL((k_form_q<NP, false, float>), grid, block, lds, s, V32, L.ld32, L.m, (int)L.n, L.P,
                           L.leaf_rows, L.f, T32, ws + L.off_S[0], Q1, L.ld32);
    } else {
        allow_lds(k_form_q<NP, true, float>, lds);
        hipLaunchKernelGGL((k_form_q<NP, true, float>), grid, block, lds, s, V32, L.ld32, L.m, (int)L.n, L.P,
                           L.leaf_rows, L.f, T32, ws + L.off_S[0], Q1, L.ld32);
    }
    return hipGetLastError();
}

template <int NP>
hipError_t reorth_np(const Layout& L, double* ws, double* R, int64_t ldr, hipStream_t s)
{
    constexpr int NPB = round16(NP);
    const float* Q1 = reinterpret_cast<const float*>(ws + L.off_Q1);
    hipLaunchKernelGGL((k_gram_q1<NP>), dim3(grid_for(L.gram_waves, 4)), dim3(256), 0, s, Q1, L.ld32, L.ld32,
                       L.gram_rows, L.gram_waves, ws + L.off_Gp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t ng = (L.gram_waves + 63) / 64;
    hipLaunchKernelGGL((k_gram_sum64<NP>), dim3((NPB * NPB + 255) / 256, (unsigned)ng), dim3(256), 0, s,
                       ws + L.off_Gp, L.gram_waves, ws + L.off_Gq);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_gram_sum<NP>), dim3((NPB * NPB + 255) / 256), dim3(256), 0, s, ws + L.off_Gq, ng,
                       ws + L.off_G);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t rlds = (size_t)reorth_lds_doubles<NP>() * sizeof(double);
    allow_lds(k_reorth_factor<NP>, rlds);
    hipLaunchKernelGGL((k_reorth_factor<NP>), dim3(1), dim3(64), rlds, s, ws + L.off_G, ws + L.off_R1, (int)L.n,
                       kReorthBound, ws + L.off_R2inv, ws + L.off_info, R, ldr);
    return hipGetLastError();
}

template <int NP>
hipError_t reorth_q_np(const Layout& L, double* ws, double* Q, int64_t ldq, hipStream_t s)
{
    const float* Q1 = reinterpret_cast<const float*>(ws + L.off_Q1);
    const int64_t nblocks = (L.m + 15) / 16;
    const int64_t waves = nblocks < 8192 ? nblocks : 8192;
    hipLaunchKernelGGL((k_reorth_q<NP>), dim3(grid_for(waves, 4)), dim3(256), 0, s, Q1, L.ld32, L.m, (int)L.n,
                       ws + L.off_R2inv, Q, ldq, nblocks);
    return hipGetLastError();
}


// ---- Q^T B on a mixed plan ---------------------------------------------------
// The plan's Q is Q1 R2^{-1} (Q1 the FP32 first pass's explicit Q, R2^{-1}
// from the second pass: the identity when its check did not call for it), so
// Q^T B = R2^{-T} (Q1^T B): n x kc, written over the top n rows of B (the
// thin factor has no complement for the other rows).  Q1^T B takes the second
// pass's route: partial products of 64-row groups on the FP64 matrix cores
// (Q1's FP32 entries and their products with B exact in FP64 inputs), summed
// pairwise in two stages (k_psum64, k_psum), then R2^{-T} on the sum.
__host__ __device__ constexpr int qtb_cols(int npb) { return npb >= 32 ? 32 : 16; }

template <int NP>
__global__ void __launch_bounds__(256) k_q1tb(const float* __restrict__ Q1, int64_t ldq1, int64_t m,
                                              const double* __restrict__ B, int64_t ldb, int kc, int64_t rw,
                                              int64_t nw, double* __restrict__ Pp)
{
    constexpr int NPB = round16(NP), JB = NPB / 16, KCOL = qtb_cols(NPB), JK = KCOL / 16;
    const int wave = wave_index(), lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (w >= nw) return;
    const int q = lane >> 4, p = lane & 15;
    dbl4 acc[JB][JK];
#pragma unroll
    for (int ib = 0; ib < JB; ++ib)
#pragma unroll
        for (int jb = 0; jb < JK; ++jb) acc[ib][jb] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int64_t r0 = w * rw, r1 = (r0 + rw) < m ? (r0 + rw) : m;
    // B's columns start 16-byte aligned (aligned base, even ldb): 16-byte loads
    const bool vec2 = ((reinterpret_cast<uintptr_t>(B) & 15) == 0) && ((ldb & 1) == 0);
    for (int64_t g = r0; g < r1; g += 64) {
        // Q1: rows g + 16 q .. + 15 of column 16 b + p (the workspace holds
        // whole 64-row groups past m); B: the same rows of column 16 jb + p,
        // columns past kc read column kc - 1 and rows past m row m - 1, then zeroed
        float x[JB][16];
#pragma unroll
        for (int b = 0; b < JB; ++b) {
            const float* src = Q1 + g + 16 * q + (int64_t)(16 * b + p) * ldq1;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float4 t = *reinterpret_cast<const float4*>(src + 4 * v);
                x[b][4 * v] = t.x;
                x[b][4 * v + 1] = t.y;
                x[b][4 * v + 2] = t.z;
                x[b][4 * v + 3] = t.w;
            }
        }
        double y[JK][16];
        const bool full = g + 64 <= m;
#pragma unroll
        for (int jb = 0; jb < JK; ++jb) {
            const int c = 16 * jb + p, cc = c < kc ? c : kc - 1;
            const double* col = B + (int64_t)cc * ldb;
            if (full && vec2) {
                // 16-byte loads: the lane's 16 rows are 128 consecutive bytes
                const double2* src = reinterpret_cast<const double2*>(col + g + 16 * q);
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const double2 t = src[v];
                    y[jb][2 * v] = c < kc ? t.x : 0.0;
                    y[jb][2 * v + 1] = c < kc ? t.y : 0.0;
                }
            } else {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t r = g + 16 * q + v;
                    const int64_t rr = full ? r : (r < m ? r : m - 1);
                    const double val = col[rr];
                    y[jb][v] = (c < kc && (full || r < m)) ? val : 0.0;
                }
            }
        }
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2)
#pragma unroll
            for (int ib = 0; ib < JB; ++ib)
#pragma unroll
                for (int jb = 0; jb < JK; ++jb) acc[ib][jb] = mfma16x16x4((double)x[ib][s2], y[jb][s2], acc[ib][jb]);
    }
    double* P = Pp + w * NPB * KCOL;
#pragma unroll
    for (int ib = 0; ib < JB; ++ib)
#pragma unroll
        for (int jb = 0; jb < JK; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) P[(16 * ib + q + 4 * r) + (16 * jb + p) * NPB] = acc[ib][jb][r];
}

// Stage 1: block (x, g) sums partials [64 g, 64 g + 64) entry by entry (eight
// interleaved accumulators, combined as a tree).
template <int NP>
__global__ void __launch_bounds__(256) k_psum64(const double* __restrict__ Pp, int64_t nw, double* __restrict__ Pq)
{
    constexpr int ENT = round16(NP) * qtb_cols(round16(NP));
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t g = blockIdx.y;
    if (e >= ENT) return;
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int64_t w0 = 64 * g, wn = (nw - w0) < 64 ? (nw - w0) : 64;
    for (int64_t u = 0; u < wn; ++u) a[u % 8] += Pp[(w0 + u) * ENT + e];
    Pq[g * ENT + e] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Stage 2: one thread per entry merges the ng group sums as a binary counter.
template <int NP>
__global__ void __launch_bounds__(256) k_psum(const double* __restrict__ Pq, int64_t ng, double* __restrict__ P)
{
    constexpr int ENT = round16(NP) * qtb_cols(round16(NP));
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ENT) return;
    double stack[32];
    int64_t cnt = 0;
    for (int64_t g = 0; g < ng; ++g) {
        double cs = Pq[g * ENT + e];
        int lvl = 0;
        for (int64_t c = cnt; c & 1; c >>= 1) cs = stack[lvl++] + cs;
        stack[lvl] = cs;
        ++cnt;
    }
    double sum = 0.0;
    for (int lvl = 0; cnt >> lvl; ++lvl)
        if ((cnt >> lvl) & 1) sum = stack[lvl] + sum;
    P[e] = sum;
}

// B(i, c) = sum_{j <= i} R2^{-1}(j, i) P(j, c) for i < n, c < kc.
template <int NP>
__global__ void __launch_bounds__(256) k_q1tb_finish(const double* __restrict__ P, const double* __restrict__ R2inv,
                                                     int n, double* __restrict__ B, int64_t ldb, int kc)
{
    constexpr int NPB = round16(NP);
    for (int e = threadIdx.x; e < n * kc; e += blockDim.x) {
        const int i = e % n, c = e / n;
        double acc = 0.0;
        for (int j = 0; j <= i; ++j) acc = fma(R2inv[j + i * NPB], P[j + c * NPB], acc);
        B[i + (int64_t)c * ldb] = acc;
    }
}

template <int NP>
hipError_t qtb_mixed_np(const Layout& L, double* ws, int64_t k, double* B, int64_t ldb, hipStream_t s)
{
    constexpr int NPB = round16(NP), KCOL = qtb_cols(NPB), ENT = NPB * KCOL;
    static_assert(ENT <= NPB * NPB || NPB == 16, "the partial products fit the Gram areas");
    const float* Q1 = reinterpret_cast<const float*>(ws + L.off_Q1);
    const int64_t ng = (L.gram_waves + 63) / 64;
    for (int64_t c0 = 0; c0 < k; c0 += KCOL) {
        const int kc = (int)((k - c0) < KCOL ? (k - c0) : KCOL);
        double* Bc = B + c0 * ldb;
        hipLaunchKernelGGL((k_q1tb<NP>), dim3(grid_for(L.gram_waves, 4)), dim3(256), 0, s, Q1, L.ld32, L.m, Bc,
                           ldb, kc, L.gram_rows, L.gram_waves, ws + L.off_Gp);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) {
            hipLaunchKernelGGL((k_psum64<NP>), dim3((ENT + 255) / 256, (unsigned)ng), dim3(256), 0, s, ws + L.off_Gp,
                               L.gram_waves, ws + L.off_Gq);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL((k_psum<NP>), dim3((ENT + 255) / 256), dim3(256), 0, s, ws + L.off_Gq, ng,
                               ws + L.off_G);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL((k_q1tb_finish<NP>), dim3(1), dim3(256), 0, s, ws + L.off_G, ws + L.off_R2inv,
                               (int)L.n, Bc, ldb, kc);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace detail

template <int NP>
hipError_t leaf_factor_np(const Layout& L, const double* A, int64_t lda, double* V, int64_t ldv, double* ws,
                          bool want_q, hipStream_t s)
{
    return detail::leaf_factor_np<NP>(L, A, lda, V, ldv, ws, want_q, s);
}
template <int NP>
hipError_t build_T_np(const Layout& L, double* ws, hipStream_t s)
{
    return detail::build_T_np<NP>(L, ws, s);
}
template <int NP>
int leaf_lds_bytes_np(bool mixed, bool want_q)
{
    return 8 * (mixed ? detail::leaf_lds_doubles<float>(NP, tile_rows_f32(NP), want_q)
                      : detail::leaf_lds_doubles<double>(NP, tile_rows_for(NP), want_q));
}
template <int NP>
hipError_t tree_np(const Layout& L, double* ws, bool want_q, hipStream_t s)
{
    return detail::tree_np<NP>(L, ws, want_q, s);
}
template <int NP>
hipError_t root_np(const Layout& L, double* ws, double* R, int64_t ldr, hipStream_t s)
{
    return detail::root_np<NP>(L, ws, R, ldr, s);
}
template <int NP>
hipError_t seeds_np(const Layout& L, double* ws, hipStream_t s)
{
    return detail::seeds_np<NP>(L, ws, s);
}
template <int NP>
hipError_t form_q_np(const Layout& L, const double* A, int64_t lda, double* ws, double* Q, int64_t ldq,
                     hipStream_t s)
{
    return detail::form_q_np<NP>(L, A, lda, ws, Q, ldq, s);
}
template <int NP>
hipError_t apply_qt_np(const Layout& L, const double* A, int64_t lda, int64_t k, double* B, int64_t ldb,
                       double* ws, hipStream_t s)
{
    return detail::apply_qt_np<NP>(L, A, lda, k, B, ldb, ws, s);
}

template <int NP>
hipError_t mixed_leaf_np(const Layout& L, const double* A, int64_t lda, double* ws, bool want_q, hipStream_t s)
{
    return detail::mixed_leaf_np<NP>(L, A, lda, ws, want_q, s);
}
template <int NP>
hipError_t form_q1_np(const Layout& L, double* ws, hipStream_t s)
{
    return detail::form_q1_np<NP>(L, ws, s);
}
template <int NP>
hipError_t reorth_np(const Layout& L, double* ws, double* R, int64_t ldr, hipStream_t s)
{
    return detail::reorth_np<NP>(L, ws, R, ldr, s);
}
template <int NP>
hipError_t reorth_q_np(const Layout& L, double* ws, double* Q, int64_t ldq, hipStream_t s)
{
    return detail::reorth_q_np<NP>(L, ws, Q, ldq, s);
}
template <int NP>
hipError_t qtb_mixed_np(const Layout& L, double* ws, int64_t k, double* B, int64_t ldb, hipStream_t s)
{
    return detail::qtb_mixed_np<NP>(L, ws, k, B, ldb, s);
}

template <int NP>
hipError_t batch_factor_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                           bool want_q, int waves, hipStream_t s)
{
    return detail::batch_factor_np<NP>(C, probs, args, ws, want_q, waves, s);
}
template <int NP>
hipError_t batch_form_q_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                           int waves, bool alias, hipStream_t s)
{
    return detail::batch_form_q_np<NP>(C, probs, args, ws, waves, alias, s);
}
template <int NP>
hipError_t batch_factor_mixed_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                                 bool want_q, int waves, hipStream_t s)
{
    return detail::batch_factor_mixed_np<NP>(C, probs, args, ws, want_q, waves, s);
}
template <int NP>
hipError_t batch_form_q_mixed_np(const BatchClass& C, const BatchProblem* probs, const BatchArgs* args, double* ws,
                                 hipStream_t s)
{
    return detail::batch_form_q_mixed_np<NP>(C, probs, args, ws, s);
}

// Every per-width launcher of one padded width (used by the tsqr_np_*.hip units).
#define TSQR_INSTANTIATE(NP)                                                                                   \
    template hipError_t leaf_factor_np<NP>(const Layout&, const double*, int64_t, double*, int64_t, double*, bool, \
                                           hipStream_t);                                                     \
    template hipError_t build_T_np<NP>(const Layout&, double*, hipStream_t);                                   \
    template int leaf_lds_bytes_np<NP>(bool, bool);                                                            \
    template hipError_t tree_np<NP>(const Layout&, double*, bool, hipStream_t);                                \
    template hipError_t root_np<NP>(const Layout&, double*, double*, int64_t, hipStream_t);                    \
    template hipError_t seeds_np<NP>(const Layout&, double*, hipStream_t);                                     \
    template hipError_t form_q_np<NP>(const Layout&, const double*, int64_t, double*, double*, int64_t,        \
                                      hipStream_t);                                                          \
    template hipError_t apply_qt_np<NP>(const Layout&, const double*, int64_t, int64_t, double*, int64_t,      \
                                        double*, hipStream_t);                                               \
    template hipError_t mixed_leaf_np<NP>(const Layout&, const double*, int64_t, double*, bool, hipStream_t);  \
    template hipError_t form_q1_np<NP>(const Layout&, double*, hipStream_t);                                   \
    template hipError_t reorth_np<NP>(const Layout&, double*, double*, int64_t, hipStream_t);                  \
    template hipError_t reorth_q_np<NP>(const Layout&, double*, double*, int64_t, hipStream_t);                \
    template hipError_t qtb_mixed_np<NP>(const Layout&, double*, int64_t, double*, int64_t, hipStream_t);       \
    template hipError_t batch_factor_np<NP>(const BatchClass&, const BatchProblem*, const BatchArgs*, double*,  \
                                            bool, int, hipStream_t);                                          \
    template hipError_t batch_form_q_np<NP>(const BatchClass&, const BatchProblem*, const BatchArgs*, double*,  \
                                            int, bool, hipStream_t);                                          \
    template hipError_t batch_factor_mixed_np<NP>(const BatchClass&, const BatchProblem*, const BatchArgs*,    \
                                                  double*, bool, int, hipStream_t);                           \
    template hipError_t batch_form_q_mixed_np<NP>(const BatchClass&, const BatchProblem*, const BatchArgs*,    \
                                                  double*, hipStream_t);

}  // namespace tsqr
