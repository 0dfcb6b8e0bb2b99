// tsqr_api.cpp -- the C ABI of libtsqr (include/tsqr.h): plans, argument
// checking, workspace ownership and the order of kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "tsqr.h"
#include "tsqr_internal.h"

namespace tsqr {
bool tuned_opts(int64_t m, int64_t n, tsqr_precision prec, int want_q, tsqr_opts* out);  // tsqr_tune.cpp
}

// The leaf variant of TSQR_LEAF_AUTO where both exist (1: recursive).
#ifndef TSQR_LEAF_AUTO_REC
#define TSQR_LEAF_AUTO_REC 0
#endif

namespace tsqr {

bool make_layout(Layout& L, int64_t m, int64_t n, int64_t leaf_rows_req, int flat_len, int tree, int waves,
                 bool mixed, bool want_q, bool in_batch)
{
    if (n < 1 || n > kMaxN || m < n) return false;
    L = Layout();
    L.m = m;
    L.n = n;
    L.mixed = mixed;
    L.np = padded_width(n);
    L.npb = (int)((n + 15) / 16 * 16);
    L.mt = mixed ? tile_rows_f32(L.np) : tile_rows_for(L.np);
    // automatic waves per workgroup (leaf and Q kernels): 4 with Q, 1 for R only
    // (the fastest choices of the autotuner at m = 2^24, n = 32 and 64)
    L.waves = waves > 0 ? waves : (want_q ? 4 : 1);
    const int64_t tiles_total = (m + L.mt - 1) / L.mt;
    int64_t f;
    if (leaf_rows_req > 0) {
        f = (leaf_rows_req + L.mt - 1) / L.mt;
    } else if (tree == TSQR_TREE_FLAT) {
        f = tiles_total;
    } else if (tree == TSQR_TREE_BINARY) {
        f = 1;
    } else if (tree == TSQR_TREE_HYBRID && flat_len > 0) {
        f = flat_len;
    } else {
        // automatic.  With Q: one resident round of leaves (2048 wavefronts --
        // two per SIMD -- or 1024 where the LDS of the reflector-keeping leaf
        // kernel allows only four per CU), so that the tree is
        // as shallow as the device's parallelism allows.  R only: many short
        // chains (16384 leaves).  Chains are 1..256 tiles, and long enough that
        // the per-leaf factors (R, seed, node Y and T: about 4 np^2 doubles)
        // stay under a quarter of the leaf's f * mt * n doubles.
        // Narrow widths (np <= 24) keep about 4096 leaves.  Mixed precision caps
        // the chain at kMaxChainF32 tiles (accuracy guard: FP32 rounding grows
        // along a chain).  For a problem on its own, the quarter-of-the-data
        // guard is capped at chains of tiles/1024 tiles, rounded down to a power
        // of two (at least 2 from 48
        // columns once there are 1024 tiles): on small problems (m below
        // about 2^21 at n = 64) the parallelism of more, shorter chains
        // outweighs the larger per-leaf factors.  Measured over m = 2^16 ..
        // 2^21 and n = 16, 32, 50, 64 against chains of 1 .. 32 tiles: the
        // best chain is within a factor 2 of that cap (at m = 524288, n = 64:
        // R + Q 1.69 ms against 2.02 ms with the earlier cap of tiles/512,
        // R only 0.87 against 1.18 ms; at 2^21 rows the quarter guard binds
        // and nothing changes).  In a batch the other problems supply the
        // parallelism and the guard stays (2048 problems of m in [1000,
        // 200000]: 107 ms with it, 147 ms without).
        const bool two_per_simd = leaf_lds_bytes(L.np, mixed, want_q) <= 20480;
        const int64_t target = !want_q ? 16384 : (!two_per_simd ? 1024 : (L.np > 24 ? 2048 : 4096));
        f = tiles_total / target;
        int64_t f_mem = (16 * (int64_t)L.np * L.np + L.mt * n - 1) / (L.mt * n);
        if (!in_batch) {
            // a power of two: a chain of 15 tiles at m = 10^6, n = 50 gave 1041
            // leaves, whose Q pass (two wavefronts per leaf) overran one
            // resident round by 34 wavefronts (2.96 ms against 2.05 ms)
            int64_t cap = 1;
            while (cap * 2 <= tiles_total / 1024) cap *= 2;
            if (L.np >= 48 && tiles_total >= 1024) cap = std::max<int64_t>(cap, 2);
            f_mem = std::min<int64_t>(f_mem, cap);
        }
        f = std::max<int64_t>(std::max<int64_t>(1, f_mem), std::min<int64_t>(256, f));
        const int64_t fmax = std::min<int64_t>(mixed ? kMaxChainF32 : 256, std::max<int64_t>(1, tiles_total));
        if (mixed) f = std::min<int64_t>(f, kMaxChainF32);
        f = std::min<int64_t>(f, std::max<int64_t>(1, tiles_total));
        if (!in_batch) {
            // the leaf kernel holds `per_round` leaves at once (R only: two
            // wavefronts per SIMD, whatever the 16384-leaf target) and the last
            // leaf takes the remainder, so a chain just under the right length
            // costs a second round, or a last leaf of almost two chains: at
            // m = 6.4e6, n = 50 chains of 48 / 49 / 50 tiles (2083 / 2040 /
            // 2000 leaves, the last of 64 / 129 / 50 tiles) took 10.4 / 9.2 /
            // 6.9 ms, at m = 3e6, n = 64 chains of 22 / 23 (2130 / 2038
            // leaves) 6.7 / 4.5 ms.  Among chains from f up to twice f take
            // the one with the least f * rounds + (last leaf's excess tiles).
            const int64_t per_round = want_q ? target : (two_per_simd ? 2048 : 1024);
            auto cost = [&](int64_t g) {
                const int64_t lr = g * L.mt, P = std::max<int64_t>(1, m / lr);
                const int64_t last = (m - (P - 1) * lr + L.mt - 1) / L.mt;
                return g * ((P + per_round - 1) / per_round) + std::max<int64_t>(0, last - g);
            };
            int64_t best = f, bc = cost(f);
            for (int64_t g = f + 1; g <= std::min<int64_t>(2 * f, fmax); ++g) {
                const int64_t c = cost(g);
                if (c < bc) best = g, bc = c;
            }
            f = best;
        }
    }
    if (f < 1) f = 1;
    L.f = f;
    L.leaf_rows = f * L.mt;
    L.P = std::max<int64_t>(1, m / L.leaf_rows);
    const int64_t last_rows = m - (L.P - 1) * L.leaf_rows;
    L.ntiles_last = (last_rows + L.mt - 1) / L.mt;
    L.ntiles = (L.P - 1) * L.f + L.ntiles_last;
    L.count[0] = L.P;
    int lv = 0;
    int64_t c = L.P;
    while (c > 1) {
        if (lv + 1 > kMaxLevels) return false;
        c = (c + 1) / 2;
        L.count[++lv] = c;
    }
    L.levels = lv;

    const int64_t np2 = (int64_t)L.np * L.np;
    L.nt = (int64_t)L.np * (L.np + 1) / 2;
    int64_t off = 0;
    auto take = [&](int64_t doubles) {
        int64_t o = off;
        off += (doubles + 31) / 32 * 32;  // 256-byte alignment
        return o;
    };
    L.off_T = take(mixed ? 0 : L.ntiles * L.nt);
    // the T slots of every tree node, level after level in one run, so that
    // one T-kernel launch covers them all (off_TN[1] .. + tree_nodes * nt)
    L.tree_nodes = 0;
    for (int l = 1; l <= L.levels; ++l) L.tree_nodes += L.count[l];
    const int64_t tn0 = take(L.tree_nodes * L.nt);
    int64_t node = 0;
    for (int l = 0; l <= L.levels; ++l) {
        L.off_R[l] = take(L.count[l] * np2);
        L.off_S[l] = take(L.count[l] * np2);
        if (l >= 1) {
            L.off_Y[l] = take(L.count[l] * np2);
            L.off_TN[l] = tn0 + node * L.nt;
            node += L.count[l];
        }
    }
    L.off_D = take(L.np);
    if (mixed) {
        const int64_t npb2 = (int64_t)L.npb * L.npb;
        const int64_t m_tiles = (m + L.mt - 1) / L.mt * L.mt;  // tiles start at multiples of mt
        L.ld32 = (m_tiles + 63) / 64 * 64;
        L.off_T32 = take((L.ntiles * L.nt + 1) / 2);
        L.off_V32 = take((L.ld32 * L.npb + 1) / 2);
        L.off_Q1 = take((L.ld32 * L.npb + 1) / 2);
        const int64_t groups = L.ld32 / 64;
        L.gram_waves = std::min<int64_t>(4096, groups);
        L.gram_rows = (groups + L.gram_waves - 1) / L.gram_waves * 64;
        L.off_Gp = take(L.gram_waves * npb2);
        L.off_Gq = take((L.gram_waves + 63) / 64 * npb2);
        L.off_G = take(npb2);
        L.off_R1 = take((int64_t)L.np * L.np);
        L.off_R2inv = take(npb2);
        L.off_info = take(2);
    }
    L.total = off;
    return true;
}

bool make_layout_r_compact(Layout& L, int64_t m, int64_t n, int64_t leaf_rows_req)
{
    if (!make_layout(L, m, n, leaf_rows_req, 0, TSQR_TREE_AUTO, 0, false, false)) return false;
    // the same geometry; a workspace with only what R needs: the R of every
    // entry of every level, the signs and the root seed the root kernel writes
    const int64_t np2 = (int64_t)L.np * L.np;
    int64_t off = 0;
    auto take = [&](int64_t doubles) {
        int64_t o = off;
        off += (doubles + 31) / 32 * 32;  // 256-byte alignment
        return o;
    };
    L.off_T = 0;  // no tile factors (the R-only leaf kernel writes none)
    for (int l = 0; l <= L.levels; ++l) {
        L.off_R[l] = take(L.count[l] * np2);
        L.off_S[l] = L.off_Y[l] = L.off_TN[l] = 0;  // no node factors or seeds below the root
    }
    L.off_S[L.levels] = take(np2);
    L.off_D = take(L.np);
    L.total = off;
    return true;
}

}  // namespace tsqr

struct PhaseEvent {
    int phase;
    hipEvent_t start, stop;
};

struct tsqr_plan_s {
    tsqr::Layout L;
    tsqr_precision prec = TSQR_FP64;
    tsqr_tree tree = TSQR_TREE_AUTO;
    int want_q = 1;
    hipStream_t stream = nullptr;
    // plans with Q: the T kernel runs on a side stream, concurrently with the
    // tree levels (both need only the leaves), joined back with an event
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    double* ws = nullptr;
    int state = 0;  // 0: nothing factored, 1: factored with reflectors, 2: R only
    // profiling: event pairs recorded since the last tsqr_plan_timings
    bool profile = false;
    std::vector<PhaseEvent> events;
    tsqr_timings sums{};
};

namespace {

tsqr_status hip_status(hipError_t e)
{
    if (e == hipSuccess) return 0;
    if (e == hipErrorOutOfMemory) return 2;
    return 1;
}

// Runs one launch phase, bracketed by events when profiling is on (on stream s,
// the plan's stream by default).
template <typename F>
hipError_t run_phase(tsqr_plan_s* p, int phase, F&& launch, hipStream_t s = nullptr)
{
    if (!p->profile) return launch();
    if (!s) s = p->stream;
    PhaseEvent ev{phase, nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev.start);
    if (e == hipSuccess) e = hipEventCreate(&ev.stop);
    if (e == hipSuccess) e = hipEventRecord(ev.start, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(ev.stop, s);
    if (e == hipSuccess) {
        p->events.push_back(ev);
    } else {
        if (ev.start) hipEventDestroy(ev.start);
        if (ev.stop) hipEventDestroy(ev.stop);
    }
    return e;
}

// The T kernel after the leaves, on the side stream (fork); join_T makes the
// plan's stream wait for it.
hipError_t fork_T(tsqr_plan_s* p)
{
    hipError_t e = hipEventRecord(p->fork_ev, p->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->fork_ev, 0);
    if (e == hipSuccess)
        e = run_phase(p, TSQR_PHASE_LEAF_T, [&] { return tsqr::launch_build_T(p->L, p->ws, p->side); }, p->side);
    if (e == hipSuccess) e = hipEventRecord(p->join_ev, p->side);
    return e;
}

hipError_t join_T(tsqr_plan_s* p) { return hipStreamWaitEvent(p->stream, p->join_ev, 0); }

void release_streams(tsqr_plan_s* p)
{
    if (p->side) {
        hipStreamSynchronize(p->side);
        hipStreamDestroy(p->side);
    }
    if (p->fork_ev) hipEventDestroy(p->fork_ev);
    if (p->join_ev) hipEventDestroy(p->join_ev);
    p->side = nullptr;
    p->fork_ev = p->join_ev = nullptr;
}

hipError_t drain_events(tsqr_plan_s* p)
{
    hipError_t first = hipSuccess;
    for (PhaseEvent& ev : p->events) {
        hipError_t e = hipEventSynchronize(ev.stop);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.start, ev.stop);
        if (e == hipSuccess) {
            p->sums.ms[ev.phase] += ms;
            p->sums.calls[ev.phase] += 1;
        } else if (first == hipSuccess) {
            first = e;
        }
        hipEventDestroy(ev.start);
        hipEventDestroy(ev.stop);
    }
    p->events.clear();
    return first;
}

// Mixed precision: FP32 leaf chains, the FP64 tree and root (R1 kept in the
// workspace when Q is wanted), then Q1 in FP32 and the FP64 second pass, which
// writes R = R2 R1 to the caller.  R-only plans stop after the first pass.
tsqr_status factor_mixed(tsqr_plan_s* p, const double* A, int64_t lda, double* R, int64_t ldr)
{
    const bool want_q = p->want_q != 0;
    const tsqr::Layout& L = p->L;
    hipError_t e = run_phase(p, TSQR_PHASE_LEAF, [&] { return tsqr::launch_mixed_leaf(L, A, lda, p->ws, want_q, p->stream); });
    if (e == hipSuccess && want_q) e = fork_T(p);
    if (e == hipSuccess && L.levels > 0)
        e = run_phase(p, TSQR_PHASE_TREE, [&] { return tsqr::launch_tree(L, p->ws, want_q, p->stream); });
    if (e == hipSuccess)
        e = run_phase(p, TSQR_PHASE_ROOT, [&] {
            return want_q ? tsqr::launch_root(L, p->ws, p->ws + L.off_R1, L.np, p->stream)
                          : tsqr::launch_root(L, p->ws, R, ldr, p->stream);
        });
    if (e == hipSuccess && want_q) {
        if (L.levels > 0) e = run_phase(p, TSQR_PHASE_SEEDS, [&] { return tsqr::launch_seeds(L, p->ws, p->stream); });
        if (e == hipSuccess) e = join_T(p);
        if (e == hipSuccess) e = run_phase(p, TSQR_PHASE_Q1, [&] { return tsqr::launch_form_q1(L, p->ws, p->stream); });
        if (e == hipSuccess)
            e = run_phase(p, TSQR_PHASE_REORTH, [&] { return tsqr::launch_reorth(L, p->ws, R, ldr, p->stream); });
    }
    if (e != hipSuccess) return hip_status(e);
    p->state = want_q ? 1 : 2;
    return 0;
}

}  // namespace

extern "C" {

int tsqr_version(void) { return 100; }

const char* tsqr_status_string(tsqr_status s)
{
    if (s == 0) return "success";
    if (s < 0) return "invalid argument (the negated status is its 1-based position)";
    switch (s) {
    case 1: return "HIP runtime error";
    case 2: return "device memory exhausted";
    case 3: return "unsupported case";
    case 4: return "call out of order (no factorisation with reflectors in the plan)";
    case 5: return "class not in the autotune cache";
    case 6: return "size beyond the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
    }
}

// Argument checks shared by tsqr_plan_create and tsqr_plan_query; fills the
// layout on success.
// prec: the caller's precision argument read as an int (tsqr::abi_int)
static tsqr_status check_plan_args(int64_t m, int64_t n, int pv, const tsqr_opts* opts,
                                   tsqr_opts& o, tsqr::Layout& L)
{
    if (m < 0 || m < n) return -2;
    if (n < 0) return -3;
    if (n > tsqr::kMaxN) return 3;
    if (pv != TSQR_FP64 && pv != TSQR_MIXED) return -4;
    const tsqr_precision prec = (tsqr_precision)pv;
    std::memset(&o, 0, sizeof(o));
    o.want_q = 1;
    tsqr_opts tuned;
    if (!opts && n > 0 && tsqr::tuned_opts(m, n, prec, 1, &tuned)) opts = &tuned;
    if (opts) {
        o = *opts;
        const int tv = tsqr::abi_int(o.tree);
        if (tv < TSQR_TREE_AUTO || tv > TSQR_TREE_HYBRID) return -5;
        if (o.leaf_rows < 0 || o.tile_rows < 0 || o.flat_len < 0) return -5;
        if (o.waves != 0 && o.waves != 1 && o.waves != 2 && o.waves != 4) return -5;
        if (o.want_q != 0 && o.want_q != 1) return -5;
        const int kv = tsqr::abi_int(o.leaf_kind);
        if (kv < TSQR_LEAF_AUTO || kv > TSQR_LEAF_RECURSIVE) return -5;
    }
    if (n == 0) {
        // the empty problem (n = 0, any m >= 0): no tiles, no tree and no
        // workspace; the calls on its plan check their arguments and return
        L = tsqr::Layout{};
        L.m = m;
        L.mixed = prec == TSQR_MIXED;
        return 0;
    }
    if (!tsqr::make_layout(L, m, n, o.leaf_rows, o.flat_len, o.tree, o.waves, prec == TSQR_MIXED, o.want_q != 0))
        return 3;
    if (o.tile_rows != 0 && o.tile_rows != L.mt) return -5;
    // the recursive leaf variant: FP64 with Q at padded widths 16 and 32
    const bool rec_ok = !L.mixed && o.want_q && (L.np == 16 || L.np == 32);
    if (o.leaf_kind == TSQR_LEAF_RECURSIVE && !rec_ok && !L.mixed && o.want_q) return -5;
    L.rec = rec_ok && (o.leaf_kind == TSQR_LEAF_RECURSIVE || (o.leaf_kind == TSQR_LEAF_AUTO && TSQR_LEAF_AUTO_REC));
    return 0;
}

static void fill_info(const tsqr::Layout& L, tsqr_precision prec, tsqr_info* out)
{
    std::memset(out, 0, sizeof(*out));
    out->m = L.m;
    out->n = L.n;
    out->n_padded = L.np;
    out->tile_rows = L.mt;
    out->leaf_rows = L.leaf_rows;
    out->num_leaves = L.P;
    out->num_tiles = L.ntiles;
    out->tree_levels = L.levels;
    out->tree = L.P <= 1 ? TSQR_TREE_FLAT : (L.f == 1 ? TSQR_TREE_BINARY : TSQR_TREE_HYBRID);
    out->waves = L.waves;
    out->precision = prec;
    out->workspace_bytes = L.total * (int64_t)sizeof(double);
    out->leaf_kind = L.rec ? TSQR_LEAF_RECURSIVE : TSQR_LEAF_COMPACT_WY;
}

tsqr_status tsqr_plan_query(int64_t m, int64_t n, tsqr_precision prec, const tsqr_opts* opts, tsqr_info* out)
{
    tsqr_opts o;
    tsqr::Layout L;
    tsqr_status st = check_plan_args(m, n, tsqr::abi_int(prec), opts, o, L);
    if (st < 0) return st + 1;  // argument positions are one lower than in tsqr_plan_create
    if (st != 0) return st;
    if (!out) return -5;
    fill_info(L, prec, out);
    return 0;
}

tsqr_status tsqr_plan_create(tsqr_plan* p, int64_t m, int64_t n, tsqr_precision prec, const tsqr_opts* opts,
                             void* hip_stream)
{
    if (!p) return -1;
    *p = nullptr;
    tsqr_opts o;
    tsqr::Layout L;
    tsqr_status st = check_plan_args(m, n, tsqr::abi_int(prec), opts, o, L);
    if (st != 0) return st;
    tsqr_plan_s* P = new (std::nothrow) tsqr_plan_s();
    if (!P) return 2;
    P->L = L;
    P->prec = prec;  // validated above
    P->tree = o.tree;
    P->want_q = o.want_q;
    P->stream = (hipStream_t)hip_stream;
    if (P->L.n == 0) {  // the empty problem: nothing to allocate
        *p = P;
        return 0;
    }
    hipError_t e = hipMalloc((void**)&P->ws, (size_t)P->L.total * sizeof(double));
    if (e != hipSuccess) {
        delete P;
        return hip_status(e);
    }
    if (P->want_q) {
        e = hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&P->join_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            release_streams(P);
            hipFree(P->ws);
            delete P;
            return hip_status(e);
        }
    }
    if (P->L.mixed) {
        // the FP32 workspaces are read in whole tiles and 16-column blocks: what
        // the kernels never write (rows past the last tile, columns past np) stays zero
        const size_t bytes = (size_t)P->L.ld32 * P->L.npb * sizeof(float);
        e = hipMemsetAsync(P->ws + P->L.off_V32, 0, bytes, P->stream);
        if (e == hipSuccess) e = hipMemsetAsync(P->ws + P->L.off_Q1, 0, bytes, P->stream);
        if (e != hipSuccess) {
            release_streams(P);
            hipFree(P->ws);
            delete P;
            return hip_status(e);
        }
    }
    *p = P;
    return 0;
}

tsqr_status tsqr_factor_into(tsqr_plan p, const double* A, int64_t lda, double* V, int64_t ldv, double* R,
                             int64_t ldr)
{
    if (!p) return -1;
    if (!A && p->L.n > 0) return -2;  // an empty problem references no matrix
    if (lda < p->L.m) return -3;
    const bool want_q = p->want_q != 0;
    if (want_q && !p->L.mixed) {
        if (!V && p->L.n > 0) return -4;
        if (ldv < p->L.m) return -5;
        if ((const double*)V == A && ldv != lda) return -5;
    }
    if (!R && p->L.n > 0) return -6;
    if (ldr < p->L.n) return -7;
    p->state = 0;
    if (p->L.n == 0) {
        p->state = want_q ? 1 : 2;
        return 0;
    }
    if (p->L.mixed) return factor_mixed(p, A, lda, R, ldr);
    hipError_t e = run_phase(p, TSQR_PHASE_LEAF, [&] {
        return tsqr::launch_leaf_factor(p->L, A, lda, V, want_q ? ldv : lda, p->ws, want_q, p->stream);
    });
    // the recursive leaf variant leaves no T kernel to run
    const bool t_kernel = want_q && !p->L.rec;
    if (e == hipSuccess && t_kernel) e = fork_T(p);
    if (e == hipSuccess && p->L.levels > 0)
        e = run_phase(p, TSQR_PHASE_TREE, [&] { return tsqr::launch_tree(p->L, p->ws, want_q, p->stream); });
    if (e == hipSuccess)
        e = run_phase(p, TSQR_PHASE_ROOT, [&] { return tsqr::launch_root(p->L, p->ws, R, ldr, p->stream); });
    if (e == hipSuccess && t_kernel) e = join_T(p);
    if (e != hipSuccess) return hip_status(e);
    p->state = want_q ? 1 : 2;
    return 0;
}

tsqr_status tsqr_factor(tsqr_plan p, double* A, int64_t lda, double* R, int64_t ldr)
{
    tsqr_status st = tsqr_factor_into(p, A, lda, p && p->want_q ? A : nullptr, lda, R, ldr);
    if (st == -6) return -4;
    if (st == -7) return -5;
    return st;
}

tsqr_status tsqr_form_q(tsqr_plan p, const double* A_factored, int64_t lda, double* Q, int64_t ldq)
{
    if (!p) return -1;
    const bool empty = p->L.n == 0;  // no reflectors: Q is m x 0, nothing to write
    if (p->L.mixed) {
        // the reflectors live in the plan: A_factored and lda are not used
        if (!Q && !empty) return -4;
        if (ldq < p->L.m) return -5;
        if (p->state != 1) return 4;
        if (empty) return 0;
        return hip_status(run_phase(p, TSQR_PHASE_FORM_Q, [&] {
            return tsqr::launch_reorth_q(p->L, p->ws, Q, ldq, p->stream);
        }));
    }
    if (!A_factored && !empty) return -2;
    if (lda < p->L.m) return -3;
    if (!Q && !empty) return -4;
    if (ldq < p->L.m) return -5;
    if ((const double*)Q == A_factored && ldq != lda) return -5;
    if (p->state != 1) return 4;
    if (empty) return 0;
    hipError_t e = hipSuccess;
    if (p->L.levels > 0)
        e = run_phase(p, TSQR_PHASE_SEEDS, [&] { return tsqr::launch_seeds(p->L, p->ws, p->stream); });
    if (e == hipSuccess)
        e = run_phase(p, TSQR_PHASE_FORM_Q, [&] {
            return tsqr::launch_form_q(p->L, A_factored, lda, p->ws, Q, ldq, p->stream);
        });
    return hip_status(e);
}

tsqr_status tsqr_apply_qt(tsqr_plan p, const double* A_factored, int64_t lda, int64_t k, double* B, int64_t ldb)
{
    if (!p) return -1;
    if (p->L.mixed) {
        // the reflectors live in the plan: A_factored and lda are not used
        if (k < 0) return -4;
        if (k == 0) return 0;
        if (!B && p->L.m > 0) return -5;  // a 0 x k B is not referenced
        if (ldb < p->L.m) return -6;
        if (p->state != 1) return 4;
        if (p->L.n == 0) return 0;  // no reflectors: Q^T B = B
        return hip_status(run_phase(p, TSQR_PHASE_APPLY, [&] {
            return tsqr::launch_qtb_mixed(p->L, p->ws, k, B, ldb, p->stream);
        }));
    }
    if (!A_factored && p->L.n > 0) return -2;
    if (lda < p->L.m) return -3;
    if (k < 0) return -4;
    if (k == 0) return 0;  // nothing to apply; B may be NULL
    if (!B && p->L.m > 0) return -5;  // a 0 x k B is not referenced
    if (ldb < p->L.m) return -6;
    if (p->state != 1) return 4;
    if (p->L.n == 0) return 0;  // no reflectors: Q^T B = B
    hipError_t e = run_phase(p, TSQR_PHASE_APPLY, [&] {
        return tsqr::launch_apply_qt(p->L, A_factored, lda, k, B, ldb, p->ws, p->stream);
    });
    return hip_status(e);
}

tsqr_status tsqr_plan_info(tsqr_plan p, tsqr_info* out)
{
    if (!p) return -1;
    if (!out) return -2;
    fill_info(p->L, p->prec, out);
    if (p->L.mixed && p->state == 1 && p->L.n > 0) {
        // what the second pass measured: waits for the plan's stream
        double h[2] = {0.0, 0.0};
        hipError_t e = hipStreamSynchronize(p->stream);
        if (e == hipSuccess) e = hipMemcpy(h, p->ws + p->L.off_info, sizeof(h), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_status(e);
        out->orth_estimate = h[0];
        out->reorth_applied = h[1] != 0.0 ? 1 : 0;
    }
    return 0;
}

tsqr_status tsqr_mixed_q1(tsqr_plan p, float* Q1, int64_t ldq1)
{
    if (!p) return -1;
    if (!Q1 && p->L.n > 0) return -2;
    if (ldq1 < p->L.m) return -3;
    if (!p->L.mixed) return 3;
    if (p->state != 1) return 4;
    if (p->L.n == 0) return 0;
    hipError_t e = hipMemcpy2DAsync(Q1, (size_t)ldq1 * sizeof(float), p->ws + p->L.off_Q1,
                                    (size_t)p->L.ld32 * sizeof(float), (size_t)p->L.m * sizeof(float),
                                    (size_t)p->L.n, hipMemcpyDeviceToDevice, p->stream);
    return hip_status(e);
}

tsqr_status tsqr_plan_profile(tsqr_plan p, int enable)
{
    if (!p) return -1;
    if (enable != 0 && enable != 1) return -2;
    hipError_t e = drain_events(p);
    p->profile = enable != 0;
    if (p->profile) std::memset(&p->sums, 0, sizeof(p->sums));
    return hip_status(e);
}

tsqr_status tsqr_plan_timings(tsqr_plan p, tsqr_timings* out)
{
    if (!p) return -1;
    if (!out) return -2;
    hipError_t e = drain_events(p);
    *out = p->sums;
    return hip_status(e);
}

tsqr_status tsqr_plan_destroy(tsqr_plan p)
{
    if (!p) return -1;
    drain_events(p);
    hipError_t e = hipSuccess;
    if (p->ws) {
        e = hipStreamSynchronize(p->stream);
        release_streams(p);
        hipError_t e2 = hipFree(p->ws);
        if (e == hipSuccess) e = e2;
    }
    delete p;
    return hip_status(e);
}

}  // extern "C"
