// tsqr_batched.cpp -- batched TSQR plans: many independent tall-skinny
// problems factored by one replay of a captured HIP graph.
//
// Problems are grouped by padded width (one kernel instantiation per width).
// For each width class the plan holds device work lists -- the (problem,
// leaf) items of the leaf chains and of the explicit-Q pass, the (problem,
// node) items of every tree level, one root item per problem; for mixed
// precision also the (problem, row group) items of the second pass -- and the
// persistent batched kernels walk them.  The per-problem geometry and
// workspace offsets are uploaded once; the matrix pointers of a call go
// through a ring of pinned staging buffers to a small device table, so the
// captured graphs never change and a call costs one small copy and one graph
// launch; the host waits only when more than four calls of a kind are queued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "tsqr.h"
#include "tsqr_internal.h"

namespace tsqr {
bool tuned_opts(int64_t m, int64_t n, tsqr_precision prec, int want_q, tsqr_opts* out);  // tsqr_tune.cpp
}

constexpr int kStageRing = 4;

struct tsqr_batched_plan_s {
    int count = 0;
    tsqr_precision prec = TSQR_FP64;
    int want_q = 1;
    int waves = 0;  // leaf and Q kernels: wavefronts per workgroup
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;  // internal, only for capturing the graphs
    std::vector<tsqr::Layout> L;
    std::vector<tsqr::BatchClass> classes;
    double* ws = nullptr;
    int64_t ws_doubles = 0;
    tsqr::BatchProblem* d_probs = nullptr;
    int64_t* d_items = nullptr;
    tsqr::BatchArgs* d_args_f = nullptr;
    tsqr::BatchArgs* d_args_q = nullptr;
    // pinned staging of the per-call pointer tables: a ring of kStageRing
    // buffers per kind, each with an event recorded after its upload, so the
    // host waits only when more than kStageRing calls of a kind are queued
    tsqr::BatchArgs* h_args_f[kStageRing] = {nullptr};
    tsqr::BatchArgs* h_args_q[kStageRing] = {nullptr};
    hipEvent_t ev_f[kStageRing] = {nullptr}, ev_q[kStageRing] = {nullptr};
    int next_f = 0, next_q = 0;
    // the Q graph of calls where some Q[i] is A[i] (one wavefront per leaf,
    // see k_form_q) and of the others
    hipGraphExec_t g_factor = nullptr, g_form_q = nullptr, g_form_q_alias = nullptr;
    int state = 0;  // 0: nothing factored, 1: factored with reflectors, 2: R only
};

namespace {

tsqr_status hstatus(hipError_t e)
{
    if (e == hipSuccess) return 0;
    if (e == hipErrorOutOfMemory) return 2;
    return 1;
}

void release(tsqr_batched_plan_s* p)
{
    if (p->g_factor) hipGraphExecDestroy(p->g_factor);
    if (p->g_form_q) hipGraphExecDestroy(p->g_form_q);
    if (p->g_form_q_alias) hipGraphExecDestroy(p->g_form_q_alias);
    for (int r = 0; r < kStageRing; ++r) {
        if (p->ev_f[r]) hipEventDestroy(p->ev_f[r]);
        if (p->ev_q[r]) hipEventDestroy(p->ev_q[r]);
        if (p->h_args_f[r]) hipHostFree(p->h_args_f[r]);
        if (p->h_args_q[r]) hipHostFree(p->h_args_q[r]);
    }
    if (p->d_args_f) hipFree(p->d_args_f);
    if (p->d_args_q) hipFree(p->d_args_q);
    if (p->d_items) hipFree(p->d_items);
    if (p->d_probs) hipFree(p->d_probs);
    if (p->ws) hipFree(p->ws);
    if (p->capture) hipStreamDestroy(p->capture);
    delete p;
}

// Captures `enqueue(stream)` into an executable graph.
template <typename F>
hipError_t capture_graph(hipStream_t cap, hipGraphExec_t* exec, F&& enqueue)
{
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return e;
    hipError_t el = enqueue(cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap, &g);
    if (el != hipSuccess) e = el;
    if (e == hipSuccess) e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    return e;
}

// Uploads the pointers of one call through the next pinned staging buffer of
// the ring; waits (host side) only for the upload kStageRing calls back from
// that same buffer.  The device table is overwritten in stream order, after
// the graph replays enqueued before it have read it.
hipError_t stage_args(tsqr_batched_plan_s* p, tsqr::BatchArgs* const* hring, tsqr::BatchArgs* d,
                      hipEvent_t const* evring, int& next, double* const* A, const int64_t* lda, double* const* X,
                      const int64_t* ldx)
{
    const int r = next;
    next = (next + 1) % kStageRing;
    tsqr::BatchArgs* h = hring[r];
    hipEvent_t ev = evring[r];
    hipError_t e = hipEventSynchronize(ev);
    if (e != hipSuccess) return e;
    for (int i = 0; i < p->count; ++i) h[i] = tsqr::BatchArgs{A[i], lda[i], X[i], ldx[i]};
    e = hipMemcpyAsync(d, h, sizeof(tsqr::BatchArgs) * p->count, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipEventRecord(ev, p->stream);
    return e;
}

}  // namespace

extern "C" {

tsqr_status tsqr_batched_plan_create(tsqr_batched_plan* out, int count, const int64_t* m, const int64_t* n,
                                     tsqr_precision prec, const tsqr_opts* opts, void* hip_stream)
{
    if (!out) return -1;
    *out = nullptr;
    if (count < 1) return -2;
    if (!m) return -3;
    if (!n) return -4;
    const int pv = tsqr::abi_int(prec);
    if (pv != TSQR_FP64 && pv != TSQR_MIXED) return -5;
    tsqr_opts o;
    std::memset(&o, 0, sizeof(o));
    o.want_q = 1;
    if (opts) {
        o = *opts;
        const int tv = tsqr::abi_int(o.tree);
        if (tv < TSQR_TREE_AUTO || tv > TSQR_TREE_HYBRID) return -6;
        if (o.leaf_rows < 0 || o.tile_rows != 0 || o.flat_len < 0) return -6;
        if (o.waves != 0 && o.waves != 1 && o.waves != 2 && o.waves != 4) return -6;
        if (o.want_q != 0 && o.want_q != 1) return -6;
        const int kv = tsqr::abi_int(o.leaf_kind);
        if (kv != TSQR_LEAF_AUTO && kv != TSQR_LEAF_COMPACT_WY) return -6;
    }
    for (int i = 0; i < count; ++i) {
        if (n[i] < 0 || m[i] < 0 || m[i] < n[i]) return -3;
        if (n[i] > tsqr::kMaxN) return 3;
    }
    tsqr_batched_plan_s* p = new (std::nothrow) tsqr_batched_plan_s();
    if (!p) return 2;
    p->count = count;
    p->prec = prec;
    p->want_q = o.want_q;
    p->waves = o.waves;
    p->stream = (hipStream_t)hip_stream;
    const bool mixed = prec == TSQR_MIXED;
    p->L.resize(count);
    std::vector<tsqr::BatchProblem> bp(count);
    int64_t off = 0;
    for (int i = 0; i < count; ++i) {
        tsqr::Layout& L = p->L[i];
        if (n[i] == 0) {
            // an empty problem: no work items, no workspace, pointers not referenced
            L.m = m[i];
            bp[i].m = m[i];
            bp[i].ws_off = off;
            continue;
        }
        // without options, each problem takes the cached choice of its class (if any)
        tsqr_opts oi = o;
        tsqr_opts tuned;
        if (!opts && tsqr::tuned_opts(m[i], n[i], prec, 1, &tuned) && tuned.tile_rows == 0) {
            oi.tree = tuned.tree;
            oi.leaf_rows = tuned.leaf_rows;
            oi.flat_len = tuned.flat_len;
        }
        if (!tsqr::make_layout(L, m[i], n[i], oi.leaf_rows, oi.flat_len, oi.tree, oi.waves, mixed, o.want_q != 0,
                               true) ||
            L.levels >= tsqr::kBatchLevels) {
            delete p;
            return 3;
        }
        tsqr::BatchProblem& b = bp[i];
        b.m = L.m;
        b.n = (int)L.n;
        b.levels = L.levels;
        b.P = L.P;
        b.leaf_rows = L.leaf_rows;
        b.f = L.f;
        b.ws_off = off;
        b.off_T = L.off_T;
        b.off_D = L.off_D;
        for (int l = 0; l <= L.levels; ++l) {
            b.off_R[l] = L.off_R[l];
            b.off_S[l] = L.off_S[l];
            b.off_Y[l] = L.off_Y[l];
            b.off_TN[l] = L.off_TN[l];
            b.count[l] = L.count[l];
        }
        b.ld32 = L.ld32;
        b.off_V32 = L.off_V32;
        b.off_T32 = L.off_T32;
        b.off_Q1 = L.off_Q1;
        b.off_Gp = L.off_Gp;
        b.off_Gq = L.off_Gq;
        b.off_G = L.off_G;
        b.off_R1 = L.off_R1;
        b.off_R2inv = L.off_R2inv;
        b.off_info = L.off_info;
        b.gram_waves = L.gram_waves;
        b.gram_rows = L.gram_rows;
        off += L.total;
    }
    p->ws_doubles = off;

    // width classes, largest problems first inside each (the persistent grids
    // take items in order)
    std::vector<int> widths;
    for (int i = 0; i < count; ++i)
        if (p->L[i].n > 0 && std::find(widths.begin(), widths.end(), p->L[i].np) == widths.end())
            widths.push_back(p->L[i].np);
    std::sort(widths.begin(), widths.end());
    std::vector<std::vector<int64_t>> lists;  // host copies, concatenated below
    struct ClassLists {
        size_t leaf, root, level[tsqr::kBatchLevels], gram, gsum, rq;
    };
    std::vector<ClassLists> where;
    for (int np : widths) {
        std::vector<int> probs;
        for (int i = 0; i < count; ++i)
            if (p->L[i].np == np) probs.push_back(i);
        std::stable_sort(probs.begin(), probs.end(), [&](int a, int b) { return p->L[a].m > p->L[b].m; });
        tsqr::BatchClass C;
        C.np = np;
        C.nprob = (int64_t)probs.size();
        ClassLists w{};
        std::vector<int64_t> leaf, root;
        for (int i : probs) {
            for (int64_t q = 0; q < p->L[i].P; ++q) leaf.push_back(tsqr::batch_item(i, q));
            root.push_back(tsqr::batch_item(i, 0));
            C.max_levels = std::max(C.max_levels, p->L[i].levels);
        }
        C.n_leaf = (int64_t)leaf.size();
        w.leaf = lists.size();
        lists.push_back(leaf);
        w.root = lists.size();
        lists.push_back(root);
        for (int l = 1; l <= C.max_levels; ++l) {
            std::vector<int64_t> lv;
            for (int i : probs)
                if (p->L[i].levels >= l)
                    for (int64_t q = 0; q < p->L[i].count[l]; ++q) lv.push_back(tsqr::batch_item(i, q));
            C.n_level[l] = (int64_t)lv.size();
            w.level[l] = lists.size();
            lists.push_back(lv);
        }
        // mixed with Q: the second pass's items
        std::vector<int64_t> gram, gsum, rq;
        if (mixed && o.want_q) {
            for (int i : probs) {
                const tsqr::Layout& Li = p->L[i];
                for (int64_t g = 0; g < Li.gram_waves; ++g) gram.push_back(tsqr::batch_item(i, g));
                for (int64_t g = 0; g < (Li.gram_waves + 63) / 64; ++g) gsum.push_back(tsqr::batch_item(i, g));
                const int64_t nblocks = (Li.m + 15) / 16;
                for (int64_t c = 0; c < (nblocks + 63) / 64; ++c) rq.push_back(tsqr::batch_item(i, c));
            }
        }
        C.n_gram = (int64_t)gram.size();
        C.n_gsum = (int64_t)gsum.size();
        C.n_rq = (int64_t)rq.size();
        w.gram = lists.size();
        lists.push_back(gram);
        w.gsum = lists.size();
        lists.push_back(gsum);
        w.rq = lists.size();
        lists.push_back(rq);
        p->classes.push_back(C);
        where.push_back(w);
    }
    std::vector<int64_t> all;
    std::vector<size_t> start(lists.size());
    for (size_t k = 0; k < lists.size(); ++k) {
        start[k] = all.size();
        all.insert(all.end(), lists[k].begin(), lists[k].end());
    }

    hipError_t e = hipMalloc((void**)&p->ws, (size_t)std::max<int64_t>(1, p->ws_doubles) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_probs, sizeof(tsqr::BatchProblem) * count);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_items, sizeof(int64_t) * std::max<size_t>(1, all.size()));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_args_f, sizeof(tsqr::BatchArgs) * count);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_args_q, sizeof(tsqr::BatchArgs) * count);
    for (int r = 0; r < kStageRing && e == hipSuccess; ++r) {
        e = hipHostMalloc((void**)&p->h_args_f[r], sizeof(tsqr::BatchArgs) * count, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&p->h_args_q[r], sizeof(tsqr::BatchArgs) * count, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_f[r], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_q[r], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_probs, bp.data(), sizeof(tsqr::BatchProblem) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess && !all.empty())
        e = hipMemcpy(p->d_items, all.data(), sizeof(int64_t) * all.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release(p);
        return hstatus(e);
    }
    for (size_t c = 0; c < p->classes.size(); ++c) {
        tsqr::BatchClass& C = p->classes[c];
        C.leaf_items = p->d_items + start[where[c].leaf];
        C.root_items = p->d_items + start[where[c].root];
        for (int l = 1; l <= C.max_levels; ++l) C.level_items[l] = p->d_items + start[where[c].level[l]];
        C.gram_items = p->d_items + start[where[c].gram];
        C.gsum_items = p->d_items + start[where[c].gsum];
        C.rq_items = p->d_items + start[where[c].rq];
    }
    if (mixed && p->ws_doubles > 0) {
        // the FP32 workspaces are read in whole tiles and 16-column blocks: what
        // the kernels never write (rows past the last tile, columns past np) stays zero
        e = hipMemset(p->ws, 0, (size_t)p->ws_doubles * sizeof(double));
        if (e != hipSuccess) {
            release(p);
            return hstatus(e);
        }
    }
    *out = p;
    return 0;
}

tsqr_status tsqr_batched_factor(tsqr_batched_plan p, double* const* A, const int64_t* lda, double* const* R,
                                const int64_t* ldr)
{
    if (!p) return -1;
    if (!A) return -2;
    if (!lda) return -3;
    if (!R) return -4;
    if (!ldr) return -5;
    for (int i = 0; i < p->count; ++i) {
        const bool empty = p->L[i].n == 0;  // references no matrix
        if (!A[i] && !empty) return -2;
        if (lda[i] < p->L[i].m) return -3;
        if (!R[i] && !empty) return -4;
        if (ldr[i] < p->L[i].n) return -5;
    }
    p->state = 0;
    if (p->classes.empty()) {  // every problem is empty
        p->state = p->want_q ? 1 : 2;
        return 0;
    }
    hipError_t e = stage_args(p, p->h_args_f, p->d_args_f, p->ev_f, p->next_f, A, lda, R, ldr);
    // The width classes run one after another in one graph.  Measured at 2048
    // problems (n in {8, 16, 32, 64}): the classes as parallel branches of the
    // graph, and one graph per class on streams of their own, were no faster
    // in FP64 (114 ms both) and slower in mixed precision (131 and 140 ms
    // against 125): every class's persistent grid fills the device, so running
    // them together only shares it, and the 64-column class dominates.
    if (e == hipSuccess && !p->g_factor) {
        e = capture_graph(p->capture, &p->g_factor, [&](hipStream_t s) {
            for (const tsqr::BatchClass& C : p->classes) {
                const int waves = p->waves > 0 ? p->waves : (p->want_q ? 4 : 1);
                hipError_t el =
                    p->prec == TSQR_MIXED
                        ? tsqr::launch_batch_factor_mixed(C, p->d_probs, p->d_args_f, p->ws, p->want_q != 0, waves, s)
                        : tsqr::launch_batch_factor(C, p->d_probs, p->d_args_f, p->ws, p->want_q != 0, waves, s);
                if (el != hipSuccess) return el;
            }
            return hipSuccess;
        });
    }
    if (e == hipSuccess) e = hipGraphLaunch(p->g_factor, p->stream);
    if (e != hipSuccess) return hstatus(e);
    p->state = p->want_q ? 1 : 2;
    return 0;
}

tsqr_status tsqr_batched_form_q(tsqr_batched_plan p, double* const* A, const int64_t* lda, double* const* Q,
                                const int64_t* ldq)
{
    if (!p) return -1;
    if (!A) return -2;
    if (!lda) return -3;
    if (!Q) return -4;
    if (!ldq) return -5;
    for (int i = 0; i < p->count; ++i) {
        const bool empty = p->L[i].n == 0;  // references no matrix
        if (!A[i] && !empty) return -2;
        if (lda[i] < p->L[i].m) return -3;
        if (!Q[i] && !empty) return -4;
        if (ldq[i] < p->L[i].m) return -5;
        if (Q[i] == A[i] && ldq[i] != lda[i]) return -5;
    }
    if (p->state != 1) return 4;
    if (p->classes.empty()) return 0;  // every problem is empty
    // FP64: Q over A in any problem selects the graph with one wavefront per
    // leaf (MIXED plans read their reflectors from the workspace)
    bool alias = false;
    for (int i = 0; i < p->count && p->prec != TSQR_MIXED; ++i) alias = alias || (Q[i] == A[i] && p->L[i].n > 0);
    hipGraphExec_t* g = alias ? &p->g_form_q_alias : &p->g_form_q;
    hipError_t e = stage_args(p, p->h_args_q, p->d_args_q, p->ev_q, p->next_q, A, lda, Q, ldq);
    if (e == hipSuccess && !*g) {
        e = capture_graph(p->capture, g, [&](hipStream_t s) {
            for (const tsqr::BatchClass& C : p->classes) {
                const int waves = p->waves > 0 ? p->waves : (p->want_q ? 4 : 1);
                hipError_t el = p->prec == TSQR_MIXED
                                    ? tsqr::launch_batch_form_q_mixed(C, p->d_probs, p->d_args_q, p->ws, s)
                                    : tsqr::launch_batch_form_q(C, p->d_probs, p->d_args_q, p->ws, waves, alias, s);
                if (el != hipSuccess) return el;
            }
            return hipSuccess;
        });
    }
    if (e == hipSuccess) e = hipGraphLaunch(*g, p->stream);
    return hstatus(e);
}

tsqr_status tsqr_batched_problem_info(tsqr_batched_plan p, int index, tsqr_info* out)
{
    if (!p) return -1;
    if (index < 0 || index >= p->count) return -2;
    if (!out) return -3;
    const tsqr::Layout& L = p->L[index];
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
    out->precision = p->prec;
    out->workspace_bytes = L.total * (int64_t)sizeof(double);
    out->leaf_kind = TSQR_LEAF_COMPACT_WY;
    if (p->prec == TSQR_MIXED && p->want_q && p->state == 1 && L.n > 0) {
        // the second pass's check (synchronises the plan's stream)
        double info[2] = {0.0, 0.0};
        hipError_t e = hipStreamSynchronize(p->stream);
        int64_t off = 0;
        for (int i = 0; i < index; ++i) off += p->L[i].total;
        if (e == hipSuccess) e = hipMemcpy(info, p->ws + off + L.off_info, sizeof(info), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hstatus(e);
        out->orth_estimate = info[0];
        out->reorth_applied = info[1] != 0.0;
    }
    return 0;
}

tsqr_status tsqr_batched_plan_destroy(tsqr_batched_plan p)
{
    if (!p) return -1;
    hipError_t e = hipStreamSynchronize(p->stream);
    release(p);
    return hstatus(e);
}

}  // extern "C"
