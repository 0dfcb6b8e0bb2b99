// tsqr_tune.cpp -- the autotuner: per problem class (n, m bucket, precision,
// R or R+Q) it times candidate geometries on the device and keeps the fastest
// in a JSON cache that plans consult.
//
// Tunable here: the leaf length (tiles per flat chain, hence the tree:
// binary, hybrid or one flat chain) and the wavefronts per workgroup of the
// leaf and Q kernels.  The tile height is fixed by the width (it sizes the
// register-resident tile), and the panel width of the blocked leaf is one
// matrix-core block (16 columns), so neither is searched.  Accuracy guards: flat chains are capped at
// kMaxChainTiles tiles (a long flat chain accumulates rounding along the chain
// -- the flat tree is the least accurate shape), and for the mixed precision
// chains of FP32 tiles are capped at kMaxChainF32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "tsqr.h"
#include "tsqr_internal.h"

namespace {

constexpr int64_t kMaxChainTiles = 256;

// Deterministic fill of the scratch matrix: a counter-based hash of (i, j)
// mapped to [-1, 1) (the timing does not depend on the values).
__global__ void k_fill_pattern(double* A, int64_t m, int n, int64_t lda)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * n) return;
    const int64_t i = idx % m, j = idx / m;
    uint64_t x = (uint64_t)idx * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    x ^= x >> 31;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 29;
    A[i + j * lda] = (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

std::string class_key(int64_t m, int64_t n, tsqr_precision prec, int want_q)
{
    const int bucket = m > 0 ? (int)std::floor(std::log2((double)m)) : 0;
    char buf[96];
    std::snprintf(buf, sizeof(buf), "n%lld_m2e%d_%s_%s", (long long)n, bucket, prec == TSQR_MIXED ? "mixed" : "fp64",
                  want_q ? "rq" : "r");
    return buf;
}

// The cache is a JSON object {"entries": {key: {"tree": t, "leaf_rows": l,
// "flat_len": f, "waves": w, "ms": x}, ...}}; it is read and rewritten whole.
struct Entry {
    std::string key;
    tsqr_opts o;
    double ms;
};

bool parse_num(const std::string& s, size_t from, const char* name, double* out)
{
    const std::string pat = std::string("\"") + name + "\"";
    size_t k = s.find(pat, from);
    if (k == std::string::npos) return false;
    k = s.find(':', k + pat.size());
    if (k == std::string::npos) return false;
    char* end = nullptr;
    *out = std::strtod(s.c_str() + k + 1, &end);
    return end != s.c_str() + k + 1;
}

// Reads the entries of a cache file written by write_cache (a missing or
// unreadable file is an empty cache; a malformed entry ends the scan).
std::vector<Entry> read_cache(const char* path)
{
    std::vector<Entry> out;
    if (!path) return out;
    FILE* f = std::fopen(path, "rb");
    if (!f) return out;
    std::string s;
    char buf[4096];
    size_t r;
    while ((r = std::fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, r);
    std::fclose(f);
    size_t pos = s.find("\"entries\"");
    if (pos == std::string::npos) return out;
    pos = s.find('{', pos);
    if (pos == std::string::npos) return out;
    ++pos;
    auto skip = [&](size_t p) {
        while (p < s.size() && (s[p] == ' ' || s[p] == '\n' || s[p] == '\r' || s[p] == '\t' || s[p] == ',')) ++p;
        return p;
    };
    for (;;) {
        pos = skip(pos);
        if (pos >= s.size() || s[pos] != '"') break;  // '}' closes the entries
        const size_t q1 = s.find('"', pos + 1);
        if (q1 == std::string::npos) break;
        const size_t ob = s.find('{', q1);
        const size_t cb = ob == std::string::npos ? ob : s.find('}', ob);
        if (cb == std::string::npos) break;
        const std::string body = s.substr(ob, cb - ob + 1);
        Entry e;
        e.key = s.substr(pos + 1, q1 - pos - 1);
        std::memset(&e.o, 0, sizeof(e.o));
        double t = 0, l = 0, fl = 0, w = 0, q = 1, ms = 0;
        if (!(parse_num(body, 0, "tree", &t) && parse_num(body, 0, "leaf_rows", &l) &&
              parse_num(body, 0, "flat_len", &fl) && parse_num(body, 0, "waves", &w) &&
              parse_num(body, 0, "ms", &ms)))
            break;
        parse_num(body, 0, "want_q", &q);
        double lk = 0;
        parse_num(body, 0, "leaf_kind", &lk);
        pos = cb + 1;
        // an entry with a value no option can take is skipped (and nothing is
        // converted to an integer type that cannot hold it)
        auto whole_in = [](double x, double lo, double hi) { return x >= lo && x <= hi && x == std::floor(x); };
        if (!(whole_in(t, TSQR_TREE_AUTO, TSQR_TREE_HYBRID) && whole_in(lk, TSQR_LEAF_AUTO, TSQR_LEAF_RECURSIVE) &&
              whole_in(l, 0, 4.0e18) && whole_in(fl, 0, 2147483647.0) && whole_in(w, 0, 4) && whole_in(q, 0, 1)))
            continue;
        e.o.leaf_kind = (tsqr_leaf_kind)(int)lk;
        e.o.tree = (tsqr_tree)(int)t;
        e.o.leaf_rows = (int64_t)l;
        e.o.flat_len = (int)fl;
        e.o.waves = (int)w;
        e.o.want_q = (int)q;
        e.ms = ms;
        out.push_back(e);
    }
    return out;
}

bool write_cache(const char* path, const std::vector<Entry>& es)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    std::fprintf(f, "{\n  \"format\": \"tsqr autotune cache 1\",\n  \"entries\": {\n");
    for (size_t i = 0; i < es.size(); ++i) {
        const Entry& e = es[i];
        std::fprintf(f,
                     "    \"%s\": {\"tree\": %d, \"leaf_rows\": %lld, \"flat_len\": %d, \"waves\": %d, "
                     "\"want_q\": %d, \"leaf_kind\": %d, \"ms\": %.6f}%s\n",
                     e.key.c_str(), (int)e.o.tree, (long long)e.o.leaf_rows, e.o.flat_len, e.o.waves, e.o.want_q,
                     (int)e.o.leaf_kind, e.ms, i + 1 < es.size() ? "," : "");
    }
    std::fprintf(f, "  }\n}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

namespace tsqr {

// Options cached for this class, if any (used by plan creation when the
// caller passes no options and TSQR_TUNE_CACHE names a cache file).
bool tuned_opts(int64_t m, int64_t n, tsqr_precision prec, int want_q, tsqr_opts* out)
{
    const char* path = std::getenv("TSQR_TUNE_CACHE");
    if (!path || !*path) return false;
    const std::string key = class_key(m, n, prec, want_q);
    for (const Entry& e : read_cache(path))
        if (e.key == key) {
            *out = e.o;
            out->want_q = want_q;
            return true;
        }
    return false;
}

}  // namespace tsqr

extern "C" {

tsqr_status tsqr_tune_cache_lookup(const char* cache_path, int64_t m, int64_t n, tsqr_precision prec, int want_q,
                                   tsqr_opts* out, double* ms)
{
    if (!cache_path) return -1;
    if (m < 1 || m < n) return -2;
    if (n < 1) return -3;
    if (tsqr::abi_int(prec) != TSQR_FP64 && tsqr::abi_int(prec) != TSQR_MIXED) return -4;
    if (want_q != 0 && want_q != 1) return -5;
    if (!out) return -6;
    const std::string key = class_key(m, n, prec, want_q);
    for (const Entry& e : read_cache(cache_path))
        if (e.key == key) {
            *out = e.o;
            if (ms) *ms = e.ms;
            return 0;
        }
    return 5;  // not in the cache
}

tsqr_status tsqr_tune_cache_store(const char* cache_path, int64_t m, int64_t n, tsqr_precision prec,
                                  const tsqr_opts* opts, double ms)
{
    if (!cache_path) return -1;
    if (m < 1 || m < n) return -2;
    if (n < 1) return -3;
    if (tsqr::abi_int(prec) != TSQR_FP64 && tsqr::abi_int(prec) != TSQR_MIXED) return -4;
    if (!opts || (opts->want_q != 0 && opts->want_q != 1)) return -5;
    const int tv = tsqr::abi_int(opts->tree), kv = tsqr::abi_int(opts->leaf_kind);
    if (tv < TSQR_TREE_AUTO || tv > TSQR_TREE_HYBRID || kv < TSQR_LEAF_AUTO || kv > TSQR_LEAF_RECURSIVE) return -5;
    const std::string key = class_key(m, n, prec, opts->want_q);
    std::vector<Entry> es = read_cache(cache_path);
    bool found = false;
    for (Entry& e : es)
        if (e.key == key) {
            e.o = *opts;
            e.ms = ms;
            found = true;
        }
    if (!found) es.push_back(Entry{key, *opts, ms});
    return write_cache(cache_path, es) ? 0 : 1;
}

tsqr_status tsqr_autotune(int64_t m, int64_t n, tsqr_precision prec, int want_q, double* scratch, int64_t ld,
                          void* hip_stream, const char* cache_path, int reps, tsqr_tune_result* out)
{
    if (m < 1 || m < n) return -1;
    if (n < 1) return -2;
    if (n > tsqr::kMaxN) return 3;
    if (tsqr::abi_int(prec) != TSQR_FP64 && tsqr::abi_int(prec) != TSQR_MIXED) return -3;
    if (want_q != 0 && want_q != 1) return -4;
    if (scratch && ld < m) return -6;
    if (reps < 1) return -9;
    if (!out) return -10;
    std::memset(out, 0, sizeof(*out));
    if (cache_path) {
        double ms = 0;
        if (tsqr_tune_cache_lookup(cache_path, m, n, prec, want_q, &out->opts, &ms) == 0) {
            out->ms = ms;
            out->from_cache = 1;
            return 0;
        }
    }
    hipStream_t s = (hipStream_t)hip_stream;
    double* A = scratch;
    double* own = nullptr;
    if (!A) {
        ld = m;
        hipError_t e = hipMalloc((void**)&own, (size_t)m * n * sizeof(double));
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? 2 : 1;
        A = own;
    }
    // FP64 with Q: the reflectors go to V and Q is formed into its own buffer,
    // the form most callers run (Q over the reflectors in place gives each
    // leaf one wavefront above 48 columns, a slower kernel)
    double *Q = nullptr, *V = nullptr, *R = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipMalloc((void**)&R, (size_t)n * n * sizeof(double));
    if (he == hipSuccess && want_q) he = hipMalloc((void**)&Q, (size_t)m * n * sizeof(double));
    if (he == hipSuccess && want_q && prec == TSQR_FP64) he = hipMalloc((void**)&V, (size_t)m * n * sizeof(double));
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);

    // candidates: leaf lengths 1, 2, 4, ... tiles (a single flat chain last,
    // when within the guard) times 1, 2 or 4 wavefronts per workgroup, times
    // both leaf variants where the recursive one exists
    tsqr::Layout L0;
    tsqr_status st = 0;
    if (he == hipSuccess && !tsqr::make_layout(L0, m, n, 0, 0, TSQR_TREE_AUTO, 0, prec == TSQR_MIXED, want_q != 0)) st = 3;
    std::vector<tsqr_opts> cand;
    const bool two_kinds = st == 0 && prec == TSQR_FP64 && want_q && (L0.np == 16 || L0.np == 32);
    auto add = [&](tsqr_opts o) {
        if (!two_kinds) {
            cand.push_back(o);
            return;
        }
        for (tsqr_leaf_kind k : {TSQR_LEAF_COMPACT_WY, TSQR_LEAF_RECURSIVE}) {
            o.leaf_kind = k;
            cand.push_back(o);
        }
    };
    if (he == hipSuccess && st == 0) {
        const int64_t tiles = (m + L0.mt - 1) / L0.mt;
        const int64_t fmax = prec == TSQR_MIXED ? tsqr::kMaxChainF32 : kMaxChainTiles;
        for (int64_t f = 1; f <= std::min<int64_t>(tiles, fmax); f *= 2)
            for (int w : {1, 2, 4}) {
                tsqr_opts o;
                std::memset(&o, 0, sizeof(o));
                o.tree = f == 1 ? TSQR_TREE_BINARY : TSQR_TREE_HYBRID;
                o.flat_len = f == 1 ? 0 : (int)f;
                o.waves = w;
                o.want_q = want_q;
                add(o);
            }
        if (tiles <= fmax)
            for (int w : {1, 2, 4}) {
                tsqr_opts o;
                std::memset(&o, 0, sizeof(o));
                o.tree = TSQR_TREE_FLAT;
                o.waves = w;
                o.want_q = want_q;
                add(o);
            }
    }
    if (he == hipSuccess && st == 0 && !scratch) {
        const int64_t total = m * n;
        hipLaunchKernelGGL(k_fill_pattern, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, A, m, (int)n, ld);
        he = hipGetLastError();
    }
    double best = -1.0;
    for (size_t c = 0; he == hipSuccess && st == 0 && c < cand.size(); ++c) {
        tsqr_plan p = nullptr;
        const tsqr_status cs = tsqr_plan_create(&p, m, n, prec, &cand[c], s);
        if (cs == 2 || cs == 3) continue;  // does not fit or not available: not a candidate
        if (cs != 0) {
            st = cs;
            break;
        }
        double t_best = -1.0;
        for (int r = 0; r <= reps && st == 0; ++r) {  // r = 0 warms up
            he = hipEventRecord(e0, s);
            if (he == hipSuccess) st = tsqr_factor_into(p, A, ld, V, m, R, n);
            if (he == hipSuccess && st == 0 && want_q && prec == TSQR_FP64) st = tsqr_form_q(p, V, m, Q, m);
            if (he == hipSuccess && st == 0 && want_q && prec == TSQR_MIXED) st = tsqr_form_q(p, nullptr, m, Q, m);
            if (he == hipSuccess && st == 0) he = hipEventRecord(e1, s);
            if (he == hipSuccess && st == 0) he = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (he == hipSuccess && st == 0) he = hipEventElapsedTime(&ms, e0, e1);
            if (he == hipSuccess && st == 0 && r > 0 && (t_best < 0 || ms < t_best)) t_best = ms;
        }
        tsqr_plan_destroy(p);
        out->candidates += 1;
        if (st == 0 && he == hipSuccess && t_best >= 0 && (best < 0 || t_best < best)) {
            best = t_best;
            out->opts = cand[c];
            out->ms = t_best;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (Q) hipFree(Q);
    if (V) hipFree(V);
    if (R) hipFree(R);
    if (own) hipFree(own);
    if (he != hipSuccess) return he == hipErrorOutOfMemory ? 2 : 1;
    if (st != 0) return st;
    if (best < 0) return 3;
    if (cache_path && tsqr_tune_cache_store(cache_path, m, n, prec, &out->opts, out->ms) != 0) return 1;
    return 0;
}

}  // extern "C"
