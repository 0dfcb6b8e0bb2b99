/*
 * tsqr.h -- C ABI of libtsqr: TSQR (communication-avoiding Householder QR of a
 * tall-skinny matrix) on one AMD Instinct MI355X (gfx950).
 *
 * The method is that of Demmel, Grigori, Hoemmen and Langou, "Implementing
 * Communication-Optimal Parallel and Sequential QR Factorizations" (arXiv
 * 0809.2407): A = [A_0; ...; A_{P-1}] in P block rows (Sec. 2), a local
 * Householder QR per block row, the R factors combined up a reduction tree by
 * QRs of stacked triangles [R_a; R_b] (Alg. 1; structured QR of Sec. 3.1), a
 * flat chain qr([R; A_k]) inside each block row (Alg. 2), with Q kept implicit
 * as Householder reflectors plus a stored tree (Sec. 4.1 and 4.2).  Applying Q^T
 * is a reduction over that tree and applying Q is a broadcast (Sec. 4.1).
 *
 * Conventions shared by every call:
 *   - Matrices are column-major FP64 with a leading dimension (element (i, j)
 *     of A sits at A[i + j*lda]); every matrix pointer is a DEVICE pointer
 *     owned by the caller.
 *   - Every call is asynchronous on the HIP stream bound to the plan: it returns
 *     once its kernels are enqueued.  Launch errors are reported; a kernel fault
 *     surfaces at the caller's next synchronisation.
 *   - Status codes: 0 = success; -i = argument i (1-based, in the order of the
 *     prototype) is invalid (LAPACK "info" style); 1 = HIP runtime error,
 *     2 = device memory exhausted, 3 = unsupported case, 4 = call out of order
 *     (e.g. tsqr_form_q before tsqr_factor), 5 = class not in the autotune
 *     cache, 6 = size beyond the fixed scratch of tsqr_factor_r_noalloc.
 *   - NaN or Inf entries propagate; nothing checks for them.
 *   - A plan is not thread-safe.  Different plans are independent.
 *   - Householder conventions: H_j = I - tau_j v_j v_j^T with v_j(j) = 1,
 *     beta_j = -sgn(alpha_j) ||x_j||, sgn(0) = +1, tau_j = 0 when the part of the
 *     column below the pivot is exactly zero.  The returned R is sign-normalised
 *     (diag(R) >= 0): QR is unique up to these signs (Sec. 2).
 */
#ifndef TSQR_H
#define TSQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int tsqr_status;

/* Arithmetic of a plan.
 * FP64: every step in FP64.
 * MIXED: a first pass with the tile updates, the compact-WY factors T and the
 *   explicit Q1 in FP32 (the reflector scalars -- norm, beta, tau -- the running
 *   triangle R, the tree and the signs stay FP64), then a second pass in FP64
 *   that re-orthogonalises Q1: G = Q1^T Q1 with FP64 accumulation of the exact
 *   products of FP32 entries, ||G - I||_F (= ||R2^T R2 - I||_F) as the check,
 *   G = R2^T R2 by Cholesky, and when the check exceeds 1e-13,
 *   Q = Q1 R2^{-1} and R = R2 R1.  A is only read; the FP32 reflectors, Q1 and
 *   the second-pass factors live in the plan.  tsqr_factor runs both passes
 *   and returns the final R; tsqr_form_q writes the corrected Q; tsqr_apply_qt
 *   writes Q^T B for that Q (the thin factor only).  With want_q = 0 only the first pass runs and
 *   R carries the FP32 pass's accuracy.  The entries of A must lie within
 *   the FP32 range (FP64 plans rescale columns whose norms leave the FP64
 *   range).  The paper fixes no precision beyond FP64; this variant is the
 *   library's own. */
typedef enum { TSQR_FP64 = 0, TSQR_MIXED = 1 } tsqr_precision;

/* Reduction-tree shape (Sec. 2 and the list of tree shapes in Sec. 7):
 * FLAT = one chain over every tile (Alg. 2), BINARY = every tile is a leaf of the
 * binary tree (Alg. 1), HYBRID = flat chains of flat_len tiles inside each leaf,
 * binary above.  AUTO lets the library choose. */
typedef enum {
    TSQR_TREE_AUTO = 0,
    TSQR_TREE_BINARY = 1,
    TSQR_TREE_FLAT = 2,
    TSQR_TREE_HYBRID = 3
} tsqr_tree;

/* Local QR of the leaf tiles (Sec. 3.1; Sec. 7 names both variants):
 * COMPACT_WY = a tile is factored column by column (in 16-column panels whose
 *   compact-WY update runs on the matrix cores, where the width allows) and a
 *   second kernel forms each tile's T from tau and the tile's Gram;
 * RECURSIVE = Elmroth and Gustavson's recursive QR: the columns are halved down
 *   to 16-column blocks and each tile's T = [T_L, -T_L Y_L^T Y_R T_R; 0, T_R] is
 *   assembled inside the leaf kernel (FP64 with Q at padded widths 16 and 32;
 *   elsewhere it is status -5 at plan creation);
 * AUTO = COMPACT_WY (at m = 2^24, n = 32 the two take the same time: the
 *   recursive leaf is slower by what its T assembly costs, the tree beside no
 *   concurrent T kernel faster by about as much). */
typedef enum {
    TSQR_LEAF_AUTO = 0,
    TSQR_LEAF_COMPACT_WY = 1,
    TSQR_LEAF_RECURSIVE = 2
} tsqr_leaf_kind;

/* Plan options; a zero field means "choose automatically".
 *   tree       tree shape
 *   leaf_rows  rows per leaf (block row); rounded up to a multiple of tile_rows
 *   tile_rows  rows per tile; the library fixes it from n (it sizes the on-chip
 *              working set, the constraint m/P*n + n(n+1)/2 <= W of Sec. 4.2),
 *              a nonzero value must equal that size
 *   flat_len   tiles per leaf chain (HYBRID); leaf_rows wins if both are set
 *   waves      wavefronts per workgroup (1, 2 or 4)
 *   want_q     1 (default when opts == NULL): tsqr_factor keeps the reflectors
 *              in A for later tsqr_form_q / tsqr_apply_qt calls;
 *              0: R only, A is not written.
 *   leaf_kind  local QR of the leaf tiles (tsqr_leaf_kind); without Q, or on a
 *              MIXED plan, the variants coincide and it is ignored. */
typedef struct {
    tsqr_tree tree;
    int64_t leaf_rows;
    int64_t tile_rows;
    int flat_len;
    int waves;
    int want_q;
    tsqr_leaf_kind leaf_kind;
} tsqr_opts;

/* What the plan chose, and (MIXED) what the second pass measured. */
typedef struct {
    int64_t m, n;
    int64_t n_padded;        /* kernel column count: n rounded up to 4; 64 for n = 57..60 */
    int64_t tile_rows;       /* rows per tile */
    int64_t leaf_rows;       /* rows per leaf (the last leaf also takes the remainder) */
    int64_t num_leaves;      /* P */
    int64_t num_tiles;       /* tiles over all leaves */
    int tree_levels;         /* ceil(log2 P) */
    tsqr_tree tree;
    int waves;
    tsqr_precision precision;
    int64_t workspace_bytes; /* device memory the plan owns */
    int reorth_applied;      /* MIXED: 1 when the second pass corrected Q and R */
    double orth_estimate;    /* MIXED: ||R2^T R2 - I||_F of the second pass */
    tsqr_leaf_kind leaf_kind; /* the leaf variant that runs (COMPACT_WY or RECURSIVE) */
} tsqr_info;

typedef struct tsqr_plan_s* tsqr_plan;

/* Create a plan for m x n problems (n <= m, 0 <= n <= 64) on hip_stream (a
 * hipStream_t, NULL = the default stream).  The plan allocates its device
 * workspace (per-tile compact-WY factors T, per-node tree factors, seeds, signs)
 * with hipMalloc here and frees it in tsqr_plan_destroy.
 * The empty problem (n = 0, any m >= 0) gets a plan with no workspace: its
 * calls check their leading dimensions, reference no matrix (the pointers may
 * be NULL), launch nothing and return 0 (Q is m x 0, Q^T B = B).
 * Errors: -1 p NULL, -2 m < n or m < 0, -3 n < 0 or n > 64 (3 = unsupported for
 * n > 64), -4 bad precision, -5 bad option field; 2 out of memory. */
tsqr_status tsqr_plan_create(tsqr_plan* p, int64_t m, int64_t n, tsqr_precision prec,
                             const tsqr_opts* opts, void* hip_stream);

/* Factor A (m x n, lda >= m).  Writes R (n x n upper triangular, diag >= 0,
 * strictly lower part set to 0) at R[i + j*ldr], ldr >= n.  With want_q the
 * leaf reflectors overwrite A in place (below the diagonal of each tile, LAPACK
 * style, Sec. 4.2) and the tree is kept in the plan (Sec. 4.1); otherwise, and
 * on a MIXED plan, A is only read.  Errors: -1 p, -2 A NULL, -3 lda < m, -4 R NULL, -5 ldr < n. */
tsqr_status tsqr_factor(tsqr_plan p, double* A, int64_t lda, double* R, int64_t ldr);

/* As tsqr_factor, but A is only read and the reflectors go to V (m x n,
 * ldv >= m); later tsqr_form_q / tsqr_apply_qt calls take V in place of the
 * factored A.  V may equal A with ldv == lda (that is tsqr_factor).  With
 * want_q = 0, or on a MIXED plan (whose reflectors stay in the plan), V is not
 * used and may be NULL.
 * Errors: -1 p, -2 A NULL, -3 lda < m, -4 V NULL (want_q), -5 ldv < m or V == A
 * with ldv != lda, -6 R NULL, -7 ldr < n. */
tsqr_status tsqr_factor_into(tsqr_plan p, const double* A, int64_t lda, double* V, int64_t ldv, double* R,
                             int64_t ldr);

/* Explicit thin Q (m x n, ldq >= m) from the reflectors tsqr_factor left in A
 * and the plan's tree (the broadcast of Sec. 4.1).  A = Q R with Q^T Q = I.
 * Q may alias A (same pointer and same leading dimension; above 48 columns
 * that call gives each leaf one wavefront instead of two, since both would
 * read every reflector column of the rows whose Q they write).  On a MIXED plan
 * A_factored and lda are not used (Q may be the original A) and Q is Q1 R2^{-1}
 * from the second pass.
 * Errors: -1 p, -2 A NULL, -3 lda < m, -4 Q NULL, -5 ldq < m or aliasing with a
 * different leading dimension; 4 when the plan holds no factorisation with
 * reflectors. */
tsqr_status tsqr_form_q(tsqr_plan p, const double* A_factored, int64_t lda, double* Q, int64_t ldq);

/* B (m x k, ldb >= m) <- Q_full^T B in place, Q_full being the m x m orthogonal
 * factor of the tree (the reduction of Sec. 4.1).  Rows 0..n-1 become D Q^T B
 * with Q the thin factor returned by tsqr_form_q; rows n..m-1 hold coordinates
 * of B in the tree's basis of the orthogonal complement (they depend on the
 * tree).  k = 0 returns 0 at once (B may then be NULL, as when m = 0).  Right-hand sides are
 * processed 32 at a time.  On a MIXED plan Q is Q1 R2^{-1}, which has no
 * complement: rows 0..n-1 become Q^T B = R2^{-T} (Q1^T B) (Q1^T B summed in
 * FP64 over 64-row groups, pairwise, like the second pass's Gram), rows n..m-1
 * are left as they are, and A_factored and lda are not used (A_factored may
 * be NULL).  Errors: -1 p, -2 A NULL, -3 lda < m, -4 k < 0, -5 B NULL,
 * -6 ldb < m; 4 when the plan holds no factorisation with reflectors. */
tsqr_status tsqr_apply_qt(tsqr_plan p, const double* A_factored, int64_t lda, int64_t k, double* B,
                          int64_t ldb);

/* MIXED plans: copy the first-pass Q1 (m x n FP32, ldq1 >= m, device memory)
 * as it was before the second pass corrected it, e.g. to check the plan's
 * orth_estimate against ||Q1^T Q1 - I||_F.  Asynchronous on the plan's stream.
 * Errors: -1 p, -2 Q1 NULL, -3 ldq1 < m; 3 for an FP64 plan; 4 when the plan
 * holds no factorisation with Q. */
tsqr_status tsqr_mixed_q1(tsqr_plan p, float* Q1, int64_t ldq1);

/* What tsqr_plan_create would choose for these arguments, without allocating
 * anything or touching a device (workspace_bytes tells the device memory a
 * plan would own).  Errors: -1 m, -2 n, -3 prec, -4 opts (the checks of
 * tsqr_plan_create), -5 out NULL; 3 unsupported case. */
tsqr_status tsqr_plan_query(int64_t m, int64_t n, tsqr_precision prec, const tsqr_opts* opts, tsqr_info* out);

/* Copy what the plan chose (and what a MIXED run measured; reading those two
 * fields synchronises the plan's stream).  Errors: -1 p, -2 out NULL. */
tsqr_status tsqr_plan_info(tsqr_plan p, tsqr_info* out);

/* Per-phase device time.  With profiling on, every kernel phase a call enqueues
 * is bracketed by HIP events on the plan's stream. */
typedef enum {
    TSQR_PHASE_LEAF = 0,    /* leaf chains: local QRs of every tile (tsqr_factor) */
    TSQR_PHASE_TREE = 1,    /* binary-tree levels over the leaf R factors */
    TSQR_PHASE_ROOT = 2,    /* sign normalisation and R output */
    TSQR_PHASE_SEEDS = 3,   /* top-down seed descent of tsqr_form_q */
    TSQR_PHASE_FORM_Q = 4,  /* per-tile Q expansion of tsqr_form_q */
    TSQR_PHASE_APPLY = 5,   /* tsqr_apply_qt */
    TSQR_PHASE_Q1 = 6,      /* MIXED: the FP32 first-pass Q1 (inside tsqr_factor) */
    TSQR_PHASE_REORTH = 7,  /* MIXED: second pass -- Gram, check, Cholesky, R = R2 R1 */
    TSQR_PHASE_LEAF_T = 8,  /* plans with Q: the compact-WY T of every leaf tile (Sec. 3.2) */
    TSQR_NUM_PHASES = 9
} tsqr_phase;

typedef struct {
    double ms[TSQR_NUM_PHASES];     /* summed device milliseconds per phase */
    int64_t calls[TSQR_NUM_PHASES]; /* how many times each phase ran */
} tsqr_timings;

/* Turn per-phase event timing on (1) or off (0).  Turning it on clears the sums.
 * Errors: -1 p, -2 bad flag; 1 when the events cannot be created. */
tsqr_status tsqr_plan_profile(tsqr_plan p, int enable);

/* Sums since profiling was turned on (synchronises the plan's stream).
 * Errors: -1 p, -2 out NULL; 1 HIP error. */
tsqr_status tsqr_plan_timings(tsqr_plan p, tsqr_timings* out);

/* Free the plan and its workspace (synchronises its stream first).  The plan
 * is freed whatever the status: a HIP error of earlier work on the stream is
 * reported, but p must not be used or destroyed again.  Errors: -1 p; 1 HIP. */
tsqr_status tsqr_plan_destroy(tsqr_plan p);

/* ---- Autotuner --------------------------------------------------------------
 * Per problem class -- n, the m bucket floor(log2 m), the precision, and R
 * only or R + Q -- the tuner times candidate geometries on the device and keeps
 * the fastest: the leaf length (tiles per flat chain: 1 = binary tree over the
 * tiles, longer = hybrid, every tile = one flat chain) and the wavefronts per
 * workgroup of the leaf and Q kernels (1, 2 or 4).  The tile height is fixed
 * by n (it sizes the register-resident tile) and the leaf update is
 * unblocked, so neither is searched.  Accuracy guard: chains (and the flat
 * tree) are capped at 256 tiles (64 for the FP32 tiles of MIXED plans),
 * since rounding accumulates along a chain
 * (the flat tree is the least accurate shape of Sec. 2).  The choice of the
 * best tree is left open by the paper; this search is the library's own.
 *
 * Results are cached in a JSON file ({"entries": {class: {"tree", "leaf_rows",
 * "flat_len", "waves", "want_q", "ms"}}}).  tsqr_plan_create and
 * tsqr_batched_plan_create called with opts == NULL take the cached options of
 * their class when the environment variable TSQR_TUNE_CACHE names such a
 * file. */
typedef struct {
    tsqr_opts opts;  /* the fastest candidate (or the cached one) */
    double ms;       /* its device time for one factorisation (+ explicit Q) */
    int candidates;  /* candidates timed (0 when read from the cache) */
    int from_cache;  /* 1 when the class was found in the cache */
} tsqr_tune_result;

/* Tune the class of (m, n, prec, want_q).  scratch (m x n, ld >= m, device) is
 * only read; NULL makes the tuner allocate and fill its own.  With Q, an FP64
 * candidate is timed writing its reflectors to a buffer of their own and Q to
 * another (not Q over the reflectors in place, which above 48 columns runs a
 * slower kernel), so the tuner allocates up to three m x n matrices.  Each candidate
 * runs reps + 1 times (the first untimed) on hip_stream; the call
 * synchronises.  With cache_path, a cached class is returned at once and a
 * tuned one is stored.  Errors: -1 m, -2 n, -3 prec, -4 want_q, -6 ld < m,
 * -9 reps < 1, -10 out NULL; 3 n > 64 or no candidate ran; 1 HIP error or an
 * unwritable cache. */
tsqr_status tsqr_autotune(int64_t m, int64_t n, tsqr_precision prec, int want_q, double* scratch, int64_t ld,
                          void* hip_stream, const char* cache_path, int reps, tsqr_tune_result* out);

/* Cached options of the class of (m, n, prec, want_q), and their time when ms
 * is not NULL.  Host only.  Errors: -1 path NULL, -2 m, -3 n, -4 prec,
 * -5 want_q, -6 out NULL; 5 when the class is not in the cache.  A cache entry
 * whose values no option can take (a tree or leaf kind out of range, a
 * fractional or negative count) is skipped as if absent. */
tsqr_status tsqr_tune_cache_lookup(const char* cache_path, int64_t m, int64_t n, tsqr_precision prec, int want_q,
                                   tsqr_opts* out, double* ms);

/* Store (or replace) the options of a class in the cache file.  Host only.
 * Errors: -1 path NULL, -2 m, -3 n, -4 prec, -5 opts NULL, bad want_q or a
 * tree or leaf kind out of range; 1 when the file cannot be written. */
tsqr_status tsqr_tune_cache_store(const char* cache_path, int64_t m, int64_t n, tsqr_precision prec,
                                  const tsqr_opts* opts, double ms);

/* ---- Batched plans --------------------------------------------------------
 * Many independent problems (A_i m_i x n_i, n_i <= 64) factored together: the
 * library's own batched launch, not a construct of the paper, which treats one
 * matrix.  Each problem gets the single-problem method (leaf chains, binary
 * tree over the leaves, sign normalisation; the explicit Q by the seed
 * broadcast) and the results of a single plan with the same leaf rows
 * (tsqr_batched_problem_info reports them; a small problem in a batch keeps
 * longer leaf chains than a plan of its own would choose, since the other
 * problems supply the parallelism).  Problems of one padded width share every
 * launch: persistent kernels walk device work lists of (problem, leaf) and
 * (problem, tree node) items, one launch per phase and tree level, and the
 * whole sequence is captured once into a HIP graph that each call replays
 * (one small pointer upload and one graph launch on the plan's stream; the
 * host waits only when more than four calls of a kind are still queued, for a
 * pinned staging buffer of the upload to come free).  MIXED batched plans run the mixed path the same way
 * (FP32 first pass, FP64 second pass per problem inside the same graphs) with
 * the results of single MIXED plans; tsqr_batched_problem_info then reports
 * each problem's check (and synchronises the plan's stream).  opts apply to
 * every problem (tile_rows must be 0; the batched kernels run the compact-WY
 * leaf, so leaf_kind must be AUTO or COMPACT_WY). */
typedef struct tsqr_batched_plan_s* tsqr_batched_plan;

/* count problems with sizes m[i] x n[i] (host arrays).  An empty problem
 * (n[i] = 0) takes no work and no workspace, and its pointers may be NULL.
 * Errors: -1 p NULL, -2 count < 1, -3 m NULL or some m[i] < n[i] or m[i] < 0
 * or n[i] < 0, -4 n NULL, -5 bad precision, -6 bad option field; 3 n[i] > 64
 * or a tree too deep; 2 out of memory. */
tsqr_status tsqr_batched_plan_create(tsqr_batched_plan* p, int count, const int64_t* m, const int64_t* n,
                                     tsqr_precision prec, const tsqr_opts* opts, void* hip_stream);

/* Factor every A[i] (device pointer, lda[i] >= m[i]; host arrays of pointers
 * and leading dimensions) and write R[i] (n[i] x n[i], ldr[i] >= n[i]).  With
 * want_q the reflectors overwrite A[i] as in tsqr_factor.  Errors: -1 p, -2 A
 * or some A[i] NULL, -3 lda or some lda[i] < m[i], -4 R or some R[i] NULL,
 * -5 ldr or some ldr[i] < n[i]. */
tsqr_status tsqr_batched_factor(tsqr_batched_plan p, double* const* A, const int64_t* lda, double* const* R,
                                const int64_t* ldr);

/* Explicit thin Q[i] (m[i] x n[i], ldq[i] >= m[i]) of every problem from its
 * factored A[i]; Q[i] may alias A[i] with the same leading dimension (a call
 * with some Q[i] == A[i] replays a second graph, captured on first use, that
 * gives each leaf one wavefront: above 48 columns the other graph splits a
 * leaf's columns over two wavefronts, which both read all of its reflectors).
 * Errors as tsqr_batched_factor (-4 Q, -5 ldq or aliasing with another
 * leading dimension); 4 when no factorisation with reflectors was done. */
tsqr_status tsqr_batched_form_q(tsqr_batched_plan p, double* const* A, const int64_t* lda, double* const* Q,
                                const int64_t* ldq);

/* What the plan chose for problem `index`.  Errors: -1 p, -2 index, -3 out. */
tsqr_status tsqr_batched_problem_info(tsqr_batched_plan p, int index, tsqr_info* out);

/* Free the batched plan (synchronises its stream first).  Freed whatever the
 * status, as for tsqr_plan_destroy.  Errors: -1 p; 1 HIP. */
tsqr_status tsqr_batched_plan_destroy(tsqr_batched_plan p);

/* ---- Out-of-HBM TSQR ---------------------------------------------------------
 * A matrix that lives in HOST memory, factored by streaming it through the
 * GPU in blocks of block_rows rows: the out-of-DRAM sequential TSQR of
 * Sec. 7.1 (Alg. 2) one level up the memory hierarchy, with HBM as the fast
 * memory.  A flat tree over the blocks: R_0 from A_0, then R_k =
 * qr([R_{k-1}; A_k]), each stacked block factored on the device by this
 * library's TSQR (R only).  Two device buffers of (n + block_rows) x n
 * doubles: block k + 1 is copied in on a copy stream of the plan's own while
 * block k is factored on hip_stream.  A last block of fewer than n rows joins
 * the one before it.  block_rows = 0 chooses blocks of about 1 GiB. */
typedef struct tsqr_stream_plan_s* tsqr_stream_plan;

/* Errors: -1 p NULL, -2 m < 1 or m < n, -3 n < 1 (3 for n > 64), -4
 * 0 < block_rows < n; 2 out of device memory. */
tsqr_status tsqr_stream_plan_create(tsqr_stream_plan* p, int64_t m, int64_t n, int64_t block_rows,
                                    void* hip_stream);

/* R (n x n, ldr >= n, DEVICE memory, sign-normalised upper triangular) of A
 * (m x n, lda >= m, HOST memory, only read; pinned memory lets the copies run
 * asynchronously, pageable memory is copied through staging buffers).
 * Asynchronous on hip_stream: A must stay valid until the stream has passed
 * the call.  Errors: -1 p, -2 A NULL, -3 lda < m, -4 R NULL, -5 ldr < n. */
tsqr_status tsqr_stream_factor(tsqr_stream_plan p, const double* A, int64_t lda, double* R, int64_t ldr);

/* The rows per block and the block count the plan uses.  Errors: -1 p,
 * -2 block_rows NULL, -3 nblocks NULL. */
tsqr_status tsqr_stream_plan_info(tsqr_stream_plan p, int64_t* block_rows, int64_t* nblocks);

/* Free the plan (synchronises its streams).  Errors: -1 p; 1 HIP error. */
tsqr_status tsqr_stream_plan_destroy(tsqr_stream_plan p);

/* ---- CAQR: general m x n matrices (Sec. 6, Alg. 3) ---------------------------
 * The QR factorization of an m x n matrix (m >= n, any n) by panels of
 * `panel` columns (at most 64; 0 = 32), right-looking: panel j (the active
 * rows jb .. m-1) is factored by TSQR, then Q_j^T -- the leaf updates and the
 * updates up the panel's reduction tree (Sec. 3.2) -- is applied to the
 * trailing columns, whose top rows become R's row block and whose other rows
 * are the next active matrix.  One TSQR plan per panel (created here).  Q
 * stays implicit: the reflectors overwrite A panel by panel, the trees stay
 * in the plan; tsqr_caqr_apply_qt applies Q^T. */
typedef struct tsqr_caqr_plan_s* tsqr_caqr_plan;

/* n = 0 (any m >= 0) gives a plan with no panels, whose calls reference no
 * matrix and return 0.  Errors: -1 p NULL, -2 m < 0 or m < n, -3 n < 0,
 * -4 panel < 0 or > 64; 2 out of memory. */
tsqr_status tsqr_caqr_plan_create(tsqr_caqr_plan* p, int64_t m, int64_t n, int64_t panel, void* hip_stream);

/* Factor A (m x n, lda >= m, device; overwritten by the panels' reflectors
 * and, above them, R's row blocks) and write R (n x n, ldr >= n, device:
 * upper triangular, diag >= 0, strictly lower part zero).  Asynchronous.
 * Errors: -1 p, -2 A NULL, -3 lda < m, -4 R NULL, -5 ldr < n. */
tsqr_status tsqr_caqr_factor(tsqr_caqr_plan p, double* A, int64_t lda, double* R, int64_t ldr);

/* tsqr_caqr_factor with k right-hand sides carried along (Alg. 3 on the
 * augmented matrix [A B]): the k columns that follow A's n columns in the
 * same array (B = A + n lda, leading dimension lda, so the array holds
 * n + k columns) join each panel's trailing update, one pass of Q_j^T over
 * both, and on return hold Q^T B: the values tsqr_caqr_apply_qt gives after
 * tsqr_caqr_factor, with n/b fewer passes up the panels' trees.  k = 0 is
 * tsqr_caqr_factor.  Asynchronous.  Errors: as tsqr_caqr_factor, and -6
 * k < 0. */
tsqr_status tsqr_caqr_factor_rhs(tsqr_caqr_plan p, double* A, int64_t lda, double* R, int64_t ldr, int64_t k);

/* B (m x k, ldb >= m, device) <- Q^T B in place, Q = Q_0 diag(I, Q_1) ... the
 * orthogonal factor of the last tsqr_caqr_factor (A_factored its output).
 * Rows 0..n-1 become D Q_thin^T B (D the signs that made diag(R) >= 0); the
 * others hold coordinates in the panels' bases of the complement.  k = 0
 * returns at once.  Errors: -1 p, -2 A NULL, -3 lda < m, -4 k < 0, -5 B NULL,
 * -6 ldb < m; 4 before a factorisation. */
tsqr_status tsqr_caqr_apply_qt(tsqr_caqr_plan p, const double* A_factored, int64_t lda, int64_t k, double* B,
                               int64_t ldb);

/* The panel width and the number of panels.  Errors: -1 p, -2 / -3 NULL. */
tsqr_status tsqr_caqr_plan_info(tsqr_caqr_plan p, int64_t* panel, int64_t* npanels);

/* Free the plan and its panel plans (synchronises the stream).  Errors: -1 p; 1 HIP. */
tsqr_status tsqr_caqr_plan_destroy(tsqr_caqr_plan p);

/* ---- Comparison methods (Sec. 5) ----------------------------------------------
 * TSQR's competitors, for the stability and cost contrast the paper draws:
 *   CHOLQR   CholeskyQR: G = A^T A, G = R^T R (Cholesky), Q = A R^{-1}; one
 *            reduction, but the orthogonality of Q degrades with kappa(A)^2
 *            and the factorisation breaks down once kappa(A)^2 eps ~ 1;
 *   CHOLQR2  CholeskyQR applied to A and then to its Q, R = R2 R1 (not in the
 *            paper: the usual repair of CholeskyQR, orthogonal to working
 *            precision while kappa(A)^2 eps < 1);
 *   CGS      classical Gram-Schmidt: r_ij = q_i^T a_j (i < j), q_j = the
 *            normalised a_j - sum r_ij q_i;
 *   MGS      modified Gram-Schmidt: q_j = v_j / ||v_j||, then
 *            v_k -= (q_j^T v_k) q_j for every later k (loss of orthogonality
 *            about kappa eps).
 * All FP64 and without pivoting.  Q (m x n, ldq >= m) is explicit and may
 * alias A (same leading dimension: A is then overwritten); R (n x n,
 * ldr >= n) is upper triangular with a positive diagonal.  A breakdown (a
 * Cholesky pivot that is not positive; a zero norm in Gram-Schmidt) is
 * recorded on the device, Q and R are then not meaningful, and
 * tsqr_cmp_breakdown reports it.  Plans own their workspace (hipMalloc in
 * create, hipFree in destroy) and are bound to (m, n, method, stream). */
typedef enum {
    TSQR_CMP_CHOLQR = 0,
    TSQR_CMP_CHOLQR2 = 1,
    TSQR_CMP_CGS = 2,
    TSQR_CMP_MGS = 3
} tsqr_cmp_method;

typedef struct tsqr_cmp_plan_s* tsqr_cmp_plan;

/* Errors: -1 p NULL, -2 m < 1 or m < n, -3 n < 1 (3 for n > 64), -4 bad
 * method; 2 out of memory. */
tsqr_status tsqr_cmp_plan_create(tsqr_cmp_plan* p, int64_t m, int64_t n, tsqr_cmp_method method, void* hip_stream);

/* Q and R of A (m x n, lda >= m) by the plan's method; asynchronous.
 * Errors: -1 p, -2 A NULL, -3 lda < m, -4 Q NULL, -5 ldq < m or Q == A with
 * ldq != lda, -6 R NULL, -7 ldr < n. */
tsqr_status tsqr_cmp_factor(tsqr_cmp_plan p, const double* A, int64_t lda, double* Q, int64_t ldq, double* R,
                            int64_t ldr);

/* The breakdown of the last tsqr_cmp_factor: *column = 0 when none, else
 * j + 1 for the first column j where the method broke down (synchronises
 * the plan's stream).  Errors: -1 p, -2 column NULL; 1 HIP error. */
tsqr_status tsqr_cmp_breakdown(tsqr_cmp_plan p, int* column);

/* Free the plan (synchronises its stream).  Errors: -1 p; 1 HIP error. */
tsqr_status tsqr_cmp_plan_destroy(tsqr_cmp_plan p);

/* ---- Allocation-free entry point ------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The FP64
 * R-only factorisation of tsqr_factor with want_q = 0 (leaf chains, binary
 * tree over the leaves, sign normalisation; the same kernels) without a plan:
 * its workspace (the R factors of every tree level, the signs) lives in a
 * fixed 64 MiB device array of the library, of which each GPU holds one copy
 * until the process ends.  The call allocates nothing and needs no set-up;
 * its first call on a device looks the array's address up.
 *   m x n A (lda >= m, device) is only read; R (n x n, ldr >= n, device)
 *   receives the sign-normalised upper-triangular factor (strictly lower part
 *   zero).  Asynchronous on hip_stream, which must belong to the current
 *   device.  info (host, may be NULL) receives the geometry chosen.
 * Geometry: 16384 leaves (as R-only plans) or fewer, longer chains when their
 * R factors would not fit the array; chains of more than 256 tiles are
 * refused with status 6 (at 64 columns that is m above about 2^24 rows, at
 * 32 columns about 2^27).  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other host threads) race.
 * n = 0 returns 0 at once (A and R may then be NULL).
 * Errors: -1 m < 0 or m < n, -2 n < 0 (3 for n > 64), -3 A NULL, -4 lda < m,
 * -5 R NULL, -6 ldr < n; 6 beyond the array; 1 HIP error. */
tsqr_status tsqr_factor_r_noalloc(int64_t m, int64_t n, const double* A, int64_t lda, double* R, int64_t ldr,
                                  void* hip_stream, tsqr_info* info);

/* Static, human-readable text for a status code. */
const char* tsqr_status_string(tsqr_status s);

/* Library version as major*10000 + minor*100 + patch. */
int tsqr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TSQR_H */
