/*
 * tsqr_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle for TSQR.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or call
 * this file: only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or helper with the GPU
 * library; the two are compared element by element on the same seeded inputs.
 *
 * What is computed (Demmel, Grigori, Hoemmen, Langou, "Implementing
 * Communication-Optimal Parallel and Sequential QR Factorizations"):
 *
 *   - the plain Householder QR of one block (the "local QR" that every node of the
 *     reduction tree performs; Sec. 4.2, Alg. 1 step 1 and Alg. 2 step 2),
 *   - TSQR on a hybrid tree: each leaf (a block row, Sec. 2) is reduced by a flat
 *     chain over its tiles, i.e. qr(A_0), then qr([R; A_k]) for k = 1.. (Alg. 2,
 *     eq. "seq4:final"), and the leaf R factors are combined on a binary tree by
 *     qr([R_a; R_b]) with the lower index on top and an odd node passed up
 *     unchanged (Alg. 1, eq. "par4:final").  leaf_rows >= m gives the flat tree,
 *     tile_rows == leaf_rows gives the binary tree.
 *   - the explicit thin Q, as the product of the stored factors applied to [D; 0]
 *     from the root down (Sec. 2: the thin Q is the product of the block-diagonal
 *     factors times [I; 0]; applying Q is a broadcast, Sec. 4.1),
 *   - Q^T B, applying the stored factors bottom-up (applying Q^T is a reduction,
 *     Sec. 4.1).
 *
 * Conventions (the paper fixes none of them beyond "Householder vectors below the
 * diagonal, tau stored separately", Sec. 4.2):
 *   H_j = I - tau_j v_j v_j^T, v_j(j) = 1, beta_j = -sgn(alpha_j) ||x_j||,
 *   tau_j = (beta_j - alpha_j) / beta_j, sgn(0) = +1; when the part of the column
 *   below the pivot is exactly zero, tau_j = 0 and H_j = I.
 *   After the reduction R is sign-normalised: D = diag(sgn(R_jj)), R <- D R,
 *   Q <- Q D (QR is unique up to these signs, Sec. 2).
 *
 * Every matrix is column-major with a leading dimension.  Tree nodes use a dense
 * Householder QR of the stacked matrix: the zeros of the stacked triangles make
 * the reflectors come out with the [I; upper-triangular] structure of eq.
 * "fact_2rs" by themselves, without any special code.
 *
 * Parallelism: OpenMP across leaves and across the nodes of one tree level.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* Test-only switch that plants a known mistake, so that the test-suite can show
 * that its pins catch it.  0 = the correct oracle. */
static int g_mutation = 0;
void orc_set_mutation(int code) { g_mutation = code; }
int orc_get_mutation(void) { return g_mutation; }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

static double sgn(double x) { return x < 0.0 ? -1.0 : 1.0; }

/* ------------------------------------------------------------------------- */
/* Local Householder QR of one m x n block, in place (LAPACK dgeqr2 layout).   */
/* Reflector j is generated for j < min(m, n).                                */
/* ------------------------------------------------------------------------- */
void orc_householder_qr(int64_t m, int64_t n, double* A, int64_t lda, double* tau)
{
    int64_t r = m < n ? m : n;
    for (int64_t j = 0; j < r; ++j) {
        double alpha = A[IDX(j, j, lda)];
        double s = 0.0;
        for (int64_t i = j + 1; i < m; ++i) s += A[IDX(i, j, lda)] * A[IDX(i, j, lda)];
        if (s == 0.0) {
            tau[j] = 0.0;
            for (int64_t i = j + 1; i < m; ++i) A[IDX(i, j, lda)] = 0.0;
            continue;
        }
        double norm = sqrt(alpha * alpha + s);
        double beta = -sgn(alpha) * norm;
        if (g_mutation == 2) tau[j] = (alpha - beta) / beta; /* planted: wrong sign */
        else tau[j] = (beta - alpha) / beta;
        double scale = 1.0 / (alpha - beta);
        for (int64_t i = j + 1; i < m; ++i) A[IDX(i, j, lda)] *= scale;
        A[IDX(j, j, lda)] = beta;
        for (int64_t c = j + 1; c < n; ++c) {
            double w = (g_mutation == 1) ? 0.0 : A[IDX(j, c, lda)]; /* planted: drop pivot term */
            for (int64_t i = j + 1; i < m; ++i) w += A[IDX(i, j, lda)] * A[IDX(i, c, lda)];
            double tw = tau[j] * w;
            A[IDX(j, c, lda)] -= tw;
            for (int64_t i = j + 1; i < m; ++i) A[IDX(i, c, lda)] -= tw * A[IDX(i, j, lda)];
        }
    }
}

/* X (m x k) <- H_0 H_1 ... H_{r-1} X : applies Q of a factored block. */
void orc_apply_q(int64_t m, int64_t n, const double* V, int64_t ldv, const double* tau,
                 int64_t k, double* X, int64_t ldx)
{
    int64_t r = m < n ? m : n;
    for (int64_t j = r - 1; j >= 0; --j) {
        if (tau[j] == 0.0) continue;
        for (int64_t c = 0; c < k; ++c) {
            double w = X[IDX(j, c, ldx)];
            for (int64_t i = j + 1; i < m; ++i) w += V[IDX(i, j, ldv)] * X[IDX(i, c, ldx)];
            double tw = tau[j] * w;
            X[IDX(j, c, ldx)] -= tw;
            for (int64_t i = j + 1; i < m; ++i) X[IDX(i, c, ldx)] -= tw * V[IDX(i, j, ldv)];
        }
    }
}

/* X (m x k) <- H_{r-1} ... H_1 H_0 X : applies Q^T of a factored block. */
void orc_apply_qt(int64_t m, int64_t n, const double* V, int64_t ldv, const double* tau,
                  int64_t k, double* X, int64_t ldx)
{
    if (g_mutation == 6) { orc_apply_q(m, n, V, ldv, tau, k, X, ldx); return; } /* planted */
    int64_t r = m < n ? m : n;
    for (int64_t j = 0; j < r; ++j) {
        if (tau[j] == 0.0) continue;
        for (int64_t c = 0; c < k; ++c) {
            double w = X[IDX(j, c, ldx)];
            for (int64_t i = j + 1; i < m; ++i) w += V[IDX(i, j, ldv)] * X[IDX(i, c, ldx)];
            double tw = tau[j] * w;
            X[IDX(j, c, ldx)] -= tw;
            for (int64_t i = j + 1; i < m; ++i) X[IDX(i, c, ldx)] -= tw * V[IDX(i, j, ldv)];
        }
    }
}

/* Sign-normalisation: d[j] = sgn(R_jj), R <- D R, strictly lower part set to 0. */
static void sign_normalise(int64_t n, const double* Rin, int64_t ldin, double* d, double* R, int64_t ldr)
{
    for (int64_t j = 0; j < n; ++j) d[j] = sgn(Rin[IDX(j, j, ldin)]);
    for (int64_t c = 0; c < n; ++c)
        for (int64_t i = 0; i < n; ++i) {
            double v = (i <= c) ? Rin[IDX(i, c, ldin)] : 0.0;
            if (g_mutation == 5) R[IDX(i, c, ldr)] = d[c] * v; /* planted: scales columns */
            else R[IDX(i, c, ldr)] = d[i] * v;
        }
}

/* Reference result (the plain definition): one Householder QR of the whole
 * matrix, sign-normalised.  R is n x n; Q (optional) is the thin m x n factor. */
int orc_qr_reference(int64_t m, int64_t n, const double* A, int64_t lda, double* R, int64_t ldr,
                     double* Q, int64_t ldq)
{
    if (m < n || n < 1) return -1;
    double* W = (double*)malloc(sizeof(double) * (size_t)m * (size_t)n);
    double* tau = (double*)malloc(sizeof(double) * (size_t)n);
    double* d = (double*)malloc(sizeof(double) * (size_t)n);
    if (!W || !tau || !d) { free(W); free(tau); free(d); return -2; }
    for (int64_t c = 0; c < n; ++c) memcpy(W + IDX(0, c, m), A + IDX(0, c, lda), sizeof(double) * (size_t)m);
    orc_householder_qr(m, n, W, m, tau);
    sign_normalise(n, W, m, d, R, ldr);
    if (Q) {
        for (int64_t c = 0; c < n; ++c) {
            for (int64_t i = 0; i < m; ++i) Q[IDX(i, c, ldq)] = 0.0;
            Q[IDX(c, c, ldq)] = d[c];
        }
        orc_apply_q(m, n, W, m, tau, n, Q, ldq);
    }
    free(W); free(tau); free(d);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* TSQR on the hybrid tree.                                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t rows;  /* rows of the stacked matrix factored at this stage */
    double* V;     /* rows x n, column-major, ld = rows: R on and above the diagonal, v below */
    double* tau;   /* n */
} stage_t;

typedef struct {
    int64_t row0, rows;   /* rows of A owned by the leaf */
    int64_t ntiles;
    stage_t* st;          /* st[0] = qr(A_0); st[k] = qr([R; A_k]) */
} leaf_t;

typedef struct {
    int pass;             /* 1: odd node passed up unchanged (Q = I) */
    stage_t st;           /* qr([R_a; R_b]) when pass == 0 */
    int64_t home_a, home_b; /* first leaf of the left and right subtree */
} node_t;

static void stage_alloc(stage_t* s, int64_t rows, int64_t n)
{
    s->rows = rows;
    s->V = (double*)calloc((size_t)rows * (size_t)n, sizeof(double));
    s->tau = (double*)calloc((size_t)n, sizeof(double));
}
static void stage_free(stage_t* s) { free(s->V); free(s->tau); s->V = s->tau = NULL; }

/* Leaf partition: P = max(1, floor(m / leaf_rows)) leaves; leaf i owns rows
 * [i*leaf_rows, (i+1)*leaf_rows) and the last leaf also owns the remainder. */
int64_t orc_num_leaves(int64_t m, int64_t leaf_rows)
{
    int64_t P = leaf_rows > 0 ? m / leaf_rows : 1;
    return P < 1 ? 1 : P;
}

/* Number of tree levels and the node count of each level (binary pairing). */
int orc_tree_levels(int64_t P, int64_t* counts, int max_levels)
{
    int L = 0;
    int64_t c = P;
    while (c > 1 && L < max_levels) {
        c = (c + 1) / 2;
        if (counts) counts[L] = c;
        ++L;
    }
    return L;
}

/* The R factor of a stage: upper n x n of its V array. */
static void stage_R(const stage_t* s, int64_t n, double* R /* n x n, ld n */)
{
    for (int64_t c = 0; c < n; ++c)
        for (int64_t i = 0; i < n; ++i) R[IDX(i, c, n)] = (i <= c) ? s->V[IDX(i, c, s->rows)] : 0.0;
}

static void factor_leaf(leaf_t* lf, int64_t n, const double* A, int64_t lda, int64_t tile_rows)
{
    int64_t rows = lf->rows;
    int64_t T = (rows + tile_rows - 1) / tile_rows;
    lf->ntiles = T;
    lf->st = (stage_t*)calloc((size_t)T, sizeof(stage_t));
    double* R = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
    for (int64_t k = 0; k < T; ++k) {
        int64_t t0 = lf->row0 + k * tile_rows;
        int64_t mk = (k == T - 1) ? (lf->row0 + rows - t0) : tile_rows;
        stage_t* s = &lf->st[k];
        if (k == 0) {
            stage_alloc(s, mk, n);
            for (int64_t c = 0; c < n; ++c)
                for (int64_t i = 0; i < mk; ++i) s->V[IDX(i, c, mk)] = A[IDX(t0 + i, c, lda)];
        } else {
            stage_alloc(s, n + mk, n);
            for (int64_t c = 0; c < n; ++c) {
                for (int64_t i = 0; i < n; ++i) s->V[IDX(i, c, n + mk)] = R[IDX(i, c, n)];
                for (int64_t i = 0; i < mk; ++i) s->V[IDX(n + i, c, n + mk)] = A[IDX(t0 + i, c, lda)];
            }
        }
        orc_householder_qr(s->rows, n, s->V, s->rows, s->tau);
        stage_R(s, n, R);
    }
    free(R);
}

struct orc_tsqr_state {
    int64_t m, n, P;
    leaf_t* leaves;
    int L;                 /* tree levels */
    int64_t* count;        /* count[l] = nodes at level l+1 */
    node_t** nodes;        /* nodes[l][i] */
    double* Rroot;         /* n x n before normalisation */
    double* d;             /* signs */
};
typedef struct orc_tsqr_state orc_tsqr_state;

/* Factor: leaves (flat chains), then the binary tree. */
orc_tsqr_state* orc_tsqr_factor(int64_t m, int64_t n, const double* A, int64_t lda,
                                int64_t leaf_rows, int64_t tile_rows)
{
    if (m < n || n < 1 || leaf_rows < 1 || tile_rows < 1) return NULL;
    orc_tsqr_state* S = (orc_tsqr_state*)calloc(1, sizeof(orc_tsqr_state));
    S->m = m; S->n = n;
    int64_t P = orc_num_leaves(m, leaf_rows);
    S->P = P;
    S->leaves = (leaf_t*)calloc((size_t)P, sizeof(leaf_t));
    for (int64_t i = 0; i < P; ++i) {
        S->leaves[i].row0 = i * leaf_rows;
        S->leaves[i].rows = (i == P - 1) ? (m - i * leaf_rows) : leaf_rows;
        if (g_mutation == 7 && P > 1 && i == P - 1) S->leaves[i].rows = leaf_rows; /* planted: drops the remainder */
    }
    /* a leaf's first tile must hold at least n rows */
    int64_t trows = tile_rows < n ? n : tile_rows;

    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < P; ++i) factor_leaf(&S->leaves[i], n, A, lda, trows);

    /* binary tree */
    S->count = (int64_t*)calloc(64, sizeof(int64_t));
    S->L = orc_tree_levels(P, S->count, 64);
    S->nodes = (node_t**)calloc((size_t)(S->L > 0 ? S->L : 1), sizeof(node_t*));
    /* R of every entry of the current level, plus the first leaf of its subtree */
    int64_t cur = P;
    double* Rcur = (double*)malloc(sizeof(double) * (size_t)P * (size_t)n * (size_t)n);
    int64_t* home = (int64_t*)malloc(sizeof(int64_t) * (size_t)P);
    for (int64_t i = 0; i < P; ++i) {
        leaf_t* lf = &S->leaves[i];
        stage_R(&lf->st[lf->ntiles - 1], n, Rcur + (size_t)i * n * n);
        home[i] = i;
    }
    for (int l = 0; l < S->L; ++l) {
        int64_t nc = S->count[l];
        node_t* nd = (node_t*)calloc((size_t)nc, sizeof(node_t));
        S->nodes[l] = nd;
        double* Rnext = (double*)malloc(sizeof(double) * (size_t)nc * (size_t)n * (size_t)n);
        int64_t* hnext = (int64_t*)malloc(sizeof(int64_t) * (size_t)nc);
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t q = 0; q < nc; ++q) {
            int64_t a = 2 * q, b = 2 * q + 1;
            nd[q].home_a = home[a];
            hnext[q] = home[a];
            if (b >= cur) {
                nd[q].pass = 1;
                nd[q].home_b = -1;
                memcpy(Rnext + (size_t)q * n * n, Rcur + (size_t)a * n * n, sizeof(double) * (size_t)n * (size_t)n);
                continue;
            }
            nd[q].home_b = home[b];
            stage_t* s = &nd[q].st;
            stage_alloc(s, 2 * n, n);
            const double* Ra = Rcur + (size_t)a * n * n;
            const double* Rb = Rcur + (size_t)b * n * n;
            for (int64_t c = 0; c < n; ++c)
                for (int64_t i = 0; i < n; ++i) {
                    s->V[IDX(i, c, 2 * n)] = Ra[IDX(i, c, n)];
                    s->V[IDX(n + i, c, 2 * n)] = Rb[IDX(i, c, n)];
                }
            orc_householder_qr(2 * n, n, s->V, 2 * n, s->tau);
            stage_R(s, n, Rnext + (size_t)q * n * n);
        }
        free(Rcur); free(home);
        Rcur = Rnext; home = hnext; cur = nc;
    }
    S->Rroot = Rcur; /* n x n */
    free(home);
    S->d = (double*)malloc(sizeof(double) * (size_t)n);
    double* tmp = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
    sign_normalise(n, S->Rroot, n, S->d, tmp, n);
    free(tmp);
    return S;
}

void orc_tsqr_free(orc_tsqr_state* S)
{
    if (!S) return;
    for (int64_t i = 0; i < S->P; ++i) {
        for (int64_t k = 0; k < S->leaves[i].ntiles; ++k) stage_free(&S->leaves[i].st[k]);
        free(S->leaves[i].st);
    }
    free(S->leaves);
    for (int l = 0; l < S->L; ++l) {
        for (int64_t q = 0; q < S->count[l]; ++q)
            if (!S->nodes[l][q].pass) stage_free(&S->nodes[l][q].st);
        free(S->nodes[l]);
    }
    free(S->nodes); free(S->count); free(S->Rroot); free(S->d);
    free(S);
}

/* Sign-normalised R (n x n, upper, diag >= 0). */
void orc_tsqr_R(const orc_tsqr_state* S, double* R, int64_t ldr)
{
    double* d = (double*)malloc(sizeof(double) * (size_t)S->n);
    sign_normalise(S->n, S->Rroot, S->n, d, R, ldr);
    free(d);
}

void orc_tsqr_signs(const orc_tsqr_state* S, double* d)
{
    memcpy(d, S->d, sizeof(double) * (size_t)S->n);
}

/* Explicit thin Q (m x n): the stored factors applied to [D; 0] from the root
 * down.  The seed of a node's input is an n x n block; a node maps seed S to
 * [S_a; S_b] = Q_node [S; 0], a pass-through node hands S down unchanged. */
void orc_tsqr_form_q(const orc_tsqr_state* S, double* Q, int64_t ldq)
{
    int64_t n = S->n, P = S->P;
    size_t nn = (size_t)n * (size_t)n;
    /* seeds of the current level, root first */
    double* seeds = (double*)calloc(nn, sizeof(double));
    for (int64_t j = 0; j < n; ++j) seeds[IDX(j, j, n)] = S->d[j];
    for (int l = S->L - 1; l >= 0; --l) {
        int64_t nc = S->count[l];
        int64_t below = (l == 0) ? P : S->count[l - 1];
        double* nxt = (double*)calloc((size_t)below * nn, sizeof(double));
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t q = 0; q < nc; ++q) {
            const node_t* nd = &S->nodes[l][q];
            const double* Sq = seeds + (size_t)q * nn;
            int64_t a = 2 * q, b = 2 * q + 1;
            if (g_mutation == 3) { int64_t t = a; a = b; b = t; } /* planted: children swapped */
            if (nd->pass) {
                memcpy(nxt + (size_t)(2 * q) * nn, Sq, nn * sizeof(double));
                continue;
            }
            double* X = (double*)calloc(2 * nn, sizeof(double)); /* 2n x n, ld 2n */
            for (int64_t c = 0; c < n; ++c)
                for (int64_t i = 0; i < n; ++i) X[IDX(i, c, 2 * n)] = Sq[IDX(i, c, n)];
            if (g_mutation == 4) orc_apply_qt(2 * n, n, nd->st.V, 2 * n, nd->st.tau, n, X, 2 * n); /* planted */
            else orc_apply_q(2 * n, n, nd->st.V, 2 * n, nd->st.tau, n, X, 2 * n);
            for (int64_t c = 0; c < n; ++c)
                for (int64_t i = 0; i < n; ++i) {
                    nxt[(size_t)a * nn + IDX(i, c, n)] = X[IDX(i, c, 2 * n)];
                    nxt[(size_t)b * nn + IDX(i, c, n)] = X[IDX(n + i, c, 2 * n)];
                }
            free(X);
        }
        free(seeds);
        seeds = nxt;
    }
    /* leaves: the flat chain from its last stage down to stage 0 */
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < P; ++i) {
        const leaf_t* lf = &S->leaves[i];
        double* Sk = (double*)malloc(nn * sizeof(double));
        memcpy(Sk, seeds + (size_t)i * nn, nn * sizeof(double));
        for (int64_t k = lf->ntiles - 1; k >= 0; --k) {
            const stage_t* s = &lf->st[k];
            int64_t rows = s->rows;
            double* X = (double*)calloc((size_t)rows * (size_t)n, sizeof(double));
            for (int64_t c = 0; c < n; ++c)
                for (int64_t r = 0; r < n; ++r) X[IDX(r, c, rows)] = Sk[IDX(r, c, n)];
            orc_apply_q(rows, n, s->V, rows, s->tau, n, X, rows);
            int64_t tile_first = (k == 0) ? 0 : n;           /* rows of X that belong to tile k */
            /* A-row offset of tile k inside the leaf */
            int64_t off = 0;
            for (int64_t t = 0; t < k; ++t) off += (t == 0) ? lf->st[0].rows : (lf->st[t].rows - n);
            for (int64_t c = 0; c < n; ++c)
                for (int64_t r = tile_first; r < rows; ++r)
                    Q[IDX(lf->row0 + off + (r - tile_first), c, ldq)] = X[IDX(r, c, rows)];
            if (k > 0)
                for (int64_t c = 0; c < n; ++c)
                    for (int64_t r = 0; r < n; ++r) Sk[IDX(r, c, n)] = X[IDX(r, c, rows)];
            free(X);
        }
        free(Sk);
    }
    free(seeds);
}

/* B (m x k) <- Q_full^T B, Q_full being TSQR's m x m orthogonal factor, with the
 * signs D applied to the first n rows, so rows 0..n-1 hold D Q_thin^T B.  The
 * other rows hold the coordinates in the tree's own basis of the complement. */
void orc_tsqr_apply_qt(const orc_tsqr_state* S, int64_t k, double* B, int64_t ldb)
{
    int64_t n = S->n, P = S->P;
    /* leaves: stage 0 on tile 0, then [C; B_k] for each later tile; C lives in
     * the top n rows of tile 0 */
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < P; ++i) {
        const leaf_t* lf = &S->leaves[i];
        int64_t r0 = lf->row0;
        const stage_t* s0 = &lf->st[0];
        orc_apply_qt(s0->rows, n, s0->V, s0->rows, s0->tau, k, B + IDX(r0, 0, ldb), ldb);
        int64_t off = s0->rows;
        for (int64_t t = 1; t < lf->ntiles; ++t) {
            const stage_t* s = &lf->st[t];
            int64_t rows = s->rows, mk = rows - n;
            double* X = (double*)malloc(sizeof(double) * (size_t)rows * (size_t)k);
            for (int64_t c = 0; c < k; ++c) {
                for (int64_t r = 0; r < n; ++r) X[IDX(r, c, rows)] = B[IDX(r0 + r, c, ldb)];
                for (int64_t r = 0; r < mk; ++r) X[IDX(n + r, c, rows)] = B[IDX(r0 + off + r, c, ldb)];
            }
            orc_apply_qt(rows, n, s->V, rows, s->tau, k, X, rows);
            for (int64_t c = 0; c < k; ++c) {
                for (int64_t r = 0; r < n; ++r) B[IDX(r0 + r, c, ldb)] = X[IDX(r, c, rows)];
                for (int64_t r = 0; r < mk; ++r) B[IDX(r0 + off + r, c, ldb)] = X[IDX(n + r, c, rows)];
            }
            free(X);
            off += mk;
        }
    }
    /* tree, bottom-up: node (a, b) maps [C_a; C_b] to Q_node^T [C_a; C_b] */
    for (int l = 0; l < S->L; ++l) {
        int64_t nc = S->count[l];
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t q = 0; q < nc; ++q) {
            const node_t* nd = &S->nodes[l][q];
            if (nd->pass) continue;
            int64_t ra = S->leaves[nd->home_a].row0, rb = S->leaves[nd->home_b].row0;
            double* X = (double*)malloc(sizeof(double) * (size_t)(2 * n) * (size_t)k);
            for (int64_t c = 0; c < k; ++c)
                for (int64_t r = 0; r < n; ++r) {
                    X[IDX(r, c, 2 * n)] = B[IDX(ra + r, c, ldb)];
                    X[IDX(n + r, c, 2 * n)] = B[IDX(rb + r, c, ldb)];
                }
            orc_apply_qt(2 * n, n, nd->st.V, 2 * n, nd->st.tau, k, X, 2 * n);
            for (int64_t c = 0; c < k; ++c)
                for (int64_t r = 0; r < n; ++r) {
                    B[IDX(ra + r, c, ldb)] = X[IDX(r, c, 2 * n)];
                    B[IDX(rb + r, c, ldb)] = X[IDX(n + r, c, 2 * n)];
                }
            free(X);
        }
    }
    /* root: signs */
    for (int64_t c = 0; c < k; ++c)
        for (int64_t r = 0; r < n; ++r) B[IDX(r, c, ldb)] *= S->d[r];
}

/* Stage access for structural tests: the V array and tau of a tree node or of a
 * chain stage.  Returns rows, or -1 when the index does not exist. */
int64_t orc_tsqr_node(const orc_tsqr_state* S, int level, int64_t q, const double** V, const double** tau)
{
    if (level < 0 || level >= S->L || q < 0 || q >= S->count[level]) return -1;
    const node_t* nd = &S->nodes[level][q];
    if (nd->pass) return 0;
    *V = nd->st.V; *tau = nd->st.tau;
    return nd->st.rows;
}

int64_t orc_tsqr_leaf_stage(const orc_tsqr_state* S, int64_t leaf, int64_t k, const double** V, const double** tau)
{
    if (leaf < 0 || leaf >= S->P) return -1;
    const leaf_t* lf = &S->leaves[leaf];
    if (k < 0 || k >= lf->ntiles) return -1;
    *V = lf->st[k].V; *tau = lf->st[k].tau;
    return lf->st[k].rows;
}

/* First leaf of the left and right subtree of node q at level ``level``
 * (level 0 = the first combining stage); right = -1 for a pass-through node. */
int orc_tsqr_node_homes(const orc_tsqr_state* S, int level, int64_t q, int64_t* left, int64_t* right)
{
    if (level < 0 || level >= S->L || q < 0 || q >= S->count[level]) return -1;
    *left = S->nodes[level][q].home_a;
    *right = S->nodes[level][q].pass ? -1 : S->nodes[level][q].home_b;
    return 0;
}

int64_t orc_tsqr_num_leaves(const orc_tsqr_state* S) { return S->P; }
int orc_tsqr_num_levels(const orc_tsqr_state* S) { return S->L; }
