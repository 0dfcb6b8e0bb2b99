/*
 * cmp_oracle.c -- plain FP64 CPU oracle of TSQR's competitors (Sec. 5 of
 * Demmel, Grigori, Hoemmen, Langou, "Implementing Communication-Optimal
 * Parallel and Sequential QR Factorizations"): CholeskyQR, classical and
 * modified Gram-Schmidt, and CholeskyQR applied twice.
 *
 * TEST INFRASTRUCTURE ONLY, like tsqr_oracle.c (linked into the same library):
 * nothing on the product path may link, load or call it, and it shares no code
 * with the GPU library.
 *
 * Each routine is the textbook definition written out with plain loops:
 *   CholeskyQR:  G = A^T A, G = R^T R (Cholesky, R upper with a positive
 *                diagonal), Q = A R^{-1}.
 *   CGS:         for j: r_ij = q_i^T a_j (i < j, a_j the column of A),
 *                v = a_j - sum_i r_ij q_i, r_jj = ||v||, q_j = v / r_jj.
 *   MGS:         V = A; for j: r_jj = ||v_j||, q_j = v_j / r_jj, then for every
 *                k > j: r_jk = q_j^T v_k, v_k <- v_k - r_jk q_j.
 *   CholeskyQR2: (Q1, R1) = CholeskyQR(A), (Q, R2) = CholeskyQR(Q1), R = R2 R1.
 * All return 0, or j + 1 when column j breaks the method down (a Cholesky pivot
 * that is not positive, or a zero norm in Gram-Schmidt); Q and R are then only
 * partly written.  Matrices are column-major with leading dimensions; R is
 * n x n with its strictly lower part set to zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CIDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

int orc_get_mutation(void); /* tsqr_oracle.c: the planted-mistake switch of the tests */

static void zero_lower(int64_t n, double* R, int64_t ldr)
{
    for (int64_t c = 0; c < n; ++c)
        for (int64_t i = c + 1; i < n; ++i) R[CIDX(i, c, ldr)] = 0.0;
}

int orc_cholqr(int64_t m, int64_t n, const double* A, int64_t lda, double* Q, int64_t ldq, double* R, int64_t ldr)
{
    /* G = A^T A (upper triangle) */
    double* G = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i <= j; ++i) {
            double s = 0.0;
            for (int64_t r = 0; r < m; ++r) s += A[CIDX(r, i, lda)] * A[CIDX(r, j, lda)];
            G[CIDX(i, j, n)] = s;
        }
    /* Cholesky, row by row of R: r_jj = sqrt(g_jj - sum_{k<j} r_kj^2),
     * r_jc = (g_jc - sum_{k<j} r_kj r_kc) / r_jj */
    zero_lower(n, R, ldr);
    int info = 0;
    for (int64_t j = 0; j < n && !info; ++j) {
        double d = G[CIDX(j, j, n)];
        for (int64_t k = 0; k < j; ++k) d -= R[CIDX(k, j, ldr)] * R[CIDX(k, j, ldr)];
        if (!(d > 0.0)) {
            info = (int)j + 1;
            break;
        }
        const double rjj = orc_get_mutation() == 9 ? d : sqrt(d); /* planted: no square root */
        R[CIDX(j, j, ldr)] = rjj;
        for (int64_t c = j + 1; c < n; ++c) {
            double s = G[CIDX(j, c, n)];
            for (int64_t k = 0; k < j; ++k) s -= R[CIDX(k, j, ldr)] * R[CIDX(k, c, ldr)];
            R[CIDX(j, c, ldr)] = s / rjj;
        }
    }
    free(G);
    if (info) return info;
    /* Q = A R^{-1}: each row q solves q R = a by forward substitution */
    for (int64_t r = 0; r < m; ++r)
        for (int64_t j = 0; j < n; ++j) {
            double s = A[CIDX(r, j, lda)];
            for (int64_t k = 0; k < j; ++k) s -= Q[CIDX(r, k, ldq)] * R[CIDX(k, j, ldr)];
            Q[CIDX(r, j, ldq)] = s / R[CIDX(j, j, ldr)];
        }
    return 0;
}

int orc_cholqr2(int64_t m, int64_t n, const double* A, int64_t lda, double* Q, int64_t ldq, double* R, int64_t ldr)
{
    double* Q1 = (double*)malloc(sizeof(double) * (size_t)m * (size_t)n);
    double* R1 = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
    double* R2 = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
    int info = orc_cholqr(m, n, A, lda, Q1, m, R1, n);
    if (!info) info = orc_cholqr(m, n, Q1, m, Q, ldq, R2, n);
    if (!info) {
        /* R = R2 R1, both upper triangular */
        for (int64_t c = 0; c < n; ++c)
            for (int64_t i = 0; i < n; ++i) {
                double s = 0.0;
                for (int64_t k = i; k <= c; ++k) s += R2[CIDX(i, k, n)] * R1[CIDX(k, c, n)];
                R[CIDX(i, c, ldr)] = i <= c ? s : 0.0;
            }
    }
    free(Q1);
    free(R1);
    free(R2);
    return info;
}

int orc_cgs(int64_t m, int64_t n, const double* A, int64_t lda, double* Q, int64_t ldq, double* R, int64_t ldr)
{
    zero_lower(n, R, ldr);
    double* v = (double*)malloc(sizeof(double) * (size_t)m);
    int info = 0;
    for (int64_t j = 0; j < n && !info; ++j) {
        for (int64_t r = 0; r < m; ++r) v[r] = A[CIDX(r, j, lda)];
        /* every coefficient against the original column a_j (the classical form) */
        for (int64_t i = 0; i < j; ++i) {
            double s = 0.0;
            for (int64_t r = 0; r < m; ++r) {
                /* planted: the partly orthogonalised v instead of a_j (that is MGS) */
                const double x = orc_get_mutation() == 8 ? v[r] : A[CIDX(r, j, lda)];
                s += Q[CIDX(r, i, ldq)] * x;
            }
            R[CIDX(i, j, ldr)] = s;
            if (orc_get_mutation() == 8)
                for (int64_t r = 0; r < m; ++r) v[r] -= s * Q[CIDX(r, i, ldq)];
        }
        if (orc_get_mutation() != 8)
            for (int64_t i = 0; i < j; ++i)
                for (int64_t r = 0; r < m; ++r) v[r] -= R[CIDX(i, j, ldr)] * Q[CIDX(r, i, ldq)];
        double s = 0.0;
        for (int64_t r = 0; r < m; ++r) s += v[r] * v[r];
        const double rjj = sqrt(s);
        if (rjj == 0.0) {
            info = (int)j + 1;
            break;
        }
        R[CIDX(j, j, ldr)] = rjj;
        for (int64_t r = 0; r < m; ++r) Q[CIDX(r, j, ldq)] = v[r] / rjj;
    }
    free(v);
    return info;
}

int orc_mgs(int64_t m, int64_t n, const double* A, int64_t lda, double* Q, int64_t ldq, double* R, int64_t ldr)
{
    zero_lower(n, R, ldr);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t r = 0; r < m; ++r) Q[CIDX(r, j, ldq)] = A[CIDX(r, j, lda)];
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t r = 0; r < m; ++r) s += Q[CIDX(r, j, ldq)] * Q[CIDX(r, j, ldq)];
        const double rjj = sqrt(s);
        if (rjj == 0.0) return (int)j + 1;
        R[CIDX(j, j, ldr)] = rjj;
        for (int64_t r = 0; r < m; ++r) Q[CIDX(r, j, ldq)] /= rjj;
        /* planted: only the next column is projected, later ones keep their q_j part */
        const int64_t kend = orc_get_mutation() == 10 ? (j + 2 < n ? j + 2 : n) : n;
        for (int64_t k = j + 1; k < kend; ++k) {
            double d = 0.0;
            for (int64_t r = 0; r < m; ++r) d += Q[CIDX(r, j, ldq)] * Q[CIDX(r, k, ldq)];
            R[CIDX(j, k, ldr)] = d;
            for (int64_t r = 0; r < m; ++r) Q[CIDX(r, k, ldq)] -= d * Q[CIDX(r, j, ldq)];
        }
    }
    return 0;
}
