/*
 * CPU oracle for Strassen's block-recursive matrix inversion.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library and is deliberately plain:
 * double precision throughout, no blocking, no fusion, no reordering beyond
 * what the definitions below state, built with -ffp-contract=off so that
 * every a - b*c is a rounded product followed by a rounded difference.
 *
 * Storage: every matrix is column-major with a leading dimension, the layout
 * of the paper's matrix blocks (the block data structure of Sec. 3.2).
 *
 * Functions
 *   oracle_gemm          C = A * B, plain triple loop, k summed in ascending
 *                        order (the definition of the matrix product that the
 *                        paper's `multiply` computes, Sec. 3.3).
 *   oracle_gj_inv        O1: Gauss-Jordan elimination on [A | I] with partial
 *                        pivoting (one concrete choice for the leaf inversion,
 *                        whose method the paper leaves open, Alg. 1).
 *   oracle_strassen_inv  O2: the block-inverse identity of Alg. 1 (Sec. 3.1),
 *                        recursing on the leading block and on the (negated)
 *                        Schur complement until a block reaches the leaf
 *                        threshold, whose inverse O1 computes.
 *   oracle_ns_step       one Newton(-Schulz) refinement step
 *                        X' = X + X (I - A X) (Sec. 2.1 cites Newton iteration
 *                        as the stabiliser of Strassen inversion).
 *
 * Readings of the paper that this file fixes (the paper is silent):
 *   - leaf test: recurse while m > leaf, invert when m <= leaf (Alg. 1 tests
 *     n = threshold, Alg. 2 tests size/blockSize = 1; both only consider
 *     n = 2^p, Sec. 4);
 *   - split of an order-m block when m is not leaf * 2^k: the leading block
 *     has order n1 = 64 * ceil(m / 128) for m >= 128 and ceil(m / 2) below;
 *     this is exact halving whenever m = leaf * 2^k with leaf a multiple of 64
 *     (or any power of two);
 *   - pivot choice: largest |entry| in the pivot column at or below the
 *     diagonal, ties to the smallest row index; an exactly zero or
 *     non-finite pivot column stops the elimination and reports the 1-based
 *     column (LAPACK getrf convention).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define AT(p, i, j, ld) ((p)[(int64_t)(i) + (int64_t)(j) * (int64_t)(ld)])

int oracle_version(void) { return 1; }

/* C (m x n, ldc) = A (m x k, lda) * B (k x n, ldb). */
void oracle_gemm(const double *A, int64_t lda, const double *B, int64_t ldb,
                 double *C, int64_t ldc, int64_t m, int64_t n, int64_t k)
{
    /* threads only for products large enough to repay their start-up; each
     * column is the same sum either way */
#pragma omp parallel for schedule(static) if ((double)m * (double)n * (double)k > 4.0e6)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i)
            AT(C, i, j, ldc) = 0.0;
        /* For every (i, j) the terms are added in ascending k. */
        for (int64_t p = 0; p < k; ++p) {
            const double b = AT(B, p, j, ldb);
            for (int64_t i = 0; i < m; ++i)
                AT(C, i, j, ldc) = AT(C, i, j, ldc) + AT(A, i, p, lda) * b;
        }
    }
}

/* O1.  X (n x n, ldx) = A^-1 by Gauss-Jordan on the augmented [A | I].
 * Returns 0, or k+1 when the pivot column k (0-based) holds no usable pivot
 * (all candidates zero, or any candidate non-finite); X is then unspecified. */
int oracle_gj_inv(const double *A, int64_t n, int64_t lda, double *X, int64_t ldx)
{
    if (n <= 0)
        return 0;
    const int64_t w = 2 * n; /* columns of [A | I] */
    double *M = (double *)malloc(sizeof(double) * (size_t)(n * w));
    double *f = (double *)malloc(sizeof(double) * (size_t)n);
    if (!M || !f) {
        free(M);
        free(f);
        return -1;
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            AT(M, i, j, n) = AT(A, i, j, lda);
            AT(M, i, n + j, n) = (i == j) ? 1.0 : 0.0;
        }

    int info = 0;
    for (int64_t k = 0; k < n && !info; ++k) {
        /* partial pivoting: largest |M[i,k]| for i >= k, smallest i on ties */
        int64_t p = k;
        double best = fabs(AT(M, k, k, n));
        int finite = isfinite(AT(M, k, k, n));
        for (int64_t i = k + 1; i < n; ++i) {
            const double v = fabs(AT(M, i, k, n));
            if (!isfinite(v))
                finite = 0;
            if (v > best) {
                best = v;
                p = i;
            }
        }
        if (!finite || !(best > 0.0)) {
            info = (int)(k + 1);
            break;
        }
        if (p != k)
            for (int64_t j = 0; j < w; ++j) {
                const double t = AT(M, k, j, n);
                AT(M, k, j, n) = AT(M, p, j, n);
                AT(M, p, j, n) = t;
            }
        /* scale the pivot row: every entry divided by the pivot */
        const double piv = AT(M, k, k, n);
        for (int64_t j = 0; j < w; ++j)
            AT(M, k, j, n) = AT(M, k, j, n) / piv;
        /* eliminate column k from every other row:
         * row_i <- row_i - M[i,k] * row_k, with M[i,k] taken before the step */
        for (int64_t i = 0; i < n; ++i)
            f[i] = AT(M, i, k, n);
#pragma omp parallel for schedule(static) if ((double)n * (double)w > 2.0e5)
        for (int64_t j = 0; j < w; ++j) {
            const double rk = AT(M, k, j, n);
            for (int64_t i = 0; i < n; ++i)
                if (i != k)
                    AT(M, i, j, n) = AT(M, i, j, n) - f[i] * rk;
        }
    }
    if (!info)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
                AT(X, i, j, ldx) = AT(M, i, n + j, n);
    free(M);
    free(f);
    return info;
}

/* Order of the leading block when an order-m block is split. */
int64_t oracle_split(int64_t m)
{
    if (m >= 128)
        return 64 * ((m + 127) / 128);
    return (m + 1) / 2;
}

static double *dalloc(int64_t r, int64_t c)
{
    size_t cnt = (size_t)((r > 0 ? r : 1) * (c > 0 ? c : 1));
    return (double *)malloc(sizeof(double) * cnt);
}

/* Copy / negate / subtract helpers on (r x c) column-major views. */
static void mat_sub(const double *P, int64_t ldp, const double *Q, int64_t ldq,
                    double *R, int64_t ldr, int64_t r, int64_t c)
{
    for (int64_t j = 0; j < c; ++j)
        for (int64_t i = 0; i < r; ++i)
            AT(R, i, j, ldr) = AT(P, i, j, ldp) - AT(Q, i, j, ldq);
}

static void mat_neg(const double *P, int64_t ldp, double *R, int64_t ldr, int64_t r, int64_t c)
{
    for (int64_t j = 0; j < c; ++j)
        for (int64_t i = 0; i < r; ++i)
            AT(R, i, j, ldr) = -AT(P, i, j, ldp);
}

static void mat_copy(const double *P, int64_t ldp, double *R, int64_t ldr, int64_t r, int64_t c)
{
    for (int64_t j = 0; j < c; ++j)
        for (int64_t i = 0; i < r; ++i)
            AT(R, i, j, ldr) = AT(P, i, j, ldp);
}

/* Factors of one split of an order-m block into A11 (n1 x n1), A12, A21 and
 * A22 (n2 x n2).  With P = A11^-1 and the Schur complement S = A22 - A21 P A12
 * the inverse is
 *
 *     [ P + (P A12) S^-1 (A21 P)     -(P A12) S^-1 ]
 *     [ -S^-1 (A21 P)                 S^-1         ]
 *
 * Alg. 1 carries N = -S instead (A21 (P A12) - A22) and its inverse T = N^-1,
 * so that the off-diagonal blocks are (P A12) T and T (A21 P) with no sign
 * change and the lower-right block is -T.  The fields hold, per split:
 *   inv11   P                      n1 x n1
 *   rowfac  A21 P                  n2 x n1
 *   colfac  P A12                  n1 x n2
 *   negs    N = A21 colfac - A22   n2 x n2
 *   invn    T = N^-1               n2 x n2
 *   work    A21 colfac (n2 x n2), later colfac C21 (n1 x n1)            */
struct split_factors {
    double *inv11, *rowfac, *colfac, *negs, *invn, *work;
};

static void factors_free(struct split_factors *f)
{
    free(f->inv11);
    free(f->rowfac);
    free(f->colfac);
    free(f->negs);
    free(f->invn);
    free(f->work);
}

static int factors_alloc(struct split_factors *f, int64_t n1, int64_t n2)
{
    const int64_t big = n1 > n2 ? n1 : n2;
    f->inv11 = dalloc(n1, n1);
    f->rowfac = dalloc(n2, n1);
    f->colfac = dalloc(n1, n2);
    f->negs = dalloc(n2, n2);
    f->invn = dalloc(n2, n2);
    f->work = dalloc(big, big);
    return f->inv11 && f->rowfac && f->colfac && f->negs && f->invn && f->work;
}

/* O2.  C (m x m, ldc) = A^-1.  col0 is the global column offset of this
 * block, so that a failing leaf reports a global 1-based column.  Every
 * product is the plain triple loop and every difference a separate rounding,
 * in the order below: the two factors, the negated Schur complement (product
 * first, then the difference with A22), its inverse, the two off-diagonal
 * blocks, the leading block's correction, and the negation of T. */
static int strassen_rec(const double *A, int64_t m, int64_t lda, double *C, int64_t ldc,
                        int64_t leaf, int64_t col0)
{
    if (m <= leaf) {
        const int info = oracle_gj_inv(A, m, lda, C, ldc);
        return info > 0 ? (int)(info + col0) : info;
    }
    const int64_t n1 = oracle_split(m), n2 = m - n1;
    const double *a12 = &AT(A, 0, n1, lda), *a21 = &AT(A, n1, 0, lda), *a22 = &AT(A, n1, n1, lda);
    double *c11 = &AT(C, 0, 0, ldc), *c12 = &AT(C, 0, n1, ldc);
    double *c21 = &AT(C, n1, 0, ldc), *c22 = &AT(C, n1, n1, ldc);
    struct split_factors f;
    int info = -1;
    if (!factors_alloc(&f, n1, n2))
        goto out;

    info = strassen_rec(A, n1, lda, f.inv11, n1, leaf, col0);
    if (info)
        goto out;
    oracle_gemm(a21, lda, f.inv11, n1, f.rowfac, n2, n2, n1, n1);
    oracle_gemm(f.inv11, n1, a12, lda, f.colfac, n1, n1, n2, n1);
    oracle_gemm(a21, lda, f.colfac, n1, f.work, n2, n2, n2, n1);
    mat_sub(f.work, n2, a22, lda, f.negs, n2, n2, n2);
    info = strassen_rec(f.negs, n2, n2, f.invn, n2, leaf, col0 + n1);
    if (info)
        goto out;
    oracle_gemm(f.colfac, n1, f.invn, n2, c12, ldc, n1, n2, n2);
    oracle_gemm(f.invn, n2, f.rowfac, n2, c21, ldc, n2, n1, n2);
    oracle_gemm(f.colfac, n1, c21, ldc, f.work, n1, n1, n1, n2);
    mat_sub(f.inv11, n1, f.work, n1, c11, ldc, n1, n1);
    mat_neg(f.invn, n2, c22, ldc, n2, n2);
out:
    factors_free(&f);
    return info;
}

int oracle_strassen_inv(const double *A, int64_t n, int64_t lda, double *X, int64_t ldx,
                        int64_t leaf)
{
    if (n <= 0)
        return 0;
    if (leaf < 1)
        return -2;
    return strassen_rec(A, n, lda, X, ldx, leaf, 0);
}

/* R (c x r, ldr) = P^T for P (r x c, ldp). */
static void mat_transpose(const double *P, int64_t ldp, double *R, int64_t ldr, int64_t r, int64_t c)
{
    for (int64_t j = 0; j < c; ++j)
        for (int64_t i = 0; i < r; ++i)
            AT(R, j, i, ldr) = AT(P, i, j, ldp);
}

/* Lower triangle mirrored onto the upper one: P[i][j] = P[j][i] for j > i. */
static void mat_mirror_lower(double *P, int64_t ldp, int64_t m)
{
    for (int64_t j = 1; j < m; ++j)
        for (int64_t i = 0; i < j; ++i)
            AT(P, i, j, ldp) = AT(P, j, i, ldp);
}

/* O3: O2 specialised to a symmetric A (the positive-definite matrices the
 * paper targets, Sec. 2.1).  Then A12 = A21^T and every inverse the recursion
 * forms is symmetric, so the column factor P A12 is the transpose of the row
 * factor A21 P and is never formed:
 *   N   = A21 (P A12) - A22 = rowfac A12 - A22,
 *   C12 = (P A12) T         = (T rowfac)^T = C21^T,
 *   C11 = P - (P A12) C21   = P - C12 rowfac,
 * four products per split instead of six.  N and C11 are symmetric too: only
 * their lower triangles are kept, mirrored onto the upper ones, so that every
 * block a split passes on (N to the recursion, C11 and C22 to its caller) is
 * exactly symmetric outside the leaves.  Passing the rounding asymmetry of N
 * and C11 on instead would break colfac = rowfac^T one level down, and the
 * residual would grow like kappa u.  Both triangles of A are read, so this is
 * the symmetric specialisation only for an exactly symmetric A. */
static int strassen_spd_rec(const double *A, int64_t m, int64_t lda, double *C, int64_t ldc,
                            int64_t leaf, int64_t col0)
{
    if (m <= leaf) {
        const int info = oracle_gj_inv(A, m, lda, C, ldc);
        return info > 0 ? (int)(info + col0) : info;
    }
    const int64_t n1 = oracle_split(m), n2 = m - n1;
    const double *a12 = &AT(A, 0, n1, lda), *a21 = &AT(A, n1, 0, lda), *a22 = &AT(A, n1, n1, lda);
    double *c11 = &AT(C, 0, 0, ldc), *c12 = &AT(C, 0, n1, ldc);
    double *c21 = &AT(C, n1, 0, ldc), *c22 = &AT(C, n1, n1, ldc);
    struct split_factors f;
    int info = -1;
    if (!factors_alloc(&f, n1, n2))
        goto out;

    info = strassen_spd_rec(A, n1, lda, f.inv11, n1, leaf, col0);
    if (info)
        goto out;
    oracle_gemm(a21, lda, f.inv11, n1, f.rowfac, n2, n2, n1, n1);
    oracle_gemm(f.rowfac, n2, a12, lda, f.work, n2, n2, n2, n1);
    mat_sub(f.work, n2, a22, lda, f.negs, n2, n2, n2);
    mat_mirror_lower(f.negs, n2, n2);
    info = strassen_spd_rec(f.negs, n2, n2, f.invn, n2, leaf, col0 + n1);
    if (info)
        goto out;
    oracle_gemm(f.invn, n2, f.rowfac, n2, c21, ldc, n2, n1, n2);
    mat_transpose(c21, ldc, c12, ldc, n2, n1);
    oracle_gemm(c12, ldc, f.rowfac, n2, f.work, n1, n1, n1, n2);
    mat_sub(f.inv11, n1, f.work, n1, c11, ldc, n1, n1);
    mat_mirror_lower(c11, ldc, n1);
    mat_neg(f.invn, n2, c22, ldc, n2, n2);
out:
    factors_free(&f);
    return info;
}

int oracle_strassen_inv_spd(const double *A, int64_t n, int64_t lda, double *X, int64_t ldx,
                            int64_t leaf)
{
    if (n <= 0)
        return 0;
    if (leaf < 1)
        return -2;
    return strassen_spd_rec(A, n, lda, X, ldx, leaf, 0);
}

/* Leaf of O4: A = L U without pivoting (Doolittle: unit lower L), then
 * Li = L^-1 by forward substitution and Ui = U^-1 by back substitution, each
 * written as a full m x m block (zeros in the other triangle).  Returns 0, or
 * the 1-based column of the first zero or non-finite pivot. */
int oracle_lu_leaf(const double *A, int64_t m, int64_t lda, double *Li, int64_t ldl, double *Ui,
                   int64_t ldu)
{
    double *F = dalloc(m, m);
    if (!F)
        return -1;
    mat_copy(A, lda, F, m, m, m);
    int info = 0;
    for (int64_t k = 0; k < m && !info; ++k) {
        const double piv = AT(F, k, k, m);
        if (piv == 0.0 || !isfinite(piv)) {
            info = (int)(k + 1);
            break;
        }
        for (int64_t i = k + 1; i < m; ++i)
            AT(F, i, k, m) = AT(F, i, k, m) / piv;                 /* multiplier l_ik */
        for (int64_t j = k + 1; j < m; ++j)
            for (int64_t i = k + 1; i < m; ++i)
                AT(F, i, j, m) = AT(F, i, j, m) - AT(F, i, k, m) * AT(F, k, j, m);
    }
    for (int64_t j = 0; j < m && !info; ++j) {
        /* column j of L^-1: x_j = 1, x_i = -sum_{j<=k<i} l_ik x_k for i > j */
        for (int64_t i = 0; i < m; ++i) {
            double x = 0.0;
            if (i == j) {
                x = 1.0;
            } else if (i > j) {
                for (int64_t k = j; k < i; ++k)
                    x = x - AT(F, i, k, m) * AT(Li, k, j, ldl);
            }
            AT(Li, i, j, ldl) = x;
        }
        /* column j of U^-1: x_j = 1/u_jj, x_i = -(sum_{i<k<=j} u_ik x_k)/u_ii for i < j */
        for (int64_t i = m - 1; i >= 0; --i) {
            double x = 0.0;
            if (i == j) {
                x = 1.0 / AT(F, j, j, m);
            } else if (i < j) {
                for (int64_t k = i + 1; k <= j; ++k)
                    x = x - AT(F, i, k, m) * AT(Ui, k, j, ldu);
                x = x / AT(F, i, i, m);
            }
            AT(Ui, i, j, ldu) = x;
        }
    }
    free(F);
    return info;
}

/* Block recursion of O4: Li = L^-1 and Ui = U^-1 of the factors of A = L U
 * (no pivoting across or inside blocks), Li and Ui written as full blocks.
 *   (Li11, Ui11) = rec(A11);  U12 = Li11 A12;  L21 = A21 Ui11;
 *   S = A22 - L21 U12;  (Li22, Ui22) = rec(S);
 *   Li21 = -Li22 (L21 Li11);  Ui12 = -(Ui11 U12) Ui22;
 *   Li12 = 0;  Ui21 = 0. */
static int lu_rec(const double *A, int64_t m, int64_t lda, double *Li, int64_t ldl, double *Ui,
                  int64_t ldu, int64_t leaf, int64_t col0)
{
    if (m <= leaf) {
        int info = oracle_lu_leaf(A, m, lda, Li, ldl, Ui, ldu);
        return info > 0 ? (int)(info + col0) : info;
    }
    const int64_t n1 = oracle_split(m), n2 = m - n1;
    const double *A12 = &AT(A, 0, n1, lda), *A21 = &AT(A, n1, 0, lda), *A22 = &AT(A, n1, n1, lda);
    double *U12 = dalloc(n1, n2), *L21 = dalloc(n2, n1), *P = dalloc(n2, n2);
    double *S = dalloc(n2, n2), *T1 = dalloc(n2, n1), *T2 = dalloc(n1, n2);
    int info = -1;
    if (!U12 || !L21 || !P || !S || !T1 || !T2)
        goto done;
    info = lu_rec(A, n1, lda, Li, ldl, Ui, ldu, leaf, col0);
    if (info)
        goto done;
    oracle_gemm(Li, ldl, A12, lda, U12, n1, n1, n2, n1);                /* U12 = Li11 A12  */
    oracle_gemm(A21, lda, Ui, ldu, L21, n2, n2, n1, n1);                /* L21 = A21 Ui11  */
    oracle_gemm(L21, n2, U12, n1, P, n2, n2, n2, n1);                   /* P = L21 U12     */
    mat_sub(A22, lda, P, n2, S, n2, n2, n2);                            /* S = A22 - P     */
    info = lu_rec(S, n2, n2, &AT(Li, n1, n1, ldl), ldl, &AT(Ui, n1, n1, ldu), ldu, leaf, col0 + n1);
    if (info)
        goto done;
    oracle_gemm(L21, n2, Li, ldl, T1, n2, n2, n1, n1);                  /* T1 = L21 Li11   */
    oracle_gemm(Ui, ldu, U12, n1, T2, n1, n1, n2, n1);                  /* T2 = Ui11 U12   */
    oracle_gemm(&AT(Li, n1, n1, ldl), ldl, T1, n2, &AT(Li, n1, 0, ldl), ldl, n2, n1, n2);
    mat_neg(&AT(Li, n1, 0, ldl), ldl, &AT(Li, n1, 0, ldl), ldl, n2, n1); /* Li21 = -Li22 T1 */
    oracle_gemm(T2, n1, &AT(Ui, n1, n1, ldu), ldu, &AT(Ui, 0, n1, ldu), ldu, n1, n2, n2);
    mat_neg(&AT(Ui, 0, n1, ldu), ldu, &AT(Ui, 0, n1, ldu), ldu, n1, n2); /* Ui12 = -T2 Ui22 */
    for (int64_t j = n1; j < m; ++j)
        for (int64_t i = 0; i < n1; ++i)
            AT(Li, i, j, ldl) = 0.0;                                    /* Li12 = 0        */
    for (int64_t j = 0; j < n1; ++j)
        for (int64_t i = n1; i < m; ++i)
            AT(Ui, i, j, ldu) = 0.0;                                    /* Ui21 = 0        */
done:
    free(U12);
    free(L21);
    free(P);
    free(S);
    free(T1);
    free(T2);
    return info;
}

/* O4: inversion through a block LU factorisation, the method the paper
 * compares against (Sec. 5, after Liu et al.): A = L U without pivoting,
 * L^-1 and U^-1 by block recursion, then X = U^-1 L^-1. */
int oracle_lu_inv(const double *A, int64_t n, int64_t lda, double *X, int64_t ldx, int64_t leaf)
{
    if (n <= 0)
        return 0;
    if (leaf < 1)
        return -2;
    double *Li = dalloc(n, n), *Ui = dalloc(n, n);
    int info = -1;
    if (Li && Ui) {
        info = lu_rec(A, n, lda, Li, n, Ui, n, leaf, 0);
        if (!info)
            oracle_gemm(Ui, n, Li, n, X, ldx, n, n, n);                  /* X = Ui Li       */
    }
    free(Li);
    free(Ui);
    return info;
}

/* One refinement step: Xn = X + X (I - A X). */
int oracle_ns_step(const double *A, int64_t n, int64_t lda, const double *X, int64_t ldx,
                   double *Xn, int64_t ldxn)
{
    double *AX = dalloc(n, n), *R = dalloc(n, n), *XR = dalloc(n, n);
    int rc = -1;
    if (AX && R && XR) {
        oracle_gemm(A, lda, X, ldx, AX, n, n, n, n);
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
                AT(R, i, j, n) = ((i == j) ? 1.0 : 0.0) - AT(AX, i, j, n);
        oracle_gemm(X, ldx, R, n, XR, n, n, n, n);
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
                AT(Xn, i, j, ldxn) = AT(X, i, j, ldx) + AT(XR, i, j, n);
        rc = 0;
    }
    free(AX);
    free(R);
    free(XR);
    return rc;
}

/* Copy used by tests that build matrices from views. */
void oracle_copy(const double *P, int64_t ldp, double *R, int64_t ldr, int64_t r, int64_t c)
{
    mat_copy(P, ldp, R, ldr, r, c);
}
