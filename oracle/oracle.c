/*
 * Plain FP64 CPU oracle for the tiled Cholesky factorisation and solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * What it computes
 * ----------------
 * The paper (Section 5.1, "Array Partitioning") names the Cholesky
 * factorisation as the standard user of matrix partitioning into sub-matrix
 * handles, and Section 2 fixes the execution model: tasks with read-only,
 * write-only or read-write buffer parameters whose dependency graph follows
 * from those access modes plus the order of submission, and (Section 3) an
 * annotated program stays a valid sequential program.  The oracle is that
 * sequential program: the tile tasks of a right-looking tiled Cholesky
 * (POTRF, TRSM, SYRK, GEMM) and of the forward/backward solve, executed one
 * after another in submission order.
 *
 * Arithmetic contract (every function below):
 *   - IEEE binary64, round to nearest even; build with -ffp-contract=off so
 *     that no product is fused into an addition;
 *   - each dot-product subtraction is one rounded product followed by one
 *     rounded subtraction, in increasing index order for the factor and the
 *     forward solve, in decreasing index order for the backward solve;
 *   - correctly rounded division and square root (libm sqrt).
 * With that contract every element of the factor receives exactly the same
 * operation sequence as in the unblocked textbook algorithm, whatever the
 * tile size, so the tiled and unblocked routines agree bit for bit.
 *
 * Storage: row-major, leading dimension `ld` in elements; only the lower
 * triangle (row >= column) of a symmetric matrix is read or written.
 *
 * OpenMP is used only across independent output rows inside one tile
 * operation; it never changes the operation sequence of any element, so
 * results do not depend on the thread count.
 *
 * The panel solve may also be taken through the inverse of the diagonal
 * factor: or_trtri_tile forms W = L^{-1} by forward substitution on the
 * columns of the identity, or_trsm_inv_tile applies X <- X W^T.  Both are the
 * plain definitions of those operations; the tiled factor above always uses
 * the substitution (or_trsm_tile).
 *
 * Checkers accumulate in x87 80-bit long double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(p, ld, i, j) ((p)[(int64_t)(i) * (ld) + (j)])

/* ------------------------------------------------------------------------ */
/* Tile tasks of the factorisation                                           */
/* ------------------------------------------------------------------------ */

/* POTRF on one diagonal tile: D = L L^T, lower, in place.
 * Column by column: the pivot s = d_jj - sum_{p<j} d_jp^2 (p increasing); if s
 * is not strictly positive (or NaN) the factorisation breaks down and the
 * 1-based local column is returned; otherwise d_jj = sqrt(s) and each entry
 * below it becomes (d_ij - sum_{p<j} d_ip d_jp) / d_jj.  Returns 0 on success. */
int64_t or_potrf_tile(int64_t nb, double *d, int64_t ld)
{
    for (int64_t j = 0; j < nb; ++j) {
        double s = AT(d, ld, j, j);
        for (int64_t p = 0; p < j; ++p) {
            double prod = AT(d, ld, j, p) * AT(d, ld, j, p);
            s = s - prod;
        }
        if (!(s > 0.0))
            return j + 1;
        double piv = sqrt(s);
        AT(d, ld, j, j) = piv;
#pragma omp parallel for schedule(static) if (nb - j > 256)
        for (int64_t i = j + 1; i < nb; ++i) {
            double t = AT(d, ld, i, j);
            for (int64_t p = 0; p < j; ++p) {
                double prod = AT(d, ld, i, p) * AT(d, ld, j, p);
                t = t - prod;
            }
            AT(d, ld, i, j) = t / piv;
        }
    }
    return 0;
}

/* TRSM on one panel tile: X <- X L^{-T} with L lower, non-unit (the
 * right-side, lower, transposed solve of the tiled Cholesky).  Each row x of
 * X is independent: x_j = (x_j - sum_{p<j} x_p l_jp) / l_jj, p increasing. */
void or_trsm_tile(int64_t m, int64_t nb, const double *l, int64_t ldl,
                  double *x, int64_t ldx)
{
#pragma omp parallel for schedule(static) if (m > 64)
    for (int64_t i = 0; i < m; ++i) {
        double *row = x + i * ldx;
        for (int64_t j = 0; j < nb; ++j) {
            double t = row[j];
            for (int64_t p = 0; p < j; ++p) {
                double prod = row[p] * AT(l, ldl, j, p);
                t = t - prod;
            }
            row[j] = t / AT(l, ldl, j, j);
        }
    }
}

/* Inverse of a lower-triangular tile: lower(W) <- L^{-1}, column by column.
 * Column j of W solves L w = e_j by forward substitution; its entries above
 * row j are zero and are not stored (the strictly upper part of W is left
 * as it was).  w_i = (delta_ij - sum_{j<=p<i} l_ip w_p) / l_ii, p increasing. */
void or_trtri_tile(int64_t nb, const double *l, int64_t ldl, double *w, int64_t ldw)
{
#pragma omp parallel for schedule(static) if (nb > 64)
    for (int64_t j = 0; j < nb; ++j) {
        for (int64_t i = j; i < nb; ++i) {
            double t = (i == j) ? 1.0 : 0.0;
            for (int64_t p = j; p < i; ++p) {
                double prod = AT(l, ldl, i, p) * AT(w, ldw, p, j);
                t = t - prod;
            }
            AT(w, ldw, i, j) = t / AT(l, ldl, i, i);
        }
    }
}

/* The panel solve through an explicit inverse: X <- X W^T with W lower
 * triangular (W = L^{-1} gives X L^{-T}).  x_ic = sum_{p<=c} x_ip w_cp, p
 * increasing, on a copy of the row. */
void or_trsm_inv_tile(int64_t m, int64_t nb, const double *w, int64_t ldw,
                      double *x, int64_t ldx)
{
#pragma omp parallel for schedule(static) if (m > 64)
    for (int64_t i = 0; i < m; ++i) {
        double *row = x + i * ldx;
        double *in = (double *)malloc((size_t)nb * sizeof(double));
        memcpy(in, row, (size_t)nb * sizeof(double));
        for (int64_t c = 0; c < nb; ++c) {
            double t = 0.0;
            for (int64_t p = 0; p <= c; ++p) {
                double prod = in[p] * AT(w, ldw, c, p);
                t = t + prod;
            }
            row[c] = t;
        }
        free(in);
    }
}

/* GEMM update of an off-diagonal tile: C <- C - X Y^T, with X (m x kb) and
 * Y (nn x kb).  Every c_ij receives its kb subtractions in increasing p.
 * Y is first copied into a transposed scratch (a copy, no arithmetic) so the
 * loop over j is unit-stride; the per-element operation order is unchanged. */
void or_gemm_tile(int64_t m, int64_t nn, int64_t kb,
                  const double *x, int64_t ldx, const double *y, int64_t ldy,
                  double *c, int64_t ldc)
{
    if (m <= 0 || nn <= 0 || kb <= 0)
        return;
    double *yt = (double *)malloc(sizeof(double) * (size_t)(kb * nn));
    for (int64_t j = 0; j < nn; ++j)
        for (int64_t p = 0; p < kb; ++p)
            yt[p * nn + j] = AT(y, ldy, j, p);
#pragma omp parallel for schedule(static) if (m > 32)
    for (int64_t i = 0; i < m; ++i) {
        double *crow = c + i * ldc;
        const double *xrow = x + i * ldx;
        for (int64_t p = 0; p < kb; ++p) {
            const double xp = xrow[p];
            const double *yrow = yt + p * nn;
            for (int64_t j = 0; j < nn; ++j) {
                double prod = xp * yrow[j];
                crow[j] = crow[j] - prod;
            }
        }
    }
    free(yt);
}

/* SYRK update of a diagonal tile, lower half only: C <- C - X X^T for i >= j.
 * Same per-element order as the GEMM update; the strictly upper part of C
 * is never touched. */
void or_syrk_tile(int64_t nb, int64_t kb, const double *x, int64_t ldx,
                  double *c, int64_t ldc)
{
    if (nb <= 0 || kb <= 0)
        return;
    double *xt = (double *)malloc(sizeof(double) * (size_t)(kb * nb));
    for (int64_t j = 0; j < nb; ++j)
        for (int64_t p = 0; p < kb; ++p)
            xt[p * nb + j] = AT(x, ldx, j, p);
#pragma omp parallel for schedule(dynamic, 16) if (nb > 32)
    for (int64_t i = 0; i < nb; ++i) {
        double *crow = c + i * ldc;
        const double *xrow = x + i * ldx;
        for (int64_t p = 0; p < kb; ++p) {
            const double xp = xrow[p];
            const double *trow = xt + p * nb;
            for (int64_t j = 0; j <= i; ++j) {
                double prod = xp * trow[j];
                crow[j] = crow[j] - prod;
            }
        }
    }
    free(xt);
}

/* ------------------------------------------------------------------------ */
/* Tile tasks of the solve                                                   */
/* ------------------------------------------------------------------------ */

/* Forward TRSM on one RHS block: B <- L^{-1} B, L (nb x nb) lower non-unit,
 * B (nb x r).  y_i = (b_i - sum_{p<i} l_ip y_p) / l_ii, p increasing. */
void or_trsm_left_tile(int64_t nb, int64_t r, const double *l, int64_t ldl,
                       double *bm, int64_t ldb)
{
    for (int64_t c = 0; c < r; ++c)
        for (int64_t i = 0; i < nb; ++i) {
            double t = AT(bm, ldb, i, c);
            for (int64_t p = 0; p < i; ++p) {
                double prod = AT(l, ldl, i, p) * AT(bm, ldb, p, c);
                t = t - prod;
            }
            AT(bm, ldb, i, c) = t / AT(l, ldl, i, i);
        }
}

/* Backward TRSM on one RHS block: B <- L^{-T} B.
 * x_i = (b_i - sum_{p>i} l_pi x_p) / l_ii, p decreasing from the last row. */
void or_trsm_left_t_tile(int64_t nb, int64_t r, const double *l, int64_t ldl,
                         double *bm, int64_t ldb)
{
    for (int64_t c = 0; c < r; ++c)
        for (int64_t i = nb - 1; i >= 0; --i) {
            double t = AT(bm, ldb, i, c);
            for (int64_t p = nb - 1; p > i; --p) {
                double prod = AT(l, ldl, p, i) * AT(bm, ldb, p, c);
                t = t - prod;
            }
            AT(bm, ldb, i, c) = t / AT(l, ldl, i, i);
        }
}

/* Forward RHS update: B_I <- B_I - L_IK B_K (L_IK is m x kb), p increasing. */
void or_gemm_rhs_n(int64_t m, int64_t r, int64_t kb,
                   const double *l, int64_t ldl, const double *bk, int64_t ldbk,
                   double *bi, int64_t ldbi)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < r; ++c) {
            double t = AT(bi, ldbi, i, c);
            for (int64_t p = 0; p < kb; ++p) {
                double prod = AT(l, ldl, i, p) * AT(bk, ldbk, p, c);
                t = t - prod;
            }
            AT(bi, ldbi, i, c) = t;
        }
}

/* Backward RHS update: B_I <- B_I - L_KI^T X_K, where L_KI is (kb x m) and
 * X_K (kb x r); p runs over the rows of block K in decreasing order. */
void or_gemm_rhs_t(int64_t m, int64_t r, int64_t kb,
                   const double *l, int64_t ldl, const double *xk, int64_t ldxk,
                   double *bi, int64_t ldbi)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < r; ++c) {
            double t = AT(bi, ldbi, i, c);
            for (int64_t p = kb - 1; p >= 0; --p) {
                double prod = AT(l, ldl, p, i) * AT(xk, ldxk, p, c);
                t = t - prod;
            }
            AT(bi, ldbi, i, c) = t;
        }
}

/* ------------------------------------------------------------------------ */
/* Task dispatch by kind and tile coordinates (used to replay any order)     */
/* ------------------------------------------------------------------------ */

enum {
    OR_POTRF = 0, OR_TRSM = 1, OR_SYRK = 2, OR_GEMM = 3,
    OR_TRSM_L = 4, OR_GEMM_RHS_N = 5, OR_TRSM_LT = 6, OR_GEMM_RHS_T = 7
};

static int64_t tile_rows(int64_t n, int64_t b, int64_t t)
{
    int64_t r = n - t * b;
    return r < b ? r : b;
}

/* Runs one tile task.  Factor tasks: POTRF(k) uses (k,-,-), TRSM(i,k) and
 * SYRK(i,k) use (i,-,k), GEMM(i,j,k) uses all three.  Solve tasks act on the
 * RHS block matrix B (n x r): TRSM_L(K)/TRSM_LT(K) use (K,-,-);
 * GEMM_RHS_N(I,K) computes B_I -= L_IK B_K; GEMM_RHS_T(I,K) computes
 * B_I -= L_KI^T B_K.  Returns the POTRF breakdown column (global, 1-based),
 * or 0. */
int64_t or_run_task(int kind, int64_t n, int64_t b, double *a, int64_t lda,
                    int64_t ti, int64_t tj, int64_t tk,
                    double *bm, int64_t ldb, int64_t r)
{
    switch (kind) {
    case OR_POTRF: {
        int64_t nb = tile_rows(n, b, ti);
        double *d = a + ti * b * lda + ti * b;
        int64_t info = or_potrf_tile(nb, d, lda);
        return info ? ti * b + info : 0;
    }
    case OR_TRSM:
        or_trsm_tile(tile_rows(n, b, ti), b,
                     a + tk * b * lda + tk * b, lda,
                     a + ti * b * lda + tk * b, lda);
        return 0;
    case OR_SYRK:
        or_syrk_tile(tile_rows(n, b, ti), b,
                     a + ti * b * lda + tk * b, lda,
                     a + ti * b * lda + ti * b, lda);
        return 0;
    case OR_GEMM:
        or_gemm_tile(tile_rows(n, b, ti), tile_rows(n, b, tj), b,
                     a + ti * b * lda + tk * b, lda,
                     a + tj * b * lda + tk * b, lda,
                     a + ti * b * lda + tj * b, lda);
        return 0;
    case OR_TRSM_L:
        or_trsm_left_tile(tile_rows(n, b, ti), r, a + ti * b * lda + ti * b, lda,
                          bm + ti * b * ldb, ldb);
        return 0;
    case OR_TRSM_LT:
        or_trsm_left_t_tile(tile_rows(n, b, ti), r, a + ti * b * lda + ti * b, lda,
                            bm + ti * b * ldb, ldb);
        return 0;
    case OR_GEMM_RHS_N:
        or_gemm_rhs_n(tile_rows(n, b, ti), r, tile_rows(n, b, tk),
                      a + ti * b * lda + tk * b, lda,
                      bm + tk * b * ldb, ldb, bm + ti * b * ldb, ldb);
        return 0;
    case OR_GEMM_RHS_T:
        or_gemm_rhs_t(tile_rows(n, b, ti), r, tile_rows(n, b, tk),
                      a + tk * b * lda + ti * b, lda,
                      bm + tk * b * ldb, ldb, bm + ti * b * ldb, ldb);
        return 0;
    default:
        return -1;
    }
}

/* ------------------------------------------------------------------------ */
/* Whole factorisation and solve in submission order                         */
/* ------------------------------------------------------------------------ */

/* Right-looking tiled Cholesky, tasks run in submission order:
 *   for k: POTRF(k); for i>k: TRSM(i,k); for i>k: SYRK(i,k), then for
 *   k<j<i: GEMM(i,j,k).
 * Every later task depends (transitively) on POTRF(k), so a breakdown there
 * stops the factorisation; the returned info is the global 1-based column. */
int64_t or_potrf_tiled(int64_t n, double *a, int64_t lda, int64_t b)
{
    if (n <= 0)
        return 0;
    if (b <= 0)
        return -1;
    int64_t t = (n + b - 1) / b;
    for (int64_t k = 0; k < t; ++k) {
        int64_t info = or_run_task(OR_POTRF, n, b, a, lda, k, 0, 0, NULL, 0, 0);
        if (info)
            return info;
        for (int64_t i = k + 1; i < t; ++i)
            or_run_task(OR_TRSM, n, b, a, lda, i, 0, k, NULL, 0, 0);
        for (int64_t i = k + 1; i < t; ++i) {
            or_run_task(OR_SYRK, n, b, a, lda, i, 0, k, NULL, 0, 0);
            for (int64_t j = k + 1; j < i; ++j)
                or_run_task(OR_GEMM, n, b, a, lda, i, j, k, NULL, 0, 0);
        }
    }
    return 0;
}

/* Unblocked textbook Cholesky (the definition the tiled routine must equal). */
int64_t or_potrf_unblocked(int64_t n, double *a, int64_t lda)
{
    for (int64_t j = 0; j < n; ++j) {
        double s = AT(a, lda, j, j);
        for (int64_t p = 0; p < j; ++p) {
            double prod = AT(a, lda, j, p) * AT(a, lda, j, p);
            s = s - prod;
        }
        if (!(s > 0.0))
            return j + 1;
        double piv = sqrt(s);
        AT(a, lda, j, j) = piv;
        for (int64_t i = j + 1; i < n; ++i) {
            double t = AT(a, lda, i, j);
            for (int64_t p = 0; p < j; ++p) {
                double prod = AT(a, lda, i, p) * AT(a, lda, j, p);
                t = t - prod;
            }
            AT(a, lda, i, j) = t / piv;
        }
    }
    return 0;
}

/* Tiled solve with the factor L (lower tiles of a), B (n x r) in place:
 * forward for K ascending: TRSM_L(K), then GEMM_RHS_N(I,K) for I>K;
 * backward for K descending: TRSM_LT(K), then GEMM_RHS_T(I,K) for I<K,
 * issued with I descending. */
void or_potrs_tiled(int64_t n, int64_t r, const double *l, int64_t ldl,
                    double *bm, int64_t ldb, int64_t b)
{
    if (n <= 0 || r <= 0 || b <= 0)
        return;
    double *a = (double *)l; /* solve tasks only read the factor */
    int64_t t = (n + b - 1) / b;
    for (int64_t k = 0; k < t; ++k) {
        or_run_task(OR_TRSM_L, n, b, a, ldl, k, 0, 0, bm, ldb, r);
        for (int64_t i = k + 1; i < t; ++i)
            or_run_task(OR_GEMM_RHS_N, n, b, a, ldl, i, 0, k, bm, ldb, r);
    }
    for (int64_t k = t - 1; k >= 0; --k) {
        or_run_task(OR_TRSM_LT, n, b, a, ldl, k, 0, 0, bm, ldb, r);
        for (int64_t i = k - 1; i >= 0; --i)
            or_run_task(OR_GEMM_RHS_T, n, b, a, ldl, i, 0, k, bm, ldb, r);
    }
}

/* Unblocked forward and backward substitution (the definition). */
void or_potrs_unblocked(int64_t n, int64_t r, const double *l, int64_t ldl,
                        double *bm, int64_t ldb)
{
    or_trsm_left_tile(n, r, l, ldl, bm, ldb);
    or_trsm_left_t_tile(n, r, l, ldl, bm, ldb);
}

/* ------------------------------------------------------------------------ */
/* Checkers (extended precision)                                             */
/* ------------------------------------------------------------------------ */

static double sym_at(const double *a, int64_t lda, int64_t i, int64_t j)
{
    return i >= j ? AT(a, lda, i, j) : AT(a, lda, j, i);
}

/* Exact-order backward error ||A - L L^T||_F / ||A||_F over the full
 * symmetric A (read from its lower triangle), accumulated in long double. */
double or_backward_error_fro(int64_t n, const double *a, int64_t lda,
                             const double *l, int64_t ldl)
{
    long double num = 0.0L, den = 0.0L;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : num, den)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j <= i; ++j) {
            long double s = 0.0L;
            for (int64_t p = 0; p <= j; ++p)
                s += (long double)AT(l, ldl, i, p) * (long double)AT(l, ldl, j, p);
            long double d = (long double)AT(a, lda, i, j) - s;
            long double av = (long double)AT(a, lda, i, j);
            long double w = (i == j) ? 1.0L : 2.0L;
            num += w * d * d;
            den += w * av * av;
        }
    }
    return den > 0 ? (double)sqrtl(num / den) : (double)sqrtl(num);
}

/* Randomised backward-error estimate ||(A - L L^T) Z||_F / ||A Z||_F with Z
 * an n x nz probe matrix (row-major), in long double; O(n^2 nz). */
double or_backward_error_est(int64_t n, const double *a, int64_t lda,
                             const double *l, int64_t ldl,
                             const double *z, int64_t nz)
{
    long double *w = (long double *)calloc((size_t)(n * nz), sizeof(long double));
    /* W = L^T Z */
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p)
        for (int64_t c = 0; c < nz; ++c) {
            long double s = 0.0L;
            for (int64_t i = p; i < n; ++i)
                s += (long double)AT(l, ldl, i, p) * (long double)z[i * nz + c];
            w[p * nz + c] = s;
        }
    long double num = 0.0L, den = 0.0L;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : num, den)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < nz; ++c) {
            long double az = 0.0L, lw = 0.0L;
            for (int64_t j = 0; j < n; ++j)
                az += (long double)sym_at(a, lda, i, j) * (long double)z[j * nz + c];
            for (int64_t p = 0; p <= i; ++p)
                lw += (long double)AT(l, ldl, i, p) * w[p * nz + c];
            num += (az - lw) * (az - lw);
            den += az * az;
        }
    free(w);
    return den > 0 ? (double)sqrtl(num / den) : (double)sqrtl(num);
}

/* Sampled entries of A - L L^T: out[s] = A_ij - sum_{p<=min(i,j)} L_ip L_jp
 * for (i,j) = (rows[s], cols[s]), in long double, rounded to double. */
void or_sampled_residual(int64_t n, const double *a, int64_t lda,
                         const double *l, int64_t ldl, int64_t ns,
                         const int64_t *rows, const int64_t *cols, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i = rows[s], j = cols[s];
        if (i < j) { int64_t t = i; i = j; j = t; }
        long double acc = (long double)AT(a, lda, i, j);
        for (int64_t p = 0; p <= j; ++p)
            acc -= (long double)AT(l, ldl, i, p) * (long double)AT(l, ldl, j, p);
        out[s] = (double)acc;
    }
    (void)n;
}

/* Residual R = B - A X for symmetric A (lower triangle read), X and B n x r,
 * accumulated in long double and rounded once to double. */
void or_residual_ld(int64_t n, int64_t r, const double *a, int64_t lda,
                    const double *x, int64_t ldx, const double *bm, int64_t ldb,
                    double *res, int64_t ldr)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < r; ++c) {
            long double s = (long double)AT(bm, ldb, i, c);
            for (int64_t j = 0; j < n; ++j)
                s -= (long double)sym_at(a, lda, i, j) * (long double)AT(x, ldx, j, c);
            AT(res, ldr, i, c) = (double)s;
        }
}

/* Same residual in plain binary64 (j increasing, no fused operations). */
void or_residual_f64(int64_t n, int64_t r, const double *a, int64_t lda,
                     const double *x, int64_t ldx, const double *bm, int64_t ldb,
                     double *res, int64_t ldr)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < r; ++c) {
            double s = AT(bm, ldb, i, c);
            for (int64_t j = 0; j < n; ++j) {
                double prod = sym_at(a, lda, i, j) * AT(x, ldx, j, c);
                s = s - prod;
            }
            AT(res, ldr, i, c) = s;
        }
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
