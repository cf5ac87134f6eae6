/*
 * Oracle: plain, slow, obviously correct FP64 Cholesky factorization and
 * triangular solves on the CPU.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * What it computes.  The paper's workload is the tile Cholesky factorization
 * DPOTRF of PLASMA in double precision (section 4.1, "Benchmarks"; tiles of
 * 512, section 4.1 "Methodology").  Its result has a plain definition: for a
 * symmetric positive definite A, L is the unique lower-triangular matrix with
 * a positive diagonal such that A = L L^T.  The tile algorithm reaches that
 * same L, up to the order of floating-point rounding.  This file therefore
 * writes the definition out with the textbook unblocked right-looking
 * (outer-product) algorithm, column by column, with no blocking, no fusion
 * and no reordering.
 *
 * Conventions (readings where the paper is silent):
 *  - matrices are column-major with a leading dimension; only the lower
 *    triangle is read or written; the strict upper triangle is never touched;
 *  - a pivot that is not > 0 (zero, negative or NaN) stops the factorization
 *    and returns info = its 1-based column, as LAPACK does;
 *  - sqrt and division are IEEE-754 correctly rounded (no fast math); the
 *    build disables floating-point contraction so every product is rounded
 *    before it is subtracted.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(M, ld, i, j) ((M)[(size_t)(j) * (size_t)(ld) + (size_t)(i)])

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/*
 * Cholesky factorization A = L L^T (definition above), unblocked
 * right-looking order.  On return the lower triangle of A holds L.
 * Returns 0, or k > 0 when the pivot of column k (1-based) is not positive;
 * then columns before k hold L and the rest of A is partly updated.
 * The trailing update of column j only reads column k and writes column j,
 * so the columns are independent and may run on separate threads without
 * changing a single rounding.
 */
int64_t oracle_potrf(int64_t n, double *A, int64_t lda) {
    for (int64_t k = 0; k < n; ++k) {
        double d = AT(A, lda, k, k);
        if (!(d > 0.0)) return k + 1;
        double l_kk = sqrt(d);
        AT(A, lda, k, k) = l_kk;
        for (int64_t i = k + 1; i < n; ++i) AT(A, lda, i, k) = AT(A, lda, i, k) / l_kk;
#pragma omp parallel for schedule(static) if (n - k > 256)
        for (int64_t j = k + 1; j < n; ++j) {
            double l_jk = AT(A, lda, j, k);
            for (int64_t i = j; i < n; ++i)
                AT(A, lda, i, j) = AT(A, lda, i, j) - AT(A, lda, i, k) * l_jk;
        }
    }
    return 0;
}

/*
 * Solve A X = B given the factor L (lower triangle of L), by forward
 * substitution L Y = B followed by back substitution L^T X = Y, one
 * right-hand side column at a time.  B is overwritten by X.
 *   y_i = (b_i - sum_{k<i} L_ik y_k) / L_ii
 *   x_i = (y_i - sum_{k>i} L_ki x_k) / L_ii
 */
void oracle_potrs(int64_t n, const double *L, int64_t ldl, int64_t nrhs, double *B, int64_t ldb) {
#pragma omp parallel for schedule(static) if (nrhs > 1)
    for (int64_t c = 0; c < nrhs; ++c) {
        double *b = B + (size_t)c * (size_t)ldb;
        for (int64_t i = 0; i < n; ++i) {
            double s = b[i];
            for (int64_t k = 0; k < i; ++k) s = s - AT(L, ldl, i, k) * b[k];
            b[i] = s / AT(L, ldl, i, i);
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = b[i];
            for (int64_t k = i + 1; k < n; ++k) s = s - AT(L, ldl, k, i) * b[k];
            b[i] = s / AT(L, ldl, i, i);
        }
    }
}

/*
 * Residual R = B - A X for symmetric A given by its lower triangle,
 * accumulated in long double (x86 80-bit extended precision) so that the
 * residual of an FP64 solution is itself accurate to well below FP64
 * rounding.  R is rounded to double at the end.
 */
void oracle_residual(int64_t n, const double *A, int64_t lda, int64_t nrhs, const double *X,
                     int64_t ldx, const double *B, int64_t ldb, double *R, int64_t ldr) {
#pragma omp parallel for schedule(static) if (n > 256)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t c = 0; c < nrhs; ++c) {
            const double *x = X + (size_t)c * (size_t)ldx;
            long double s = (long double)B[(size_t)c * (size_t)ldb + (size_t)i];
            for (int64_t j = 0; j < n; ++j) {
                double a = (i >= j) ? AT(A, lda, i, j) : AT(A, lda, j, i);
                s -= (long double)a * (long double)x[j];
            }
            R[(size_t)c * (size_t)ldr + (size_t)i] = (double)s;
        }
    }
}

/*
 * Entry (i, j) of L L^T for the lower-triangular L, in long double:
 * sum_{k <= min(i,j)} L_ik L_jk.  Used to check sampled entries of a large
 * factor against A one by one.
 */
double oracle_llt_entry(const double *L, int64_t ldl, int64_t i, int64_t j) {
    int64_t m = i < j ? i : j;
    long double s = 0.0L;
    for (int64_t k = 0; k <= m; ++k) s += (long double)AT(L, ldl, i, k) * (long double)AT(L, ldl, j, k);
    return (double)s;
}

/*
 * Adjoint of the Cholesky factorization (reverse-mode derivative).  Given
 * the factor L of A and Lbar = df/dL for a scalar f (both lower triangles),
 * computes Abar = df/dA for the symmetric A and overwrites the lower
 * triangle of Lbar with the lower triangle of Abar.
 *
 * The derivative of the factorization is not stated in the paper; the
 * oracle takes the plainest definition: the reverse of each arithmetic step
 * of oracle_potrf above, run in the opposite order (reverse-mode
 * differentiation of that program, with every value it reverses read from
 * the final L, which is where oracle_potrf leaves it).  The forward step k
 *     l = sqrt(a_kk);  a_ik := a_ik / l  (i > k);
 *     a_ij := a_ij - a_ik a_jk  (j > k, i >= j)
 * has the reverse (adjoints p, starting from Lbar)
 *     p_ik -= p_ij l_jk  and  p_jk -= p_ij l_ik   for j > k, i >= j
 *     p_ik := p_ik / l_kk,  p_kk -= p_ik l_ik      for i > k
 *     p_kk := p_kk / (2 l_kk).
 * The first line, collected per row r > k of column k:
 *     p_rk -= sum_{k<j<=r} p_rj l_jk + sum_{i>=r} p_ir l_ik
 * (the term i = j = r appears in both sums: the square in the update of
 * a_rr).  p is then the derivative with respect to the entries the program
 * reads, the lower triangle of A; since a_ij for i > j stands for both
 * a_ij and a_ji of the symmetric matrix, Abar_ij = p_ij / 2 off the
 * diagonal and Abar_ii = p_ii, which is the last step.
 */
void oracle_chol_adjoint(int64_t n, const double *L, int64_t ldl, double *P, int64_t ldp) {
    for (int64_t k = n - 1; k >= 0; --k) {
#pragma omp parallel for schedule(static) if (n - k > 256)
        for (int64_t r = k + 1; r < n; ++r) {
            double s = 0.0;
            for (int64_t j = k + 1; j <= r; ++j) s = s + AT(P, ldp, r, j) * AT(L, ldl, j, k);
            for (int64_t i = r; i < n; ++i) s = s + AT(P, ldp, i, r) * AT(L, ldl, i, k);
            AT(P, ldp, r, k) = AT(P, ldp, r, k) - s;
        }
        double l_kk = AT(L, ldl, k, k);
        double t = AT(P, ldp, k, k);
        for (int64_t i = k + 1; i < n; ++i) {
            AT(P, ldp, i, k) = AT(P, ldp, i, k) / l_kk;
            t = t - AT(P, ldp, i, k) * AT(L, ldl, i, k);
        }
        AT(P, ldp, k, k) = t / (2.0 * l_kk);
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j + 1; i < n; ++i) AT(P, ldp, i, j) = AT(P, ldp, i, j) * 0.5;
}
