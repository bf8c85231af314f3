/*
 * CPU oracle: plain FP64 loops used by the oracle's Python driver.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into oracle/liboracle.so,
 * which only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load.  It shares no code with the HIP library.
 *
 * Each routine is the textbook definition written out with no blocking or
 * reordering beyond an OpenMP split of the outer (row) loop, so the order of
 * every floating-point sum is the natural one.
 */
#include <stdint.h>

/* Y = A X for a CSR matrix A (n rows) and a row-major block X (ncols_a x p).
 * Y is row-major n x p.  Sparse times dense (Section 2.2: the products H X, B X). */
void oracle_csr_spmm(int64_t n, int64_t p, const int64_t *row_ptr, const int32_t *col,
                     const double *val, const double *X, double *Y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double *y = Y + i * p;
        for (int64_t c = 0; c < p; ++c) y[c] = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const double a = val[e];
            const double *x = X + (int64_t)col[e] * p;
            for (int64_t c = 0; c < p; ++c) y[c] += a * x[c];
        }
    }
}

/* Column-shifted operator of the preconditioner (eq. precondition-T):
 * Y[:,l] = (Lh - lam[l] B) X[:,l], with Lh = L/2 given as its own values. */
void oracle_csr_shifted_spmm(int64_t n, int64_t p, const int64_t *row_ptr, const int32_t *col,
                             const double *lh_val, const double *b_val, const double *lam,
                             const double *X, double *Y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double *y = Y + i * p;
        for (int64_t c = 0; c < p; ++c) y[c] = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const double *x = X + (int64_t)col[e] * p;
            for (int64_t c = 0; c < p; ++c) y[c] += (lh_val[e] - lam[c] * b_val[e]) * x[c];
        }
    }
}
