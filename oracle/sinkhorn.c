/*
 * Log-domain Sinkhorn iterations on a materialised float64 cost matrix:
 * the compiled part of the FP64 oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the oracle (and through it tests/,
 * __graft_entry__.smoke() and bench.py's cpu_baseline leg) loads this code.
 * It shares nothing with the HIP library.
 *
 * It computes exactly what the oracle's NumPy Sinkhorn computes, in plain
 * loops, for problems where NumPy's temporaries make that too slow
 * (N = M = 20,000 and above).  With the Sinkhorn operators of Appendix A.1,
 *   T_row(g)_i = -eps log sum_j exp(log b_j + (g_j - C_ij) / eps),
 *   T_col(f)_j = -eps log sum_i exp(log a_i + (f_i - C_ij) / eps),
 * one iteration of Algorithm 3 (symmetric) is
 *   f <- (f + T_row(g)) / 2,  g <- (g + T_col(f)) / 2   (both from iterate n),
 * and of Algorithm 2 (alternating) f <- T_row(g), then g <- T_col(f).
 * Every log-sum-exp is shifted by the maximum over its whole row (column),
 * and a non-finite maximum is replaced by 0, as in the NumPy form.  Columns
 * are read as rows of the transposed matrix, which the caller passes.
 * Rows (columns) are independent, so they are split over OpenMP threads;
 * each one is reduced by a single thread in index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* glibc's libmvec provides vector variants of exp (documented error below
   4 ulp); this declaration lets the compiler call them from the
   elementwise loop, as math.h itself does under -ffast-math. */
double exp(double) __attribute__((simd("notinbranch")));

/* out_i = -eps * lse_j (logw_j + (h_j - c_ij) / eps), c row-major rows x cols.
   Per row: the exponents v_j into a buffer and their maximum; then
   exp(v_j - max) (an elementwise loop the compiler may vectorise); then the
   sum over j in index order. */
static void softmin_rows(const double* c, int64_t rows, int64_t cols, const double* logw, const double* h,
                         double eps, double* out) {
#pragma omp parallel
    {
        double* v = (double*)malloc(sizeof(double) * (size_t)cols);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < rows; ++i) {
            const double* ci = c + i * cols;
            double mx = -INFINITY;
            for (int64_t j = 0; j < cols; ++j) {
                v[j] = logw[j] + (h[j] - ci[j]) / eps;
                if (v[j] > mx) mx = v[j];
            }
            if (!isfinite(mx)) mx = 0.0;
#pragma omp simd
            for (int64_t j = 0; j < cols; ++j) v[j] = exp(v[j] - mx);
            double s = 0.0;
            for (int64_t j = 0; j < cols; ++j) s += v[j];
            out[i] = -eps * (mx + log(s));
        }
        free(v);
    }
}

/* n_iter iterations in place on f (n) and g (m).  c: n x m, ct: its
   transpose (m x n), both row-major.  Returns 0, or -1 on a failed
   allocation. */
int oracle_sinkhorn(const double* c, const double* ct, int64_t n, int64_t m, const double* a, const double* b,
                    double eps, int n_iter, int symmetric, double* f, double* g) {
    double* la = (double*)malloc(sizeof(double) * n);
    double* lb = (double*)malloc(sizeof(double) * m);
    double* tf = (double*)malloc(sizeof(double) * n);
    double* tg = (double*)malloc(sizeof(double) * m);
    if (!la || !lb || !tf || !tg) {
        free(la);
        free(lb);
        free(tf);
        free(tg);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) la[i] = log(a[i]);
    for (int64_t j = 0; j < m; ++j) lb[j] = log(b[j]);
    for (int it = 0; it < n_iter; ++it) {
        if (symmetric) {
            softmin_rows(c, n, m, lb, g, eps, tf);
            softmin_rows(ct, m, n, la, f, eps, tg);
            for (int64_t i = 0; i < n; ++i) f[i] = 0.5 * (f[i] + tf[i]);
            for (int64_t j = 0; j < m; ++j) g[j] = 0.5 * (g[j] + tg[j]);
        } else {
            softmin_rows(c, n, m, lb, g, eps, f);
            softmin_rows(ct, m, n, la, f, eps, g);
        }
    }
    free(la);
    free(lb);
    free(tf);
    free(tg);
    return 0;
}
