/*
 * Plain CPU oracle for the matrix power kernel.  TEST INFRASTRUCTURE ONLY:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this code.  It shares no code, header or helper with the HIP path.
 *
 * What it computes (Lacey et al., "Cache Blocking of Distributed-Memory
 * Parallel Matrix Power Kernels"):
 *
 *   - the matrix power kernel as defined in Sec. "RACE Applied to the Matrix
 *     Power Kernel": all y_k = A^k x for k = 1..p, each obtained from the
 *     previous one by a sparse matrix-vector product y_k = A y_{k-1}, i.e. the
 *     back-to-back SpMV of Alg. 1 ("Traditional Distributed MPK") without the
 *     halo exchange (one process);
 *   - the three-term recurrence of the Chebyshev application, Eq.
 *     (anderson_spmv): v_{k+1} = 2 H v_k - v_{k-1}, v_1 = H v_0, generalised to
 *     y_{j+1} = alpha_j (A y_j) + beta_j y_j + gamma_j y_{j-1}.
 *
 * Everything is FP64 with sequential in-row accumulation in stored order;
 * build with -O2 -ffp-contract=off so that no multiply-add is fused.
 * OpenMP splits the rows only, which leaves every row's arithmetic unchanged.
 *
 * Layouts: CSR with 0-based int32 row pointers and columns; x is n x R and
 * Y is p x n x R, both row-major with the right-hand side fastest:
 *   Y[(k-1)*n*R + i*R + r] = (y_k)_{i,r}.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One SpMV, y = A x, for R right-hand sides; values in double. */
static void spmv_f64(int64_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                     int R, const double *x, double *y) {
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        for (int r = 0; r < R; ++r) {
            double s = 0.0;
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                s += val[e] * x[(int64_t)col[e] * R + r];
            y[i * R + r] = s;
        }
    }
}

/* Same, with values stored in single precision and promoted before the product. */
static void spmv_f32(int64_t n, const int32_t *rowptr, const int32_t *col, const float *val,
                     int R, const double *x, double *y) {
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        for (int r = 0; r < R; ++r) {
            double s = 0.0;
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                s += (double)val[e] * x[(int64_t)col[e] * R + r];
            y[i * R + r] = s;
        }
    }
}

/* Powers: y_k = A y_{k-1}, y_0 = x.  value_bits selects double or float values. */
int oracle_powers(int64_t n, const int32_t *rowptr, const int32_t *col, const void *val,
                  int value_bits, int R, const double *x, int p, double *Y, int nthreads) {
    if (n < 0 || R < 1 || p < 1) return 1;
    set_threads(nthreads);
    const int64_t stride = n * R;
    for (int k = 1; k <= p; ++k) {
        const double *in = (k == 1) ? x : Y + (int64_t)(k - 2) * stride;
        double *out = Y + (int64_t)(k - 1) * stride;
        if (value_bits == 32)
            spmv_f32(n, rowptr, col, (const float *)val, R, in, out);
        else
            spmv_f64(n, rowptr, col, (const double *)val, R, in, out);
    }
    return 0;
}

/* Recurrence: y_{j+1} = alpha_j (A y_j) + beta_j y_j + gamma_j y_{j-1}, j = 0..p-1,
 * with y_0 = x; the gamma term is absent for j = 0.  A coefficient that is
 * exactly zero omits its term: the Chebyshev recurrence of Sec. "Application:
 * Chebyshev Time Propagation" has no beta term, and the general form reduces
 * to it term by term. */
int oracle_recur(int64_t n, const int32_t *rowptr, const int32_t *col, const void *val,
                 int value_bits, int R, const double *x, int p, const double *alpha,
                 const double *beta, const double *gamma, double *Y, int nthreads) {
    if (n < 0 || R < 1 || p < 1) return 1;
    set_threads(nthreads);
    const int64_t stride = n * R;
    double *t = (double *)malloc((size_t)(stride > 0 ? stride : 1) * sizeof(double));
    if (!t) return 2;
    for (int j = 0; j < p; ++j) {
        const double *yj = (j == 0) ? x : Y + (int64_t)(j - 1) * stride;
        const double *yjm1 = (j == 0) ? NULL : (j == 1 ? x : Y + (int64_t)(j - 2) * stride);
        double *out = Y + (int64_t)j * stride;
        if (value_bits == 32)
            spmv_f32(n, rowptr, col, (const float *)val, R, yj, t);
        else
            spmv_f64(n, rowptr, col, (const double *)val, R, yj, t);
        int64_t m;
#pragma omp parallel for schedule(static)
        for (m = 0; m < stride; ++m) {
            double v = alpha[j] * t[m];
            if (beta[j] != 0.0) v += beta[j] * yj[m];
            if (yjm1 && gamma[j] != 0.0) v += gamma[j] * yjm1[m];
            out[m] = v;
        }
    }
    free(t);
    return 0;
}
