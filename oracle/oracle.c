/*
 * CPU oracle for the row-partitioned SpMV y = A x  (TEST INFRASTRUCTURE ONLY).
 *
 * This file is the checker, not the product: only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark load it.  It shares no source with
 * the HIP library.
 *
 * What it computes (Sec. III-A of the paper): a rank's entries of y are the
 * full-row products of its owned rows of A with x.  Splitting A = A_L + A_R
 * changes only how the sum is reached, never its value, so the reference for
 * every row is the plain definition
 *
 *     y[i] = sum_k A[i, k] * x[k]
 *
 * evaluated here as accurately as FP64 allows: each row is one dot product
 * computed with the compensated algorithm Dot2 of Ogita, Rump and Oishi
 * ("Accurate sum and dot product", SIAM J. Sci. Comput. 26(6), 2005), whose
 * result is as accurate as a product evaluated in twice the working
 * precision and then rounded.  Alongside, absax[i] = sum_k |A[i,k]| |x[k]|
 * gives the scale for the per-row tolerance.
 *
 * Building blocks (both error-free transformations from the same article):
 *   TwoSum(a, b)     -> (s, e) with s = fl(a + b), a + b = s + e exactly
 *                       (Knuth's branch-free form).
 *   TwoProduct(a, b) -> (p, e) with p = fl(a * b), a * b = p + e exactly
 *                       (the error term read off with one fused multiply-add).
 *
 * Must be compiled without floating-point contraction or fast-math
 * (-ffp-contract=off), otherwise the error-free transformations break.
 * Rows are independent, so they are spread over OpenMP threads; the sum inside
 * each row is sequential in CSR order.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void two_product(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* Dot2 over the entries [b, e) of one CSR row. */
static inline double row_dot2(int64_t b, int64_t e, const int32_t *col,
                              const double *val, const double *x, double *abs_out)
{
    double p = 0.0, s = 0.0, a = 0.0;
    for (int64_t k = b; k < e; ++k) {
        double h, r, q;
        double xv = x[col[k]];
        two_product(val[k], xv, &h, &r);
        two_sum(p, h, &p, &q);
        s += q + r;
        a += fabs(val[k]) * fabs(xv);
    }
    *abs_out = a;
    return p + s;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * y[i] = Dot2(A[i,:], x) and absax[i] = |A[i,:]| . |x| for i in [0, n_rows).
 * row_ptr[i] .. row_ptr[i+1] index col/val directly, so a block of rows of a
 * larger matrix is passed as row_ptr + first_row with the full col/val arrays.
 * absax may be NULL.  dynamic != 0 selects dynamic scheduling (skewed rows).
 */
void orc_csr_dot2(int64_t n_rows, const int32_t *row_ptr, const int32_t *col,
                  const double *val, const double *x, double *y, double *absax,
                  int dynamic)
{
    if (dynamic) {
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n_rows; ++i) {
            double a;
            y[i] = row_dot2(row_ptr[i], row_ptr[i + 1], col, val, x, &a);
            if (absax) absax[i] = a;
        }
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n_rows; ++i) {
            double a;
            y[i] = row_dot2(row_ptr[i], row_ptr[i + 1], col, val, x, &a);
            if (absax) absax[i] = a;
        }
    }
}

/*
 * The plain FP64 CSR product, y[i] = sum of fl(A[i,k] * x[k]) added left to
 * right, no compensation: the ordinary CPU way to compute a row block, timed
 * beside the oracle as the CPU throughput baseline (it is not a reference:
 * its rounding is that of any plain summation).  Scheduling as in
 * orc_csr_dot2.
 */
void orc_csr_plain(int64_t n_rows, const int32_t *row_ptr, const int32_t *col,
                   const double *val, const double *x, double *y, int dynamic)
{
    if (dynamic) {
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n_rows; ++i) {
            double s = 0.0;
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += val[k] * x[col[k]];
            y[i] = s;
        }
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n_rows; ++i) {
            double s = 0.0;
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += val[k] * x[col[k]];
            y[i] = s;
        }
    }
}

/* Dot2 of two dense vectors (used by the oracle's own self-tests). */
double orc_dot2(int64_t n, const double *a, const double *b)
{
    double p = 0.0, s = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double h, r, q;
        two_product(a[k], b[k], &h, &r);
        two_sum(p, h, &p, &q);
        s += q + r;
    }
    return p + s;
}
