/* Oracle numeric core: plain classical matrix multiplication on the CPU.
 *
 * TEST INFRASTRUCTURE ONLY. This file is never linked into the product library; only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * Built with gcc -O2 -ffp-contract=off (no fused multiply-add, no reassociation), so every
 * multiply and every add is rounded once, as in the rounding model of section 4.2.
 *
 *  orc_classical_f64  C = A*B in double, each c_ij summed sequentially over k = 0..K-1
 *                     (the sequential summation of eq. (seq_summation_error)); this is the
 *                     classical base case of the recursion (section 3.2).
 *  orc_classical_ld   selected rows of A*B accumulated in long double (x87, 64-bit
 *                     significand): the error reference standing in for the paper's
 *                     quadruple-precision classical product (section 5.1 experiments).
 *
 * Matrices are row-major with explicit leading dimensions (in elements). Rows are
 * distributed over OpenMP threads; each c_ij is computed by one thread in fixed k order,
 * so results do not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_classical_f64(int64_t m, int64_t k, int64_t n, const double *A, int64_t lda,
                       const double *B, int64_t ldb, double *C, int64_t ldc) {
    /* c_ij = ((a_i0 b_0j + a_i1 b_1j) + a_i2 b_2j) + ... : the i-k-j loop keeps the
     * sequential k order for every (i, j) while streaming rows of B. */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double *c = C + i * ldc;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            const double a = A[i * lda + p];
            const double *b = B + p * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] = c[j] + a * b[j];
        }
    }
}

void orc_classical_f32(int64_t m, int64_t k, int64_t n, const float *A, int64_t lda,
                       const float *B, int64_t ldb, float *C, int64_t ldc) {
    /* Same sequential order in single precision (unit roundoff 2^-24). */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        float *c = C + i * ldc;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0f;
        for (int64_t p = 0; p < k; ++p) {
            const float a = A[i * lda + p];
            const float *b = B + p * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] = c[j] + a * b[j];
        }
    }
}

void orc_classical_ld(int64_t nrows, const int64_t *rows, int64_t k, int64_t n,
                      const double *A, int64_t lda, const double *B, int64_t ldb,
                      long double *C, int64_t ldc) {
    /* Row rows[t] of A*B into row t of C, products and sums in long double. */
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        long double *c = C + t * ldc;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0L;
        for (int64_t p = 0; p < k; ++p) {
            const long double a = (long double)A[i * lda + p];
            const double *b = B + p * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] = c[j] + a * (long double)b[j];
        }
    }
}
