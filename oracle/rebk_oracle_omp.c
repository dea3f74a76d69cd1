/*
 * rebk_oracle_omp.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * The oracle's iteration (Du, Si and Sun, arXiv:2001.04179, Section 2,
 * Algorithm 1) with its four block products spread over OpenMP threads, for
 * the CPU timing baseline of the benchmark only.  The plain single-thread
 * oracle (rebk_oracle.c) stays the parity reference: this file sums the
 * z-step's column products in per-thread pieces, so its iterates agree with
 * the plain oracle's to rounding, not bit for bit.  The block draws are the
 * plain oracle's (it links the same Philox and threshold functions).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void oracle_block_weights(const double *A, int64_t m, int64_t n, int64_t lda,
                          const int64_t *row_off, int64_t s, const int64_t *col_off, int64_t t,
                          double *w_row, double *w_col);
int oracle_thresholds(const double *w, int64_t nb, uint64_t *T);
int64_t oracle_pick(const uint64_t *T, int64_t nb, uint64_t word);

int oracle_omp_threads(void) { return omp_get_max_threads(); }

/* Algorithm 1 from x0 = 0, z0 = b for max_iter iterations (no stop rule), threads as set by
 * OMP_NUM_THREADS.  Returns 0, or -1 on invalid input. */
int oracle_rebk_solve_omp(const double *A, int64_t m, int64_t n, int64_t lda,
                          const int64_t *row_off, int64_t s, const int64_t *col_off, int64_t t,
                          double alpha, uint64_t seed, uint64_t sys, const double *b, int64_t max_iter,
                          double *x, double *z)
{
    if (m <= 0 || n <= 0 || s <= 0 || t <= 0 || lda < n || !(alpha > 0.0)) return -1;
    double *w_row = malloc(sizeof(double) * (size_t)s), *w_col = malloc(sizeof(double) * (size_t)t);
    uint64_t *T_row = malloc(sizeof(uint64_t) * (size_t)s), *T_col = malloc(sizeof(uint64_t) * (size_t)t);
    int64_t max_nI = 0, max_nJ = 0;
    for (int64_t i = 0; i < s; ++i)
        if (row_off[i + 1] - row_off[i] > max_nI) max_nI = row_off[i + 1] - row_off[i];
    for (int64_t j = 0; j < t; ++j)
        if (col_off[j + 1] - col_off[j] > max_nJ) max_nJ = col_off[j + 1] - col_off[j];
    const int nth = omp_get_max_threads();
    double *u = malloc(sizeof(double) * (size_t)max_nI);
    double *v = malloc(sizeof(double) * (size_t)max_nJ);
    double *vpart = calloc((size_t)nth * (size_t)max_nJ, sizeof(double));
    int status = 0;
    oracle_block_weights(A, m, n, lda, row_off, s, col_off, t, w_row, w_col);
    if (oracle_thresholds(w_row, s, T_row) != 0 || oracle_thresholds(w_col, t, T_col) != 0) {
        status = -1;
        goto done;
    }
    for (int64_t c = 0; c < n; ++c) x[c] = 0.0;
    for (int64_t r = 0; r < m; ++r) z[r] = b[r];
    for (int64_t k = 1; k <= max_iter; ++k) {
        uint64_t ctr[4] = {(uint64_t)(k - 1), sys, 0, 0}, key[2] = {seed, 0}, words[4];
        oracle_philox4x64_10(ctr, key, words);
        const int64_t j = oracle_pick(T_col, t, words[0]);
        const int64_t c_lo = col_off[j], nJ = col_off[j + 1] - c_lo;
        const double coef_c = alpha / w_col[j];
        const int64_t i = oracle_pick(T_row, s, words[1]);
        const int64_t r_lo = row_off[i], nI = row_off[i + 1] - r_lo;
        const double coef_r = alpha / w_row[i];
#pragma omp parallel
        {
            const int th = omp_get_thread_num();
            double *vp = vpart + (size_t)th * (size_t)max_nJ;
            for (int64_t c = 0; c < nJ; ++c) vp[c] = 0.0;
            /* v = A_{:,J}^T z: rows split over the threads, per-thread pieces */
#pragma omp for schedule(static)
            for (int64_t r = 0; r < m; ++r)
                for (int64_t c = 0; c < nJ; ++c) vp[c] = vp[c] + A[r * lda + c_lo + c] * z[r];
#pragma omp single
            for (int64_t c = 0; c < nJ; ++c) {
                double acc = 0.0;
                for (int q = 0; q < nth; ++q) acc = acc + vpart[(size_t)q * (size_t)max_nJ + c];
                v[c] = acc;
            }
            /* z -= coef_c A_{:,J} v */
#pragma omp for schedule(static)
            for (int64_t r = 0; r < m; ++r) {
                double acc = 0.0;
                for (int64_t c = 0; c < nJ; ++c) acc = acc + A[r * lda + c_lo + c] * v[c];
                z[r] = z[r] - coef_c * acc;
            }
            /* u = A_{I,:} x - b_I + z_I (uses the new z) */
#pragma omp for schedule(static)
            for (int64_t l = 0; l < nI; ++l) {
                double acc = 0.0;
                const double *row = A + (r_lo + l) * lda;
                for (int64_t c = 0; c < n; ++c) acc = acc + row[c] * x[c];
                u[l] = (acc - b[r_lo + l]) + z[r_lo + l];
            }
            /* x -= coef_r A_{I,:}^T u: columns split over the threads */
#pragma omp for schedule(static)
            for (int64_t c = 0; c < n; ++c) {
                double acc = 0.0;
                for (int64_t l = 0; l < nI; ++l) acc = acc + A[(r_lo + l) * lda + c] * u[l];
                x[c] = x[c] - coef_r * acc;
            }
        }
    }
done:
    free(w_row); free(w_col); free(T_row); free(T_col); free(u); free(v); free(vpart);
    return status;
}
