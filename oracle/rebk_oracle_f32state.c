/*
 * rebk_oracle_f32state.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * Algorithm 1 (Du, Si and Sun, arXiv:2001.04179, Section 2) with every
 * vector of the iteration (x, z, b and the block products u, v) held in
 * FP32 and every product and sum formed in FP32, on FP32 matrix values: the
 * "all-FP32" form of the method.  It exists to measure how far that form
 * gets (the GPU library keeps its iterates in FP64 because of it); the block
 * draws are the plain oracle's (same Philox stream, same FP64 weights of the
 * FP32 values), so the two forms visit the same blocks.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void oracle_block_weights(const double *A, int64_t m, int64_t n, int64_t lda,
                          const int64_t *row_off, int64_t s, const int64_t *col_off, int64_t t,
                          double *w_row, double *w_col);
int oracle_thresholds(const double *w, int64_t nb, uint64_t *T);
int64_t oracle_pick(const uint64_t *T, int64_t nb, uint64_t word);

/* A32 (m x n row-major FP32), from x0 = 0, z0 = b; every `every` iterations (and at the end)
 * err[q] receives ||x - x_ref|| / ||x_ref|| computed in FP64 from the FP32 x.  Returns 0, or -1. */
int oracle_rebk_f32state(const float *A32, int64_t m, int64_t n, const int64_t *row_off, int64_t s,
                         const int64_t *col_off, int64_t t, double alpha, uint64_t seed, const float *b32,
                         const double *x_ref, int64_t max_iter, int64_t every, double *err, float *x_out)
{
    if (m <= 0 || n <= 0 || s <= 0 || t <= 0 || every <= 0 || !(alpha > 0.0)) return -1;
    double *Ad = malloc(sizeof(double) * (size_t)m * (size_t)n);
    double *w_row = malloc(sizeof(double) * (size_t)s), *w_col = malloc(sizeof(double) * (size_t)t);
    uint64_t *T_row = malloc(sizeof(uint64_t) * (size_t)s), *T_col = malloc(sizeof(uint64_t) * (size_t)t);
    float *x = calloc((size_t)n, sizeof(float)), *z = malloc(sizeof(float) * (size_t)m);
    float *u = malloc(sizeof(float) * (size_t)m), *v = malloc(sizeof(float) * (size_t)n);
    int status = 0;
    for (int64_t q = 0; q < m * n; ++q) Ad[q] = (double)A32[q];
    oracle_block_weights(Ad, m, n, n, row_off, s, col_off, t, w_row, w_col);
    free(Ad);
    if (oracle_thresholds(w_row, s, T_row) != 0 || oracle_thresholds(w_col, t, T_col) != 0) {
        status = -1;
        goto done;
    }
    double xr2 = 0.0;
    for (int64_t c = 0; c < n; ++c) xr2 += x_ref[c] * x_ref[c];
    for (int64_t r = 0; r < m; ++r) z[r] = b32[r];
    int64_t q_out = 0;
    for (int64_t k = 1; k <= max_iter; ++k) {
        uint64_t ctr[4] = {(uint64_t)(k - 1), 0, 0, 0}, key[2] = {seed, 0}, words[4];
        oracle_philox4x64_10(ctr, key, words);
        const int64_t j = oracle_pick(T_col, t, words[0]);
        const int64_t c_lo = col_off[j], c_hi = col_off[j + 1];
        const float coef_c = (float)(alpha / w_col[j]);
        for (int64_t c = c_lo; c < c_hi; ++c) {
            float acc = 0.0f;
            for (int64_t r = 0; r < m; ++r) acc = acc + A32[r * n + c] * z[r];
            v[c - c_lo] = acc;
        }
        for (int64_t r = 0; r < m; ++r) {
            float acc = 0.0f;
            for (int64_t c = c_lo; c < c_hi; ++c) acc = acc + A32[r * n + c] * v[c - c_lo];
            z[r] = z[r] - coef_c * acc;
        }
        const int64_t i = oracle_pick(T_row, s, words[1]);
        const int64_t r_lo = row_off[i], r_hi = row_off[i + 1];
        const float coef_r = (float)(alpha / w_row[i]);
        for (int64_t r = r_lo; r < r_hi; ++r) {
            float acc = 0.0f;
            for (int64_t c = 0; c < n; ++c) acc = acc + A32[r * n + c] * x[c];
            u[r - r_lo] = (acc - b32[r]) + z[r];
        }
        for (int64_t c = 0; c < n; ++c) {
            float acc = 0.0f;
            for (int64_t r = r_lo; r < r_hi; ++r) acc = acc + A32[r * n + c] * u[r - r_lo];
            x[c] = x[c] - coef_r * acc;
        }
        if (k % every == 0 || k == max_iter) {
            double e2 = 0.0;
            for (int64_t c = 0; c < n; ++c) {
                const double d = (double)x[c] - x_ref[c];
                e2 += d * d;
            }
            err[q_out++] = sqrt(e2 / xr2);
        }
    }
    for (int64_t c = 0; c < n; ++c) x_out[c] = x[c];
done:
    free(w_row); free(w_col); free(T_row); free(T_col); free(x); free(z); free(u); free(v);
    return status;
}
