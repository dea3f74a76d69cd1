/*
 * rebk_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, FP64 CPU implementation of the randomized extended block
 * Kaczmarz method (REBK) of Du, Si and Sun, "Randomized extended block
 * Kaczmarz for solving least squares" (arXiv:2001.04179), Section 2,
 * Algorithm 1.  It is the parity reference for the GPU library: only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or helper with the GPU library.
 *
 * Everything is written as plain loops in the order the paper states the
 * computation; the only choices the paper leaves open are fixed here:
 *
 *  - block weights ||A_{:,J_j}||_F^2 and ||A_{I_i,:}||_F^2 (Algorithm 1, the
 *    two "pick" steps) are summed in one fixed order: per matrix row, the
 *    squares of the row's entries inside the block in ascending column
 *    order; then those row partials in ascending row order.  Every product
 *    is rounded and then added (this file must be compiled with
 *    -ffp-contract=off), so the weights are reproducible bit for bit;
 *  - the block draw turns one 64-bit Philox word into a 53-bit integer d and
 *    picks the first block whose cumulative threshold
 *    T_j = floor(C_j / C_total * 2^53) exceeds d (T_last = 2^53), where C_j
 *    are the prefix sums of the weights.  A zero-weight block has
 *    T_j = T_{j-1} and is never drawn;
 *  - iteration k (1-based, Algorithm 1) draws its two blocks from
 *    Philox4x64-10 with counter (k-1, sys, 0, 0) and key (seed, 0): word 0
 *    picks the column block, word 1 the row block.
 *
 * Philox4x64-10 follows Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11 (round function, multipliers and Weyl
 * key increments as published there).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- Philox */

#define ORC_PHILOX_M0 0xD2E7470EE14C6C93ULL /* multiplier for counter word 0 */
#define ORC_PHILOX_M1 0xCA5A826395121157ULL /* multiplier for counter word 2 */
#define ORC_PHILOX_W0 0x9E3779B97F4A7C15ULL /* key increment, golden ratio */
#define ORC_PHILOX_W1 0xBB67AE8584CAA73BULL /* key increment, sqrt(3) - 1 */

static void orc_mulhilo(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* One Philox4x64 bijection of 10 rounds: out = Philox(ctr, key). */
void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { /* the key schedule bumps the key before every round but the first */
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        orc_mulhilo(ORC_PHILOX_M0, c0, &hi0, &lo0);
        orc_mulhilo(ORC_PHILOX_M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------- weights and sampling */

/*
 * Squared Frobenius norms of the row blocks A_{I_i,:} and the column blocks
 * A_{:,J_j} (the sampling weights of Algorithm 1), in the fixed order stated
 * in the header.  A is row-major with leading dimension lda.  Partitions are
 * contiguous: block i holds rows row_off[i] .. row_off[i+1]-1.
 */
void oracle_block_weights(const double *A, int64_t m, int64_t n, int64_t lda,
                          const int64_t *row_off, int64_t s,
                          const int64_t *col_off, int64_t t,
                          double *w_row, double *w_col)
{
    (void)m;
    for (int64_t i = 0; i < s; ++i) {
        double acc = 0.0;
        for (int64_t r = row_off[i]; r < row_off[i + 1]; ++r) {
            double row_part = 0.0;
            for (int64_t c = 0; c < n; ++c) {
                double a = A[r * lda + c];
                double sq = a * a;
                row_part = row_part + sq;
            }
            acc = acc + row_part;
        }
        w_row[i] = acc;
    }
    for (int64_t j = 0; j < t; ++j) {
        double acc = 0.0;
        for (int64_t r = 0; r < m; ++r) {
            double row_part = 0.0;
            for (int64_t c = col_off[j]; c < col_off[j + 1]; ++c) {
                double a = A[r * lda + c];
                double sq = a * a;
                row_part = row_part + sq;
            }
            acc = acc + row_part;
        }
        w_col[j] = acc;
    }
}

/*
 * Cumulative integer thresholds for drawing block j with probability
 * w[j] / sum(w) (Algorithm 1).  Returns -1 if the weights do not sum to a
 * positive finite number.
 */
int oracle_thresholds(const double *w, int64_t nb, uint64_t *T)
{
    const double two53 = 9007199254740992.0;
    double total = 0.0;
    for (int64_t l = 0; l < nb; ++l) {
        if (!(w[l] >= 0.0)) return -1;
        total = total + w[l];
    }
    if (!(total > 0.0) || !isfinite(total)) return -1;
    double C = 0.0;
    for (int64_t j = 0; j + 1 < nb; ++j) {
        C = C + w[j];
        T[j] = (uint64_t)floor(C / total * two53);
    }
    T[nb - 1] = (uint64_t)1 << 53;
    return 0;
}

/* First block j whose threshold exceeds the top 53 bits of the word. */
int64_t oracle_pick(const uint64_t *T, int64_t nb, uint64_t word)
{
    uint64_t d = word >> 11;
    int64_t j = 0;
    while (j < nb - 1 && !(d < T[j])) ++j;
    return j;
}

/* ------------------------------------------------------------------ REBK */

static double orc_rel_err(const double *x, const double *xr, int64_t n)
{
    double num = 0.0, den = 0.0;
    for (int64_t c = 0; c < n; ++c) {
        double d = x[c] - xr[c];
        num = num + d * d;
        den = den + xr[c] * xr[c];
    }
    if (den > 0.0) return sqrt(num) / sqrt(den);
    return sqrt(num);
}

/*
 * Run REBK (Algorithm 1) from (x0, z0) for iterations k0+1 .. k0+max_iter.
 *
 *   A        m x n, row-major, leading dimension lda (FP64)
 *   row_off  s+1 offsets of the contiguous row partition, 0 .. m
 *   col_off  t+1 offsets of the contiguous column partition, 0 .. n
 *   alpha    the constant stepsize of Algorithm 1
 *   seed,sys Philox key word and the second counter word (system id)
 *   b        right-hand side (m)
 *   x0, z0   starting iterates; NULL means x0 = 0, z0 = b (Section 3)
 *   k0       number of iterations already done (the Philox counter offset)
 *   x_ref    if not NULL: stop at the first k with ||x^k-x_ref||/||x_ref|| < tol
 *   x, z     outputs (n and m)
 *   j_trace, i_trace  if not NULL: the 0-based blocks drawn at each step
 *   iters    the number of iterations performed
 *   err      the last relative error (or -1 without x_ref)
 *
 * Returns 0 (stopped on tol or no x_ref given), 1 (max_iter reached with
 * x_ref given and tol not met), -1 (invalid input).
 */
/*
 * Algorithm 1's iteration with two optional extensions used by the refinement below:
 *   g (n entries): the z-step uses v = A_J^T z - g_J, i.e. it projects onto {A^T z = g};
 *   y (m entries): set to 0, then y_I -= coef_I u after every x-step, so that x - x0 = A^T y.
 * With g = y = NULL this is exactly Algorithm 1.
 */
static int orc_iterate(const double *A, int64_t m, int64_t n, int64_t lda,
                       const int64_t *row_off, int64_t s,
                       const int64_t *col_off, int64_t t,
                       double alpha, uint64_t seed, uint64_t sys,
                       const double *b, const double *x0, const double *z0,
                       int64_t k0, int64_t max_iter,
                       const double *x_ref, double tol,
                       const double *g, double *y,
                       double *x, double *z,
                       int32_t *j_trace, int32_t *i_trace,
                       int64_t *iters, double *err)
{
    if (m <= 0 || n <= 0 || s <= 0 || t <= 0 || lda < n || !(alpha > 0.0)) return -1;
    double *w_row = (double *)malloc(sizeof(double) * (size_t)s);
    double *w_col = (double *)malloc(sizeof(double) * (size_t)t);
    uint64_t *T_row = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)s);
    uint64_t *T_col = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)t);
    int64_t max_nI = 0, max_nJ = 0;
    for (int64_t i = 0; i < s; ++i)
        if (row_off[i + 1] - row_off[i] > max_nI) max_nI = row_off[i + 1] - row_off[i];
    for (int64_t j = 0; j < t; ++j)
        if (col_off[j + 1] - col_off[j] > max_nJ) max_nJ = col_off[j + 1] - col_off[j];
    double *u = (double *)malloc(sizeof(double) * (size_t)(max_nI > 0 ? max_nI : 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(max_nJ > 0 ? max_nJ : 1));
    int status = 0;

    oracle_block_weights(A, m, n, lda, row_off, s, col_off, t, w_row, w_col);
    if (oracle_thresholds(w_row, s, T_row) != 0 || oracle_thresholds(w_col, t, T_col) != 0) {
        status = -1;
        goto done;
    }

    /* initial iterates (Algorithm 1; Section 3 uses z0 = b, x0 = 0) */
    for (int64_t c = 0; c < n; ++c) x[c] = x0 ? x0[c] : 0.0;
    for (int64_t r = 0; r < m; ++r) z[r] = z0 ? z0[r] : b[r];
    if (y)
        for (int64_t r = 0; r < m; ++r) y[r] = 0.0;

    *iters = 0;
    *err = -1.0;
    if (x_ref) status = 1;
    for (int64_t step = 0; step < max_iter; ++step) {
        int64_t k = k0 + step + 1; /* Algorithm 1 counts k = 1, 2, ... */
        uint64_t ctr[4] = {(uint64_t)(k - 1), sys, 0, 0};
        uint64_t key[2] = {seed, 0};
        uint64_t words[4];
        oracle_philox4x64_10(ctr, key, words);

        /* pick j with probability ||A_{:,J_j}||_F^2 / ||A||_F^2 */
        int64_t j = oracle_pick(T_col, t, words[0]);
        int64_t c_lo = col_off[j], c_hi = col_off[j + 1];
        double coef_c = alpha / w_col[j];
        /* z^k = z^{k-1} - alpha/||A_{:,J}||_F^2 * A_{:,J} (A_{:,J}^T z^{k-1}) */
        for (int64_t c = c_lo; c < c_hi; ++c) {
            double acc = 0.0;
            for (int64_t r = 0; r < m; ++r) acc = acc + A[r * lda + c] * z[r];
            v[c - c_lo] = g ? acc - g[c] : acc;
        }
        for (int64_t r = 0; r < m; ++r) {
            double acc = 0.0;
            for (int64_t c = c_lo; c < c_hi; ++c) acc = acc + A[r * lda + c] * v[c - c_lo];
            z[r] = z[r] - coef_c * acc;
        }

        /* pick i with probability ||A_{I_i,:}||_F^2 / ||A||_F^2 */
        int64_t i = oracle_pick(T_row, s, words[1]);
        int64_t r_lo = row_off[i], r_hi = row_off[i + 1];
        double coef_r = alpha / w_row[i];
        /* x^k = x^{k-1} - alpha/||A_{I,:}||_F^2 * A_{I,:}^T (A_{I,:} x^{k-1} - b_I + z^k_I) */
        for (int64_t r = r_lo; r < r_hi; ++r) {
            double acc = 0.0;
            for (int64_t c = 0; c < n; ++c) acc = acc + A[r * lda + c] * x[c];
            u[r - r_lo] = (acc - b[r]) + z[r];
        }
        for (int64_t c = 0; c < n; ++c) {
            double acc = 0.0;
            for (int64_t r = r_lo; r < r_hi; ++r) acc = acc + A[r * lda + c] * u[r - r_lo];
            x[c] = x[c] - coef_r * acc;
        }
        if (y)
            for (int64_t r = r_lo; r < r_hi; ++r) y[r] = y[r] - coef_r * u[r - r_lo];

        if (j_trace) j_trace[step] = (int32_t)j;
        if (i_trace) i_trace[step] = (int32_t)i;
        *iters = step + 1;
        if (x_ref) {
            *err = orc_rel_err(x, x_ref, n);
            if (*err < tol) {
                status = 0;
                break;
            }
        }
    }

done:
    free(w_row); free(w_col); free(T_row); free(T_col); free(u); free(v);
    return status;
}

int oracle_rebk_solve(const double *A, int64_t m, int64_t n, int64_t lda,
                      const int64_t *row_off, int64_t s,
                      const int64_t *col_off, int64_t t,
                      double alpha, uint64_t seed, uint64_t sys,
                      const double *b, const double *x0, const double *z0,
                      int64_t k0, int64_t max_iter,
                      const double *x_ref, double tol,
                      double *x, double *z,
                      int32_t *j_trace, int32_t *i_trace,
                      int64_t *iters, double *err)
{
    return orc_iterate(A, m, n, lda, row_off, s, col_off, t, alpha, seed, sys, b, x0, z0, k0, max_iter,
                       x_ref, tol, NULL, NULL, x, z, j_trace, i_trace, iters, err);
}

/*
 * Iterative refinement of the augmented system of least squares, REBK as the inner solver.
 * (Not in the paper: an FP64 outer loop around Algorithm 1, so that the inner iterations may
 * run on rounded panel values.)
 *
 * The solution pair of  z + A x = b,  A^T z = 0,  x in range(A^T)  is z = (I - A A^+) b (the limit
 * of Lemma 6) and x = A^+ b (the limit of Theorem 7).  For a current pair (z, x) the residuals
 *   f = b - z - A x,   g = -A^T z
 * define the correction (dz, dx):  dz + A dx = f,  A^T dz = g.  Algorithm 1 solves it when its
 * z-step projects onto {A^T dz = g} (v = A_J^T dz - g_J) and its x-step solves A dx = f - dz,
 * started from dz = f, dx = 0 (z0 in f + range(A), x0 in range(A^T) as Theorem 7 asks).
 * The inner iterations run on Ast (the stored, possibly rounded, values; the block weights and
 * sampling tables are Ast's), the residuals and the update of x on the FP64 A:
 *   z += dz,   x += A^T dy   (dy: the x-steps' coefficients, dx = Ast^T dy),
 * so x stays in range(A^T) whatever the rounding of Ast.  The inner block sequence continues
 * the Philox counter across outer steps (outer step q runs iterations q*inner_iters + 1 ...).
 *
 * Stop rule, tested before every outer step and after the last one: with x_ref,
 * ||x - x_ref|| / ||x_ref|| < tol; without, ||f|| <= tol ||b|| and ||g|| <= tol ||A||_F ||b||.
 * err_trace (max_outer + 1 entries, may be NULL) receives the tested quantity (with x_ref the
 * relative error, else max(||f|| / ||b||, ||g|| / (||A||_F ||b||))) before each outer step.
 * Returns 0 (stopped on tol), 1 (max_outer reached), -1 (invalid input).
 */
int oracle_rebk_refine(const double *A, const double *Ast, int64_t m, int64_t n, int64_t lda,
                       const int64_t *row_off, int64_t s,
                       const int64_t *col_off, int64_t t,
                       double alpha, uint64_t seed, uint64_t sys,
                       const double *b, const double *x0, const double *x_ref, double tol,
                       int64_t inner_iters, int64_t max_outer,
                       double *x, double *z, double *err_trace,
                       int64_t *outer_done, int64_t *iters, double *err)
{
    if (m <= 0 || n <= 0 || lda < n || inner_iters <= 0 || max_outer < 0) return -1;
    double *f = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)malloc(sizeof(double) * (size_t)n);
    double *dz = (double *)malloc(sizeof(double) * (size_t)m);
    double *dx = (double *)malloc(sizeof(double) * (size_t)n);
    double *dy = (double *)malloc(sizeof(double) * (size_t)m);
    int status = 1;
    double bn = 0.0, an = 0.0;
    for (int64_t r = 0; r < m; ++r) bn = bn + b[r] * b[r];
    for (int64_t r = 0; r < m; ++r)
        for (int64_t c = 0; c < n; ++c) an = an + A[r * lda + c] * A[r * lda + c];
    bn = sqrt(bn);
    an = sqrt(an);
    for (int64_t c = 0; c < n; ++c) x[c] = x0 ? x0[c] : 0.0;
    for (int64_t r = 0; r < m; ++r) z[r] = b[r];
    *iters = 0;
    *outer_done = 0;
    for (int64_t q = 0;; ++q) {
        /* f = b - z - A x, g = -A^T z (FP64, plain loops) */
        double f2 = 0.0, g2 = 0.0;
        for (int64_t r = 0; r < m; ++r) {
            double acc = 0.0;
            for (int64_t c = 0; c < n; ++c) acc = acc + A[r * lda + c] * x[c];
            f[r] = (b[r] - z[r]) - acc;
            f2 = f2 + f[r] * f[r];
        }
        for (int64_t c = 0; c < n; ++c) {
            double acc = 0.0;
            for (int64_t r = 0; r < m; ++r) acc = acc + A[r * lda + c] * z[r];
            g[c] = -acc;
            g2 = g2 + g[c] * g[c];
        }
        double e;
        int ok;
        if (x_ref) {
            e = orc_rel_err(x, x_ref, n);
            ok = e < tol;
        } else {
            double rf = sqrt(f2) / (bn > 0.0 ? bn : 1.0);
            double rg = sqrt(g2) / (an * bn > 0.0 ? an * bn : 1.0);
            e = rf > rg ? rf : rg;
            ok = rf <= tol && rg <= tol;
        }
        if (err_trace) err_trace[q] = e;
        *err = e;
        if (ok) { status = 0; break; }
        if (q == max_outer) break;
        /* correction: Algorithm 1 on (f, g) from dz = f, dx = 0 */
        int64_t it = 0;
        double ie = -1.0;
        int st = orc_iterate(Ast, m, n, lda, row_off, s, col_off, t, alpha, seed, sys, f, NULL, f,
                             q * inner_iters, inner_iters, NULL, 0.0, g, dy, dx, dz, NULL, NULL, &it, &ie);
        if (st < 0) { status = -1; break; }
        *iters += it;
        /* z += dz, x += A^T dy */
        for (int64_t r = 0; r < m; ++r) z[r] = z[r] + dz[r];
        for (int64_t c = 0; c < n; ++c) {
            double acc = 0.0;
            for (int64_t r = 0; r < m; ++r) acc = acc + A[r * lda + c] * dy[r];
            x[c] = x[c] + acc;
        }
        *outer_done = q + 1;
    }
    free(f); free(g); free(dz); free(dx); free(dy);
    return status;
}

/* Philox words for counters (c0 + q, c1, c2, c3), q = 0 .. count-1, key (k0, k1): out[4q + w]. */
void oracle_philox_fill(const uint64_t ctr[4], const uint64_t key[2], int64_t count, uint64_t *out)
{
    for (int64_t q = 0; q < count; ++q) {
        uint64_t c[4] = {ctr[0] + (uint64_t)q, ctr[1], ctr[2], ctr[3]};
        oracle_philox4x64_10(c, key, out + 4 * q);
    }
}

/* Blocks drawn at iterations k0+1 .. k0+count of system sys (see the header). */
int oracle_sample_blocks(const double *w_row, int64_t s, const double *w_col, int64_t t,
                         uint64_t seed, uint64_t sys, int64_t k0, int64_t count,
                         int32_t *j_out, int32_t *i_out)
{
    uint64_t *T_row = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)s);
    uint64_t *T_col = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)t);
    int status = 0;
    if (oracle_thresholds(w_row, s, T_row) != 0 || oracle_thresholds(w_col, t, T_col) != 0) {
        status = -1;
    } else {
        for (int64_t q = 0; q < count; ++q) {
            uint64_t ctr[4] = {(uint64_t)(k0 + q), sys, 0, 0};
            uint64_t key[2] = {seed, 0};
            uint64_t words[4];
            oracle_philox4x64_10(ctr, key, words);
            j_out[q] = (int32_t)oracle_pick(T_col, t, words[0]);
            i_out[q] = (int32_t)oracle_pick(T_row, s, words[1]);
        }
    }
    free(T_row);
    free(T_col);
    return status;
}
