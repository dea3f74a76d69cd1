/*
 * rebk.h -- C ABI of librebk.so, a gfx950 (MI355X) implementation of the
 * randomized extended block Kaczmarz method (REBK) of Du, Si and Sun,
 * "Randomized extended block Kaczmarz for solving least squares",
 * arXiv:2001.04179.
 *
 * REBK (Section 2, Algorithm 1) approximates the minimum-norm least-squares
 * solution A^+ b of any linear system A x = b (consistent or not, over- or
 * underdetermined, full rank or not; Section 1).  Given partitions
 * {I_1..I_s} of the rows and {J_1..J_t} of the columns and a stepsize
 * alpha > 0, iteration k = 1, 2, ... does
 *
 *   j  ~ P(j) = ||A_{:,J_j}||_F^2 / ||A||_F^2
 *   z <- z - alpha / ||A_{:,J_j}||_F^2 * A_{:,J_j} (A_{:,J_j}^T z)
 *   i  ~ P(i) = ||A_{I_i,:}||_F^2 / ||A||_F^2
 *   x <- x - alpha / ||A_{I_i,:}||_F^2 * A_{I_i,:}^T (A_{I_i,:} x - b_{I_i} + z_{I_i})
 *
 * with z^0 = b and x^0 = 0 in the paper's experiments (Section 3).  x^k
 * converges in mean square to A^+ b when z^0 is in b + range(A), x^0 is in
 * range(A^T) and 0 < alpha < 2 / beta_max (Theorem 7, Remark 9).
 *
 * Conventions shared by every entry point:
 *  - Pointers named *_dev are device pointers (HIP global memory) owned by
 *    the caller; the library never frees them.  Host pointers are named
 *    without the suffix.  Vectors are dense and contiguous.
 *  - Block partitions are contiguous: block i holds rows
 *    row_offsets[i] .. row_offsets[i+1]-1 (offsets strictly increasing from
 *    0 to m); likewise for columns.  Section 3 uses equal blocks of size tau
 *    with a smaller last block.
 *  - Random draws: iteration k (1-based) draws both blocks from one
 *    Philox4x64-10 output (Salmon et al., SC'11) with counter
 *    (k-1, system, 0, 0) and key (seed, 0); word 0 picks the column block
 *    and word 1 the row block.  The top 53 bits of a word are compared
 *    against cumulative integer thresholds floor(C_j / C_total * 2^53) of
 *    the prefix sums C_j of the block weights (last threshold 2^53): the
 *    block drawn is the first whose threshold exceeds them.  Block weights
 *    are summed in FP64 in a fixed order (per matrix row, squares of the
 *    entries in ascending column order; then rows in ascending order;
 *    every product rounded before it is added), so the block sequence is
 *    reproducible bit for bit by any implementation of the same rules.
 *  - Work is enqueued on the handle's HIP stream.  Calls that return
 *    results in host memory synchronize that stream before returning.
 *  - Return codes: REBK_OK (0) or a rebk_status_t.  Negative codes are
 *    failures; the message of the last failure on the calling thread is
 *    returned by rebk_last_error().  REBK_ERR_INVALID leaves outputs
 *    untouched.  After REBK_ERR_HIP or REBK_ERR_TIMEOUT the handle must be
 *    destroyed.  Nothing in the library aborts or exits the process.
 *  - A handle is not thread-safe; use one handle per stream.
 */
#ifndef REBK_H
#define REBK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rebk_handle *rebk_handle_t;

/* Element types.  REBK_F64 and REBK_F32 are accepted for the caller's A;
 * every type is accepted for the stored panels; the iterates are FP64. */
typedef enum {
    REBK_F64 = 0,
    REBK_F32 = 1,
    REBK_BF16 = 2,
    REBK_F16 = 3
} rebk_dtype_t;

typedef enum {
    REBK_OK = 0,              /* stopped on the tolerance, or ran max_iter without a stop rule */
    REBK_NOT_CONVERGED = 1,   /* max_iter reached before the tolerance; outputs are written */
    REBK_DIVERGED = 2,        /* the error or residual became non-finite or grew 1e6-fold */
    REBK_ERR_INVALID = -1,    /* bad argument; nothing was written */
    REBK_ERR_HIP = -2,        /* a HIP runtime call failed */
    REBK_ERR_OOM = -3,        /* device allocation failed */
    REBK_ERR_TIMEOUT = -4     /* a wait of a persistent kernel (grid or team) exceeded its spin limit */
} rebk_status_t;

/* Which kernel runs the iterations. */
typedef enum {
    REBK_KERNEL_AUTO = 0,     /* WORKGROUP for tiny systems (m |J| + |I| n + 4 (m + n) <= 8192); else PIPE
                                 when its Gram matrices exist (rebk_pipe_prepare, or an earlier
                                 PIPE solve on the handle), the panels are narrower than FP64 and
                                 the call fits its limits; else GRID */
    REBK_KERNEL_WORKGROUP = 1,/* one workgroup runs the whole solve (small systems) */
    REBK_KERNEL_GRID = 2,     /* one persistent cooperative grid, one grid-wide reduction per
                                 iteration; needs ceil(n / grid) + 8 <= 256 owned columns, blocks
                                 of at most 256 columns and its slabs within 160 KB of LDS */
    REBK_KERNEL_PIPE = 3      /* the grid kernel pipelined over three iterations: the same
                                 iterates of Algorithm 1 (Section 2), the next steps' block
                                 products formed from x and z two and three iterations old and
                                 corrected with the Gram matrices A A^T and A^T A, so only one
                                 grid-wide broadcast per iteration is on the critical path.  Builds
                                 A A^T, A^T A and a row-major copy of A in FP64 on first use
                                 (8 (m^2 + n^2 + m n) bytes, kept until rebk_destroy or
                                 rebk_pipe_release; see rebk_pipe_prepare).  The column limits
                                 of GRID; its own LDS layout (5 slabs of each kind, sized by the
                                 most rows and columns a workgroup owns) within 150 KB;
                                 max|I| + max|J| + 1 <= the grid size and <= 256 (after rounding
                                 up to a multiple of 32); all workgroups co-resident; no
                                 refinement steps (rebk_solve_refined) and no static workspace */
} rebk_kernel_t;

typedef struct {
    int32_t status;      /* rebk_status_t of the solve */
    int32_t kernel;      /* rebk_kernel_t that ran */
    int64_t iterations;  /* iterations performed in this call (k counts from k0) */
    double rel_err;      /* ||x - x_ref|| / ||x_ref|| at the last check (x_ref mode),
                            max(||b - z - A x|| / ||b||, ||A^T z|| / (||A||_F ||b||)) (residual
                            mode), or -1 if nothing was checked */
    double time_ms;      /* device time of the iterations, HIP events on the handle's stream */
} rebk_result_t;

/* Options of rebk_solve_ex.  Zero-initialise and set what you need. */
typedef struct {
    const double *b_dev;     /* right-hand side, m entries (required) */
    const double *x0_dev;    /* initial x, n entries; NULL means 0 (Section 3) */
    const double *z0_dev;    /* initial z, m entries; NULL means b (Section 3) */
    int64_t k0;              /* iterations already done: this call runs k0+1, k0+2, ...
                                (resuming with the x, z of an earlier call continues that
                                run exactly) */
    int64_t max_iter;        /* at most this many iterations in this call (> 0) */
    const double *x_ref_dev; /* if not NULL, stop at the first checked k with
                                ||x^k - x_ref|| / ||x_ref|| < tol (a reference solution,
                                typically A^+ b; the experiments of Section 3 stop on the
                                true error) */
    double tol;              /* tolerance; <= 0 runs exactly max_iter iterations */
    int64_t check_every;     /* check the stop rule every this many iterations; 0 means 1
                                with x_ref and 256 in residual mode */
    double *x_out_dev;       /* result x, n entries (required; may alias x0_dev) */
    double *z_out_dev;       /* result z, m entries, or NULL (may alias z0_dev) */
    int32_t *trace_j_dev;    /* if not NULL: 0-based column block of each iteration (max_iter) */
    int32_t *trace_i_dev;    /* if not NULL: 0-based row block of each iteration (max_iter) */
    int32_t kernel;          /* rebk_kernel_t */
    int32_t grid_wgs;        /* GRID kernel: workgroups (0 = one per compute unit) */
} rebk_solve_opts_t;

/*
 * Create a solver for A (m x n, row-major, leading dimension lda >= n,
 * element type a_dtype in {REBK_F64, REBK_F32}) with the given contiguous
 * partitions (host arrays of s+1 and t+1 offsets), stepsize alpha > 0 and
 * Philox seed (Algorithm 1).
 *
 * A is copied into library-owned device panels stored as panel_dtype:
 * every row block as an n x |I_i| column-major panel, and A^T row-major, so
 * that column block j is |J_j| contiguous columns of m entries; both block
 * reads of an iteration are contiguous.  A may be freed when the call returns.  The FP64 block
 * weights ||A_{I_i,:}||_F^2 and ||A_{:,J_j}||_F^2 of the stored values and the
 * sampling thresholds are computed here (the only host synchronisation).
 *
 * stream is a hipStream_t (NULL for the default stream).  Errors:
 * REBK_ERR_INVALID for bad sizes, offsets, dtype or alpha, or if A has a
 * non-finite entry or ||A||_F = 0; REBK_ERR_OOM; REBK_ERR_HIP.
 */
int rebk_create(rebk_handle_t *out, const void *A_dev, int32_t a_dtype, int32_t panel_dtype,
                int64_t m, int64_t n, int64_t lda,
                const int64_t *row_offsets, int64_t s,
                const int64_t *col_offsets, int64_t t,
                double alpha, uint64_t seed, void *stream);

/* Release the handle and its device memory (NULL is ignored). */
void rebk_destroy(rebk_handle_t h);

/*
 * Solve with the plain interface: z^0 = b, x^0 = x0_dev (NULL means 0), at
 * most max_iter iterations, residual stop rule
 *   ||b - z - A x|| <= tol ||b||  and  ||A^T z|| <= tol ||A||_F ||b||
 * checked every 256 iterations (z converges to (I - A A^+) b, Lemma 6, and
 * then A x converges to A A^+ b).  x_out_dev receives x (n entries).
 * res (host, may be NULL) receives the result.  Returns the solve status.
 */
int rebk_solve(rebk_handle_t h, const double *b_dev, const double *x0_dev, double *x_out_dev,
               double tol, int64_t max_iter, rebk_result_t *res);

/* Solve with every option (see rebk_solve_opts_t).  Returns the solve status. */
int rebk_solve_ex(rebk_handle_t h, const rebk_solve_opts_t *opts, rebk_result_t *res);

/*
 * rebk_solve_ex for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, but the grid kernel's workspace (partial
 * sums, reduced vectors, timeout flag) and the ||x_ref||^2 slot come from a
 * static array the library holds on every device it runs on (4.25 MiB,
 * room for up to 256 workgroups and blocks with max|I| + max|J| + 1 <= 512),
 * cleared by a kernel at each call.  The caller passes inputs and outputs
 * as for rebk_solve_ex.  Only the error (x_ref) and fixed-count stop rules
 * are available: residual mode (x_ref NULL with tol > 0) returns
 * REBK_ERR_INVALID, as does REBK_KERNEL_PIPE, a system whose grid workspace
 * exceeds the static array, or a current device other than the handle's.  Every call on
 * a device shares that device's array and leaves the last call's contents
 * in it: calls that overlap on one device (several streams or host threads)
 * race and must be serialised by the caller.  Synchronizes the handle's
 * stream.  Returns the solve status.
 */
int rebk_solve_ex_static(rebk_handle_t h, const rebk_solve_opts_t *opts, rebk_result_t *res);

/*
 * Build now what REBK_KERNEL_PIPE needs (A A^T, A^T A and a row-major copy of
 * A, FP64 from the stored panel values, 8 (m^2 + n^2 + m n) bytes of device
 * memory); otherwise the first pipelined solve builds them, before its timed
 * region.  The products run through rocBLAS dgemm on the handle's stream.
 * build_ms (host, may be NULL) receives the build time in milliseconds (0 if
 * they were already built).  Synchronizes the handle's stream.  Errors:
 * REBK_ERR_INVALID for a NULL handle, REBK_ERR_OOM when the memory is not
 * available, REBK_ERR_HIP for a failed product.
 */
int rebk_pipe_prepare(rebk_handle_t h, double *build_ms);

/* Free what rebk_pipe_prepare built (NULL or nothing built is ignored). */
void rebk_pipe_release(rebk_handle_t h);

/*
 * Copy the FP64 block weights to host arrays w_row (s entries, ||A_{I_i,:}||_F^2)
 * and w_col (t entries, ||A_{:,J_j}||_F^2); either may be NULL.  Algorithm 1
 * (Section 2) draws column block j with probability ||A_{:,J_j}||_F^2 / ||A||_F^2
 * and row block i with probability ||A_{I_i,:}||_F^2 / ||A||_F^2; these are the
 * numerators, summed in FP64 in a fixed order (per row, squares in ascending
 * column order; then rows ascending; no fused multiply-add).  Errors:
 * REBK_ERR_INVALID for a NULL handle.
 */
int rebk_get_weights(rebk_handle_t h, double *w_row, double *w_col);

/*
 * Copy the sampling thresholds of Algorithm 1's two draws (Section 2) to host
 * arrays T_row (s entries) and T_col (t entries), either may be NULL:
 * T_j = floor(C_j / C_t * 2^53) for the prefix sums C_j of the weights above
 * (T_t = 2^53).  A 53-bit uniform draw d picks the first block with d < T_j, so
 * block j is drawn with probability (T_j - T_{j-1}) / 2^53, its weight's share
 * of the total rounded to 53 bits; a zero-weight block is never drawn.
 * Errors: REBK_ERR_INVALID for a NULL handle.
 */
int rebk_get_thresholds(rebk_handle_t h, uint64_t *T_row, uint64_t *T_col);

/* Sizes of the handle: m, n, s, t, the largest row block and the largest column block. */
int rebk_get_info(rebk_handle_t h, int64_t *m, int64_t *n, int64_t *s, int64_t *t,
                  int64_t *max_row_block, int64_t *max_col_block);

/*
 * Run only the block sampler of the handle on the device: the two block
 * draws of Algorithm 1 (Section 2; column block j first, then row block i)
 * for iterations k0+1 .. k0+count of system `system`.  Iteration k takes the
 * words of Philox4x64-10(counter (k-1, system, 0, 0), key (seed, 0)): the top
 * 53 bits of word 0 draw j, those of word 1 draw i, against the thresholds of
 * rebk_get_thresholds.  j_out_dev[q] and i_out_dev[q] (device int32, count
 * entries each, owned by the caller) receive the 0-based blocks of iteration
 * k0+q+1.  Synchronizes the stream.  Errors: REBK_ERR_INVALID for a NULL
 * handle or output, count < 0 or k0 < 0; REBK_ERR_HIP.
 */
int rebk_sample_blocks(rebk_handle_t h, uint64_t system, int64_t k0, int64_t count,
                       int32_t *j_out_dev, int32_t *i_out_dev);

/*
 * Philox4x64-10 on the device, as used by the sampler: for q in [0, count),
 * out_dev[4q .. 4q+3] = Philox(counter = (c0 + q, c1, c2, c3), key = (k0, k1)).
 * stream as in rebk_create.  Synchronizes the stream.
 */
int rebk_philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                       uint64_t k0, uint64_t k1, int64_t count, uint64_t *out_dev, void *stream);

/* ------------------------------------------------------------------------
 * Mixed precision with FP64 refinement.  The panels of the handle may hold
 * rounded values (BF16, FP16, FP32); the iteration then converges to the
 * least-squares solution of the rounded matrix.  This solve wins the
 * accuracy back with an outer loop in FP64 on the augmented system of least
 * squares  z + A x = b,  A^T z = 0,  x in range(A^T)  (its solution is
 * z = (I - A A^+) b, the limit of Lemma 6, and x = A^+ b, Theorem 7):
 *   f = b - z - A x,  g = -A^T z             (FP64, caller's A)
 *   correction: Algorithm 1 on the panels with the z-step projecting onto
 *     {A^T dz = g} (v = A_J^T dz - g_J) and the x-step solving A dx = f - dz,
 *     from dz = f, dx = 0, for inner_iters iterations; y accumulates the
 *     x-steps (dx = A_panels^T y)
 *   z += dz,  x += A^T y                      (FP64, caller's A: x stays in
 *                                              range(A^T) exactly)
 * The inner block sequence continues one Philox stream: outer step q runs
 * iterations q * inner_iters + 1 .. (q + 1) * inner_iters of the handle's
 * seed and system 0.
 * ------------------------------------------------------------------------ */
typedef struct {
    const double *A_dev;      /* the FP64 matrix the handle was created from (or its exact
                                 values), m x n row-major with leading dimension lda (required;
                                 read-only, caller-owned, valid during the call) */
    int64_t lda;
    const double *b_dev;      /* right-hand side, m entries (required) */
    const double *x0_dev;     /* starting x in range(A^T), n entries; NULL means 0 */
    const double *x_ref_dev;  /* if not NULL, stop when ||x - x_ref|| / ||x_ref|| < tol; else
                                 when ||f|| <= tol ||b|| and ||g|| <= tol ||A||_F ||b|| */
    double tol;               /* tested before every outer step and after the last one */
    int64_t inner_iters;      /* REBK iterations per correction solve (> 0) */
    int32_t max_outer;        /* outer steps at most (>= 0) */
    int32_t kernel;           /* rebk_kernel_t of the inner solves */
    int32_t grid_wgs;         /* as in rebk_solve_opts_t */
    double *x_out_dev;        /* result x, n entries (required) */
    double *z_out_dev;        /* result z, m entries, or NULL */
    double *err_trace;        /* host, max_outer + 1 entries, or NULL: the tested quantity
                                 (relative error, or max of the two relative residuals) before
                                 each outer step; entries after the last test are left as is */
} rebk_refine_opts_t;

/*
 * Solve by FP64 refinement around REBK (see above).  res (host, may be
 * NULL): status (REBK_OK when the stop rule held, else REBK_NOT_CONVERGED),
 * iterations = inner iterations in total, rel_err = the last tested
 * quantity, time_ms = device time of the whole loop.  Errors:
 * REBK_ERR_INVALID (bad options or sizes), REBK_ERR_OOM, REBK_ERR_HIP,
 * REBK_ERR_TIMEOUT.  Synchronizes the stream once per outer step.
 */
int rebk_solve_refined(rebk_handle_t h, const rebk_refine_opts_t *opts, rebk_result_t *res);

/* ------------------------------------------------------------------------
 * Batched solves: many independent systems, each with several right-hand
 * sides, in one call.  Every right-hand side is an exact REBK run
 * (Algorithm 1) with z^0 = b and x^0 = x0 (or 0); the right-hand sides of
 * one system share its block sequence, drawn from the Philox stream of the
 * system's id (the counter's second word), so each panel read serves all
 * of them.  Independent systems and right-hand sides are the units the
 * method parallelises over without any exchange between them.
 * ------------------------------------------------------------------------ */
typedef struct rebk_batch *rebk_batch_t;

/*
 * Group nsys existing handles (created with the same panel_dtype and on the
 * same device) into a batch.  sys_ids (host, nsys entries, may be NULL
 * meaning 0, 1, ..., nsys-1) gives each system's Philox system id.  The
 * batch refers to the handles' panels and tables: destroy the batch before
 * any of its handles.  stream as in rebk_create.  Errors: REBK_ERR_INVALID
 * (nsys < 1, a NULL handle, mixed panel types), REBK_ERR_OOM, REBK_ERR_HIP.
 */
int rebk_batch_create(rebk_batch_t *out, int32_t nsys, const rebk_handle_t *systems,
                      const uint64_t *sys_ids, void *stream);

/* Release the batch (not its handles; NULL is ignored). */
void rebk_batch_destroy(rebk_batch_t b);

/* Options of rebk_batch_solve and rebk_batch_autotune.  Zero-initialise. */
typedef struct {
    const int32_t *nrhs;            /* host, nsys entries: right-hand sides of system s (1..2^20) */
    const double *const *b_dev;     /* host array of nsys device pointers: nrhs[s] right-hand
                                       sides of m_s entries each, one after another (required) */
    const double *const *x0_dev;    /* NULL, or host array of nsys device pointers (entries may be
                                       NULL meaning x0 = 0): nrhs[s] x n_s starting points */
    const double *const *x_ref_dev; /* NULL, or host array of nsys device pointers: nrhs[s] x n_s
                                       references (typically A^+ b); required for the stop rule */
    double *const *x_out_dev;       /* host array of nsys device pointers: nrhs[s] x n_s results
                                       (required) */
    double *const *z_out_dev;       /* NULL, or host array of nsys device pointers: nrhs[s] x m_s */
    int64_t max_iter;               /* iterations at most (> 0) */
    double tol;                     /* a group of right-hand sides solved together stops at the
                                       first check where every one of them has
                                       ||x - x_ref|| / ||x_ref|| < tol; <= 0: run max_iter */
    int64_t check_every;            /* check interval (0 means 16) */
    int32_t threads;                /* threads per workgroup: 256, 512 or 1024 (0: tuned, else 512) */
    int32_t lds_budget;             /* LDS bytes per workgroup for the iterates (0: tuned, else
                                       the largest that fits) */
    int32_t max_tile;               /* most right-hand sides per workgroup: 1, 2 or 4
                                       (0: tuned, else 4) */
    int32_t xcd_order;              /* 1: dispatch the tasks of a system to one XCD (shared L2);
                                       0: plain longest-first order; -1: tuned (default 1) */
    int32_t z0_from_x0;             /* 1: where x0 is given, start from z0 = b - A x0 (computed from
                                       the stored panels) instead of z0 = b; a right-hand side
                                       whose ||b - A x0|| >= ||b|| falls back to x0 = 0, z0 = b */
    int32_t team;                   /* teams of workgroups (below): 0 automatic, -1 never, P > 0
                                       every system in teams of P workgroups (P <= 256; not with
                                       z0_from_x0) */
} rebk_batch_opts_t;

/* Result of one right-hand side of a batch. */
typedef struct {
    int64_t iterations;  /* iterations run (shared by the right-hand sides solved together) */
    double rel_err;      /* ||x - x_ref|| / ||x_ref|| at the last check, or -1 */
    int32_t status;      /* REBK_OK, REBK_NOT_CONVERGED or REBK_DIVERGED */
    int32_t tile;        /* right-hand sides solved together with this one */
    int32_t team;        /* workgroups that solved them together (0: one workgroup) */
} rebk_batch_rhs_t;

/*
 * Solve every right-hand side of every system of the batch.  Each
 * workgroup takes up to max_tile right-hand sides of one system and keeps
 * their iterates (m + n) x tile in LDS, so each system needs 8 (m + n)
 * bytes plus a little under the LDS budget.  A system's tile width is the
 * widest that fits, narrowed for systems whose single tile would outlast
 * the average load of a compute unit in the previous solve.  The tiles of
 * each width run as one kernel; the kernels of different widths run at
 * the same time on two library streams forked from and joined back into
 * the batch's stream.
 * Teams: a system whose narrowest tile alone would still outlast the average
 * load of a compute unit in the previous solve (and whose iteration reads
 * enough panel to gain from more compute units) is solved by teams instead:
 * tiles of up to 16 right-hand sides, each split over P workgroups that own
 * slices of its rows and columns and combine their block products through a
 * reduction in device memory every iteration.  All teams run in one
 * cooperative launch on the batch's stream before the other tiles, sharing
 * the compute units in proportion to their work.  Teams keep the iteration
 * and stop rule of the other tiles, with the products summed in another
 * order.  Not used with z0_from_x0.  out (host, sum of nrhs entries, system after
 * system) receives per right-hand side results; time_ms (host, may be
 * NULL) the device time from the first launch to the join.
 * Returns REBK_OK when every right-hand side stopped on the tolerance (or
 * no stop rule was given), else REBK_NOT_CONVERGED or REBK_DIVERGED; errors
 * REBK_ERR_INVALID (bad options, a system too large for LDS, forced teams
 * that do not fit the device), REBK_ERR_OOM, REBK_ERR_HIP, REBK_ERR_TIMEOUT
 * (a team's reduction exceeded its spin limit).  Synchronizes the stream.
 */
int rebk_batch_solve(rebk_batch_t b, const rebk_batch_opts_t *opts, rebk_batch_rhs_t *out,
                     double *time_ms);

/*
 * Choose threads per workgroup, LDS budget, tile size and task order for
 * this batch by timing probe_iters iterations (no stop rule) of each
 * candidate on the given options (whose x_out buffers are overwritten).
 * The choice is kept in the batch and used by later solves whose options
 * leave those fields at 0 / -1; it is also returned (host pointers, may be
 * NULL).  Synchronizes the stream.
 */
int rebk_batch_autotune(rebk_batch_t b, const rebk_batch_opts_t *opts, int64_t probe_iters,
                        int32_t *threads, int32_t *lds_budget, int32_t *max_tile, int32_t *xcd_order,
                        double *best_ms);

/*
 * Block constants of Section 2.2 for the stepsize (Remark 9: alpha = 1 / beta_max, and any
 * 0 < alpha < 2 / beta_max converges):
 *   beta_row[i] = ||A_{I_i,:}||_2^2 / ||A_{I_i,:}||_F^2   (s entries, host, may be NULL)
 *   beta_col[j] = ||A_{:,J_j}||_2^2 / ||A_{:,J_j}||_F^2   (t entries, host, may be NULL)
 *   *beta_max   = the largest of them                      (host, may be NULL)
 * of the stored panel values.  Each block's Gram matrix of its shorter side d (at most 8192) is
 * formed on the device in FP64; its largest eigenvalue is the Rayleigh quotient of a power
 * iteration, stopped when it changes by at most rtol relative or after max_steps steps
 * (*steps_max, may be NULL, receives the most steps any block took).  The quotient approaches
 * the eigenvalue from below, at a rate set by the ratio of the two largest eigenvalues.
 * Allocates sum d^2 doubles of scratch for the call.  Synchronizes the stream.
 */
int rebk_block_betas(rebk_handle_t h, int32_t max_steps, double rtol, double *beta_row, double *beta_col,
                     double *beta_max, int32_t *steps_max);

/* ------------------------------------------------------------------------
 * Learned warm start.  A network maps a right-hand side b to y; the start
 * x0 = A^T y lies in range(A^T) and z0 = b - A x0 in b + range(A), the
 * hypotheses of Theorem 7, so REBK from (x0, z0) still converges to A^+ b
 * (plain REBK from x0 = 0, z0 = b is the fallback, taken where
 * ||b - A x0|| >= ||b||).  The network is
 *   h1 = relu(W1 (s b) + c1),  h2 = relu(W2 h1 + c2),  y = W3 h2 + c3,
 *   x0 = out_scale A^T y
 * (s: a scale of the input), trained with Adam (Kingma and Ba) on
 *   loss = 1 / (2 batch) * sum over the batch ||x0 - x_target||^2.
 * Every product runs on the matrix cores with half-precision operands and
 * FP32 accumulation; the weights have FP32 masters.  Batches are row-major
 * (one right-hand side per row), batch a multiple of 64 up to max_batch.
 * ------------------------------------------------------------------------ */
typedef struct rebk_mlp *rebk_mlp_t;

/*
 * Create a network in_dim -> hidden -> hidden -> out_dim for the matrix A
 * (A_dev: out_dim x n, FP64 row-major, copied in half precision; out_dim is
 * m), with x0 = out_scale A^T y (out_scale > 0, e.g. 1/sqrt(m) so that y is
 * of order one).  All sizes must be positive multiples of 64.  Weights start
 * uniform in +-1/sqrt(fan_in) from Philox4x64-10 with the given seed, biases
 * at zero.  Errors: REBK_ERR_INVALID, REBK_ERR_OOM, REBK_ERR_HIP.
 */
int rebk_mlp_create(rebk_mlp_t *out, int32_t in_dim, int32_t hidden, const double *A_dev,
                    int64_t out_dim, int64_t n, double out_scale, int32_t max_batch, uint64_t seed,
                    void *stream);
void rebk_mlp_destroy(rebk_mlp_t w);

/* Copy parameters from / to host FP32 arrays (W1 hidden x in_dim, c1 hidden, W2 hidden x hidden,
 * c2 hidden, W3 out_dim x hidden, c3 out_dim; row-major); NULL entries are skipped. */
int rebk_mlp_set_params(rebk_mlp_t w, const float *W1, const float *c1, const float *W2,
                        const float *c2, const float *W3, const float *c3);
int rebk_mlp_get_params(rebk_mlp_t w, float *W1, float *c1, float *W2, float *c2, float *W3,
                        float *c3);

/* Inference: X0_dev (batch x n, FP64) = rows of out_scale A^T y for the rows of B_dev (batch x
 * in_dim, FP64, scaled by b_scale), formed in FP64 from the FP64 A so that x0 lies in range(A^T)
 * to FP64 rounding (training uses the half-precision product); Y_dev (batch x out_dim, FP64)
 * receives y if not NULL. */
int rebk_mlp_forward(rebk_mlp_t w, const double *B_dev, int32_t batch, double b_scale,
                     double *X0_dev, double *Y_dev);

/* Gradients of the loss for the batch (B_dev as above, Xt_dev batch x n FP64 targets), kept in the
 * network; *loss (host, may be NULL) receives the loss.  rebk_mlp_get_grads copies them to host
 * FP32 arrays laid out like the parameters. */
int rebk_mlp_grad(rebk_mlp_t w, const double *B_dev, const double *Xt_dev, int32_t batch,
                  double b_scale, double *loss);
int rebk_mlp_get_grads(rebk_mlp_t w, float *gW1, float *gc1, float *gW2, float *gc2, float *gW3,
                       float *gc3);

/* One Adam step with the kept gradients (beta1, beta2 in [0, 1), eps > 0). */
int rebk_mlp_adam(rebk_mlp_t w, double lr, double beta1, double beta2, double eps);

/* rebk_mlp_grad followed by rebk_mlp_adam(lr, 0.9, 0.999, 1e-8). */
int rebk_mlp_train_step(rebk_mlp_t w, const double *B_dev, const double *Xt_dev, int32_t batch,
                        double b_scale, double lr, double *loss);

/* Message of the last failing call on this thread ("" if none). */
const char *rebk_last_error(void);

/* Library version string. */
const char *rebk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* REBK_H */
