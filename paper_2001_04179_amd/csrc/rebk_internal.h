// Internal declarations shared by the library's translation units (kernels and host API).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rebk {

// Device-side status block written by the solve kernels.
struct DevStatus {
  int32_t status;      // rebk_status_t of the device loop
  int32_t stopped;     // 1 if the stop rule fired
  int64_t last_k;      // absolute iteration index of the returned x (k0 + iterations)
  double err2;         // ||x - x_ref||^2 at the last check (or -1)
  int64_t check_k;     // iteration of that check
};

// Everything a solve kernel needs; device pointers unless noted.
struct SolveArgs {
  const void* Arow;          // row panels: block i is an n x nI_i column-major panel at n*row_off[i]
  const void* Acol;          // column panels: A^T row-major with row stride ldc; block j is an m x nJ_j
                             // column-major panel (column stride ldc) at ldc*col_off[j]
  const int64_t* row_off;    // s+1
  const int64_t* col_off;    // t+1
  const uint64_t* T_row;     // s cumulative 53-bit thresholds
  const uint64_t* T_col;     // t cumulative 53-bit thresholds
  const double* coef_row;    // alpha / ||A_{I_i,:}||_F^2
  const double* coef_col;    // alpha / ||A_{:,J_j}||_F^2
  int64_t m, n;
  int64_t ldc;               // column-panel stride: m rounded up to kColAlign entries (pad entries are 0)
  int32_t s, t;
  int32_t max_nI, max_nJ;
  uint64_t seed, sys;
  const double* b;
  const double* x_in;        // NULL: x0 = 0
  const double* z_in;        // NULL: z0 = b
  double* x_out;
  double* z_out;             // may be NULL
  const double* x_ref;       // NULL: no reference error
  const double* g;           // NULL, or n entries: the z-step projects onto {A^T z = g} instead of
                             // {A^T z = 0} (correction equations of the refinement)
  double* y_out;             // NULL, or m entries: receives y with x - x_in = A^T y accumulated over
                             // this call's x-steps (y_I -= coef_I u), starting from 0
  double xref_sq;            // ||x_ref||^2 (host-computed)
  double tol;                // relative tolerance (<= 0: none)
  int64_t k0;
  int64_t max_iter;
  int64_t check_every;
  int32_t* trace_j;
  int32_t* trace_i;
  DevStatus* status;
};

// Synchronisation workspace of the persistent grid kernel (zeroed before every launch).
constexpr int kGridSumRing = 4;    // reduced vectors kept, one per epoch modulo the ring
constexpr int kGridSumCopies = 8;  // copies of each reduced vector (spread over memory channels)
struct GridSync {
  unsigned long long* part;  // 2 x grid vectors of stride epoch-tagged pairs (2 * stride words each)
  unsigned long long* gsum;  // kGridSumRing x kGridSumCopies reduced vectors (stride tagged pairs)
  int* timeout;              // set when a wait exceeded its spin limit
  int32_t stride;            // entries per vector (>= max_nJ + max_nI + 1, a multiple of 32)
};

// Static workspace of rebk_solve_ex_static (rebk_static.hip): room for the grid workspace of up to
// kStaticMaxGrid workgroups and a reduction stride of kStaticMaxStride entries, plus 64 words for
// the timeout flag and ||x_ref||^2.  4.25 MiB per device.
constexpr int kStaticMaxGrid = 256;
constexpr int kStaticMaxStride = 512;
constexpr size_t kStaticScratchWords = (size_t)2 * kStaticMaxGrid * kStaticMaxStride * 2 +
                                       (size_t)kGridSumRing * kGridSumCopies * kStaticMaxStride * 2 + 64;
// Address of this device's static workspace (kStaticScratchWords words), looked up once per device
// with that device current.
hipError_t static_scratch(int device, unsigned long long** ptr);
hipError_t launch_fill_zero(unsigned long long* p, size_t n, hipStream_t st);
// *out = sum of v[q]^2 in index order (one thread; the same value as a sequential host loop)
hipError_t launch_sumsq_in_order(const double* v, int64_t n, double* out, hipStream_t st);

// One system of a batch: its panels, tables and Philox stream (device copy of the handle's data).
struct BatchSys {
  const void* Arow;          // row panels, as in SolveArgs
  const void* Acol;          // column panels (A^T row-major, row stride ldc), as in SolveArgs
  const int64_t* row_off;
  const int64_t* col_off;
  const uint64_t* T_row;
  const uint64_t* T_col;
  const double* coef_row;
  const double* coef_col;
  int64_t m, n;
  int64_t ldc;
  int32_t s, t;
  int32_t max_nI, max_nJ;
  uint64_t seed, sys;
};

// The work of one workgroup: R right-hand sides of one system, solved together (they share the
// block sequence, so every panel element read serves all R of them).
struct BatchTask {
  int32_t sys;               // index into the BatchSys array; -1: empty slot
  int32_t R;                 // right-hand sides: 1, 2 or 4
  const double* b;           // R vectors of length m, one after another
  const double* x_in;        // R vectors of length n, or NULL (x0 = 0)
  const double* x_ref;       // R vectors of length n, or NULL (no error check)
  double* x_out;             // R vectors of length n
  double* z_out;             // R vectors of length m, or NULL
  int64_t* iters_out;        // one value: iterations run
  double* err2_out;          // R values: ||x - x_ref||^2 at the last check (-1 if none)
  double* xref2_out;         // R values: ||x_ref||^2
  int32_t* status_out;       // one value: 0 stopped on tol, 1 max_iter reached, 2 diverged
};

struct BatchArgs {
  const BatchSys* sys;
  const BatchTask* tasks;
  int32_t ntasks;
  int32_t max_nJ, max_nI;    // over the batch (LDS layout)
  int64_t max_iter;
  double tol;                // relative tolerance per right-hand side (<= 0: none)
  int64_t check_every;
  int32_t z0_from_x0;        // with x_in: start from z0 = b - A x0 (else z0 = b)
};

// Launchers (defined in rebk_kernels.hip).  All return hipError_t.
// Column panels store every column of A in a run of ldc = roundup(m, kColAlign) entries, so every
// run starts at a multiple of kColAlign entries (vector loads of 4 entries stay aligned).
constexpr int64_t kColAlign = 16;
inline int64_t col_stride(int64_t m) { return (m + kColAlign - 1) / kColAlign * kColAlign; }

hipError_t launch_pack(const void* A, int a_dtype, int64_t lda, int panel_dtype, int64_t m, int64_t n, int64_t ldc,
                       const int64_t* row_off_d, const int64_t* col_off_d, const int32_t* rowblk_d,
                       const int32_t* colblk_d, void* Arow, void* Acol, hipStream_t st);
hipError_t launch_finite_check(const void* A, int a_dtype, int64_t lda, int64_t m, int64_t n, int* bad,
                               hipStream_t st);
hipError_t launch_block_weights(const void* Arow, const void* Acol, int panel_dtype, int64_t m, int64_t n, int64_t ldc,
                                const int64_t* row_off_d, int32_t s, const int64_t* col_off_d, int32_t t,
                                const int32_t* rowblk_d, double* row_sq, double* colrow_sq, double* w_row,
                                double* w_col, hipStream_t st);
hipError_t launch_sample(const uint64_t* T_row, int32_t s, const uint64_t* T_col, int32_t t, uint64_t seed,
                         uint64_t sys, int64_t k0, int64_t count, int32_t* j_out, int32_t* i_out,
                         hipStream_t st);
hipError_t launch_philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                         int64_t count, uint64_t* out, hipStream_t st);
hipError_t launch_wg_solve(const SolveArgs& a, int panel_dtype, int threads, size_t lds_bytes, hipStream_t st);
size_t wg_solve_lds_bytes(const SolveArgs& a);
// row_lds: stage the row slabs in LDS (else the x-steps read them from HBM)
hipError_t launch_grid_solve(const SolveArgs& a, const GridSync& gs, int panel_dtype, int grid, bool row_lds,
                             hipStream_t st);
size_t grid_solve_lds_bytes(const SolveArgs& a, int grid, int panel_dtype, bool row_lds);
hipError_t grid_solve_max_blocks(int panel_dtype, size_t lds_bytes, bool row_lds, int* blocks_per_cu);
// Pipelined whole-chip kernel (rebk_grid.hip): G = A A^T (m x m), H = A^T A (n x n) and A
// row-major (m x n), all FP64 from the stored panel values; GridSync.part holds 4 x grid vectors.
// Its broadcast vector has at most kPipeMaxStride entries (8 registers per lane of one wave).
constexpr int kPipeMaxStride = 256;
constexpr int kPipeThreads = 512;  // eight waves: the broadcast, two per update, a gather, two copiers
hipError_t launch_pipe_solve(const SolveArgs& a, const GridSync& gs, const double* Gm, const double* Hm,
                             const double* Arm, int panel_dtype, int grid, hipStream_t st);
size_t pipe_solve_lds_bytes(const SolveArgs& a, int grid, int stride, int panel_dtype);
hipError_t pipe_solve_max_blocks(int panel_dtype, size_t lds_bytes, int* blocks_per_cu);
// A (stored panel values) as a row-major FP64 m x n matrix
hipError_t launch_unpack_rows(const void* Arow, int panel_dtype, int64_t n, const int64_t* row_off_d, int32_t s,
                              double* out, hipStream_t st);
hipError_t launch_residual(const void* Arow, const void* Acol, int panel_dtype, const SolveArgs& a,
                           const double* x, const double* z, double* partials, int nparts, hipStream_t st);
size_t batch_lds_bytes(int64_t m, int64_t n, int R, int max_nJ, int max_nI, int threads);
// One launch runs tasks of one tile width R (1, 2 or 4).
hipError_t launch_batch_solve(const BatchArgs& a, int panel_dtype, int threads, int R, size_t lds_bytes,
                              hipStream_t st);
hipError_t batch_max_blocks(int panel_dtype, int threads, int R, size_t lds_bytes, int* blocks_per_cu);
// Gram matrix of one block's shorter side: G[a1][a2] = sum_{t < L} X(a1, t) X(a2, t) with
// X(a, t) = panel[base + a * sa + t * st]; G stored row-major (d x d) at gram offset `gram`.
struct GramDesc {
  int64_t base;
  int64_t L;
  int64_t sa, st;
  int64_t gram;
  int32_t d;
  int32_t pad;
};
hipError_t launch_gram(const void* P, int panel_dtype, const GramDesc* desc, int ntiles, const int32_t* tile_block,
                       const int32_t* tile_a1, const int32_t* tile_a2, double* gram, hipStream_t st);
hipError_t launch_power(const GramDesc* desc, int nblocks, int max_d, const double* gram, int max_steps, double rtol,
                        double* lam, double* trace, int32_t* steps, hipStream_t st);

// warm-start network kernels (half-precision operands, FP32 accumulation)
hipError_t launch_gemm_f16(bool ta, bool tb, int M, int N, int K, float alpha, const _Float16* A, int lda,
                           const _Float16* B, int ldb, float beta, float* C, int ldc, hipStream_t st);
hipError_t launch_to_half_f64(const double* in, int64_t count, double scale, _Float16* out, hipStream_t st);
hipError_t launch_to_half_f32(const float* in, int64_t count, _Float16* out, hipStream_t st);
hipError_t launch_bias_act(const float* C, const float* bias, int64_t rows, int cols, int relu, _Float16* out16,
                           float* out32, hipStream_t st);
hipError_t launch_mlp_residual(const float* X0, const double* Xt, int64_t count, float* R, double* part_sq,
                               float* part_max, int nparts, hipStream_t st);
hipError_t launch_scale_half(const float* in, int64_t count, float s, _Float16* out, hipStream_t st);
hipError_t launch_relu_back(const float* D, const _Float16* H, int64_t count, _Float16* out, hipStream_t st);
hipError_t launch_colsum_half(const _Float16* D, int rows, int cols, float scale, float* out, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1, float omb1,
                       float b2, float omb2, float eps, float c1, float c2, _Float16* p16, hipStream_t st);
hipError_t launch_init_uniform(float* p, int64_t count, float bound, uint64_t seed, uint64_t tag, hipStream_t st);
hipError_t launch_widen(const float* in, int64_t count, double* out, hipStream_t st);
hipError_t launch_gemm_f64(int M, int N, int K, double alpha, const double* A, int lda, const double* B, int ldb,
                           double* C, int ldc, hipStream_t st);

// refinement kernels (FP64, caller's row-major A with leading dimension lda)
int64_t refine_chunks(int64_t m);  // row chunks of the transposed product (partial: chunks x n doubles)
hipError_t launch_resid_f(const double* A, int64_t lda, int64_t m, int64_t n, const double* b, const double* z,
                          const double* x, double* f, hipStream_t st);
hipError_t launch_gemv_t(const double* A, int64_t lda, int64_t m, int64_t n, const double* v, double alpha,
                         double beta, double* out, double* sq, double* partial, hipStream_t st);
hipError_t launch_axpy(double* y, const double* x, int64_t n, hipStream_t st);
hipError_t launch_sumsq(const double* v, int64_t n, double* partials, int nparts, hipStream_t st);
hipError_t launch_sumsq_matrix(const double* A, int64_t lda, int64_t m, int64_t n, double* partials, int nparts,
                               hipStream_t st);
hipError_t launch_err2(const double* x, const double* x_ref, int64_t n, double* partials, int nparts,
                       hipStream_t st);

constexpr int kGridThreads = 256;
constexpr int kWgThreads = 256;

}  // namespace rebk
