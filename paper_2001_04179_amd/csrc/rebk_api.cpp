// Host runtime of librebk.so: argument validation, device memory, sampling tables and the
// solve drivers behind the C ABI declared in include/rebk.h.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "rebk.h"
#include "rebk_internal.h"
#include "rebk_team.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(REBK_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

size_t dtype_size(int dt) {
  switch (dt) {
    case REBK_F64: return 8;
    case REBK_F32: return 4;
    case REBK_BF16: return 2;
    case REBK_F16: return 2;
    default: return 0;
  }
}

// Cumulative 53-bit thresholds of weights w: T_j = floor(C_j / C_total * 2^53), last = 2^53,
// with C_j the prefix sums in index order.
bool build_thresholds(const std::vector<double>& w, std::vector<uint64_t>& T) {
  const double two53 = 9007199254740992.0;
  double total = 0.0;
  for (double x : w) {
    if (!(x >= 0.0)) return false;
    total = total + x;
  }
  if (!(total > 0.0) || !std::isfinite(total)) return false;
  T.assign(w.size(), 0);
  double C = 0.0;
  for (size_t j = 0; j + 1 < w.size(); ++j) {
    C = C + w[j];
    T[j] = (uint64_t)std::floor(C / total * two53);
  }
  T.back() = (uint64_t)1 << 53;
  return true;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

}  // namespace

struct rebk_handle {
  int64_t m = 0, n = 0, s = 0, t = 0;
  int64_t ldc = 0;  // column-panel stride (m rounded up)
  int32_t max_nI = 0, max_nJ = 0;
  int panel_dtype = 0;
  double alpha = 0.0;
  uint64_t seed = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int cus = 0;
  double fro2 = 0.0;  // ||A||_F^2 (row-weight total)
  std::vector<int64_t> row_off, col_off;
  std::vector<double> w_row, w_col;
  std::vector<uint64_t> T_row_h, T_col_h;
  // device memory
  void* Arow = nullptr;
  void* Acol = nullptr;
  int64_t* row_off_d = nullptr;
  int64_t* col_off_d = nullptr;
  uint64_t* T_row = nullptr;
  uint64_t* T_col = nullptr;
  double* coef_row = nullptr;
  double* coef_col = nullptr;
  rebk::DevStatus* status_d = nullptr;
  double* partials = nullptr;  // residual / error partial sums
  int nparts = 0;
  // grid workspace
  unsigned long long* part = nullptr;
  unsigned long long* gsum = nullptr;
  int* timeout = nullptr;
  size_t part_cap = 0;
  size_t gsum_cap = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // pipelined kernel: A A^T (m x m), A^T A (n x n), A row-major (m x n), FP64
  double* pipe_G = nullptr;
  double* pipe_H = nullptr;
  double* pipe_Arm = nullptr;

  void release_pipe() {
    dfree(pipe_G);
    dfree(pipe_H);
    dfree(pipe_Arm);
  }

  ~rebk_handle() {
    dfree(Arow);
    dfree(Acol);
    dfree(row_off_d);
    dfree(col_off_d);
    dfree(T_row);
    dfree(T_col);
    dfree(coef_row);
    dfree(coef_col);
    dfree(status_d);
    dfree(partials);
    dfree(part);
    dfree(gsum);
    dfree(timeout);
    release_pipe();
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

namespace {

int check_offsets(const int64_t* off, int64_t nb, int64_t total, const char* what, int32_t* maxsz) {
  if (!off) return fail(REBK_ERR_INVALID, "%s offsets are NULL", what);
  if (nb <= 0 || nb > (1ll << 30)) return fail(REBK_ERR_INVALID, "%s block count %lld out of range", what, (long long)nb);
  if (off[0] != 0 || off[nb] != total)
    return fail(REBK_ERR_INVALID, "%s offsets must start at 0 and end at %lld", what, (long long)total);
  int64_t mx = 0;
  for (int64_t i = 0; i < nb; ++i) {
    if (off[i + 1] <= off[i]) return fail(REBK_ERR_INVALID, "%s offsets must be strictly increasing", what);
    if (off[i + 1] - off[i] > mx) mx = off[i + 1] - off[i];
  }
  if (mx > (1 << 20)) return fail(REBK_ERR_INVALID, "%s block of %lld is too large", what, (long long)mx);
  *maxsz = (int32_t)mx;
  return REBK_OK;
}

int ensure_grid_workspace(rebk_handle* h, size_t part_words, size_t gsum_words) {
  if (part_words > h->part_cap) {
    dfree(h->part);
    if (hipMalloc((void**)&h->part, part_words * sizeof(unsigned long long)) != hipSuccess)
      return fail(REBK_ERR_OOM, "cannot allocate %zu partial-sum words", part_words);
    h->part_cap = part_words;
  }
  if (gsum_words > h->gsum_cap) {
    dfree(h->gsum);
    if (hipMalloc((void**)&h->gsum, gsum_words * sizeof(unsigned long long)) != hipSuccess)
      return fail(REBK_ERR_OOM, "cannot allocate %zu group-sum words", gsum_words);
    h->gsum_cap = gsum_words;
  }
  if (!h->timeout && hipMalloc((void**)&h->timeout, sizeof(int)) != hipSuccess)
    return fail(REBK_ERR_OOM, "cannot allocate the timeout flag");
  return REBK_OK;
}

rebk::SolveArgs base_args(const rebk_handle* h) {
  rebk::SolveArgs a{};
  a.Arow = h->Arow;
  a.Acol = h->Acol;
  a.row_off = h->row_off_d;
  a.col_off = h->col_off_d;
  a.T_row = h->T_row;
  a.T_col = h->T_col;
  a.coef_row = h->coef_row;
  a.coef_col = h->coef_col;
  a.m = h->m;
  a.n = h->n;
  a.ldc = h->ldc;
  a.s = (int32_t)h->s;
  a.t = (int32_t)h->t;
  a.max_nI = h->max_nI;
  a.max_nJ = h->max_nJ;
  a.seed = h->seed;
  a.sys = 0;
  a.status = h->status_d;
  return a;
}

// Sum of nparts partial sums copied to the host (fixed order).
int host_sum(rebk_handle* h, const double* dev, int cnt, double* out) {
  std::vector<double> buf(cnt);
  HIP_TRY(hipMemcpyAsync(buf.data(), dev, cnt * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  double s = 0.0;
  for (double v : buf) s += v;
  *out = s;
  return REBK_OK;
}

bool wg_fits(const rebk_handle* h, const rebk::SolveArgs& a) {
  return rebk::wg_solve_lds_bytes(a) <= 150 * 1024;
}

// The pipelined kernel's FP64 operands: A row-major from the row panels, then G = A A^T and
// H = A^T A with rocBLAS (the row-major A is the column-major n x m matrix X = A^T, so
// G = X^T X and H = X X^T).  *ms: build time (0 when already built).
int ensure_pipe(rebk_handle* h, double* ms) {
  if (ms) *ms = 0.0;
  if (h->pipe_G) return REBK_OK;
  const int64_t m = h->m, n = h->n;
  if (m > INT32_MAX || n > INT32_MAX) return fail(REBK_ERR_INVALID, "pipelined kernel: dimensions beyond 32 bits");
  const size_t bytes = 8 * ((size_t)m * m + (size_t)n * n + (size_t)m * n);
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  if (bytes + ((size_t)1 << 30) > free_b)
    return fail(REBK_ERR_OOM, "pipelined kernel: %zu bytes of Gram matrices exceed free memory (%zu)", bytes, free_b);
  const auto t0 = std::chrono::steady_clock::now();
  if (hipMalloc((void**)&h->pipe_Arm, 8 * (size_t)m * n) != hipSuccess ||
      hipMalloc((void**)&h->pipe_G, 8 * (size_t)m * m) != hipSuccess ||
      hipMalloc((void**)&h->pipe_H, 8 * (size_t)n * n) != hipSuccess) {
    h->release_pipe();
    return fail(REBK_ERR_OOM, "pipelined kernel: cannot allocate %zu bytes", bytes);
  }
  hipError_t e = rebk::launch_unpack_rows(h->Arow, h->panel_dtype, n, h->row_off_d, (int32_t)h->s, h->pipe_Arm,
                                          h->stream);
  if (e != hipSuccess) {
    h->release_pipe();
    return fail(REBK_ERR_HIP, "unpack of A: %s", hipGetErrorString(e));
  }
  rocblas_handle bh = nullptr;
  rocblas_status bs = rocblas_create_handle(&bh);
  if (bs == rocblas_status_success) bs = rocblas_set_stream(bh, h->stream);
  if (bs == rocblas_status_success) bs = rocblas_set_atomics_mode(bh, rocblas_atomics_not_allowed);  // reproducible
  const double one = 1.0, zero = 0.0;
  const rocblas_int M = (rocblas_int)m, N = (rocblas_int)n;
  if (bs == rocblas_status_success)
    bs = rocblas_dgemm(bh, rocblas_operation_transpose, rocblas_operation_none, M, M, N, &one, h->pipe_Arm, N,
                       h->pipe_Arm, N, &zero, h->pipe_G, M);
  if (bs == rocblas_status_success)
    bs = rocblas_dgemm(bh, rocblas_operation_none, rocblas_operation_transpose, N, N, M, &one, h->pipe_Arm, N,
                       h->pipe_Arm, N, &zero, h->pipe_H, N);
  e = hipStreamSynchronize(h->stream);
  if (bh) (void)rocblas_destroy_handle(bh);
  if (bs != rocblas_status_success || e != hipSuccess) {
    h->release_pipe();
    return fail(REBK_ERR_HIP, "Gram products: rocBLAS status %d, %s", (int)bs, hipGetErrorString(e));
  }
  if (ms) ms[0] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return REBK_OK;
}

// Grid workspace handed in by the caller instead of the handle's: `words` words at `base`, cleared
// with a fill kernel (no allocation, no memset node).
struct FixedWorkspace {
  unsigned long long* base;
  size_t words;
};

// Whether the pipelined kernel runs this call on a grid of G workgroups; else the reason in why
// (when given).
bool pipe_fits(const rebk_handle* h, const rebk::SolveArgs& a, int G, char* why) {
  auto no = [&](const char* fmt, long long v1, long long v2, long long v3) {
    if (why) snprintf(why, 256, fmt, v1, v2, v3);
    return false;
  };
  if (a.g || a.y_out) return no("the pipelined kernel runs no refinement steps", 0, 0, 0);
  if (a.max_iter > INT32_MAX - 64) return no("the pipelined kernel runs at most %lld iterations per call", INT32_MAX - 64, 0, 0);
  if (G > 1024) return no("at most 1024 workgroups in the pipelined kernel (grid %lld)", G, 0, 0);
  const int stride = ((h->max_nJ + h->max_nI + 1 + 31) / 32) * 32;
  if (stride > G || stride > rebk::kPipeMaxStride)
    return no("pipelined kernel: %lld broadcast entries need as many workgroups (grid %lld) and at most %lld",
              stride, G, rebk::kPipeMaxStride);
  if ((h->n + G - 1) / G + 8 > rebk::kGridThreads)
    return no("too many columns per workgroup (%lld); use a larger grid", (h->n + G - 1) / G, 0, 0);
  if (h->max_nJ > rebk::kGridThreads)
    return no("column blocks wider than %lld columns need the one-workgroup kernel", rebk::kGridThreads, 0, 0);
  const size_t lds = rebk::pipe_solve_lds_bytes(a, G, stride, h->panel_dtype);
  if (lds > 150 * 1024) return no("pipelined kernel needs %lld bytes of LDS per workgroup", (long long)lds, 0, 0);
  int per_cu = 0;
  if (rebk::pipe_solve_max_blocks(h->panel_dtype, lds, &per_cu) != hipSuccess)
    return no("occupancy query of the pipelined kernel failed", 0, 0, 0);
  if (per_cu <= 0 || G > per_cu * h->cus)
    return no("grid of %lld workgroups cannot be co-resident (%lld per CU)", G, per_cu, 0);
  return true;
}

// One call of the iteration kernel for iterations k0+1 .. k0+iters.
int run_iterations(rebk_handle* h, rebk::SolveArgs a, int kernel, int grid_wgs, int* used_kernel,
                   const FixedWorkspace* fixed = nullptr) {
  if (kernel == REBK_KERNEL_AUTO) {
    // One workgroup wins only for tiny systems: per iteration it walks both blocks and all of z
    // and x.  Measured on MI355X: 5.7 us vs 7.3 us (whole chip) at 250 x 120 with 10 x 10 blocks,
    // 8.7 vs 7.5 at 500 x 250, 23 vs 8 at 1000 x 100 with 100 x 10 blocks.  Past that the
    // pipelined kernel, once its Gram matrices exist (rebk_pipe_prepare or an earlier pipelined
    // solve), where it fits: 3.6 us vs 7.8 us per iteration on the 20000 x 2000 workload with FP32
    // panels.  Not for FP64 panels: their slabs are twice the bytes its copy waves stage, and it
    // measured 9.5 us there against 8.3 us for the grid kernel.
    const double work = (double)h->m * h->max_nJ + (double)h->n * h->max_nI + 4.0 * (double)(h->m + h->n);
    if (wg_fits(h, a) && work <= 8192.0)
      kernel = REBK_KERNEL_WORKGROUP;
    else if (!fixed && h->pipe_G && h->panel_dtype != REBK_F64 &&
             pipe_fits(h, a, grid_wgs > 0 ? grid_wgs : h->cus, nullptr))
      kernel = REBK_KERNEL_PIPE;
    else
      kernel = REBK_KERNEL_GRID;
  }
  *used_kernel = kernel;
  if (kernel == REBK_KERNEL_WORKGROUP) {
    if (!wg_fits(h, a)) return fail(REBK_ERR_INVALID, "system too large for the one-workgroup kernel");
    HIP_TRY(rebk::launch_wg_solve(a, h->panel_dtype, rebk::kWgThreads, rebk::wg_solve_lds_bytes(a), h->stream));
    return REBK_OK;
  }
  if (kernel == REBK_KERNEL_PIPE) {
    if (fixed) return fail(REBK_ERR_INVALID, "the pipelined kernel needs allocated memory; use GRID here");
    const int G = grid_wgs > 0 ? grid_wgs : h->cus;
    char why[256];
    if (!pipe_fits(h, a, G, why)) return fail(REBK_ERR_INVALID, "%s", why);
    rebk::GridSync gs{};
    gs.stride = ((h->max_nJ + h->max_nI + 1 + 31) / 32) * 32;
    int rc = ensure_pipe(h, nullptr);
    if (rc != REBK_OK) return rc;
    const size_t part_words = (size_t)4 * G * gs.stride * 2;
    const size_t gsum_words = (size_t)rebk::kGridSumRing * rebk::kGridSumCopies * gs.stride * 2;
    rc = ensure_grid_workspace(h, part_words, gsum_words);
    if (rc != REBK_OK) return rc;
    gs.part = h->part;
    gs.gsum = h->gsum;
    gs.timeout = h->timeout;
    HIP_TRY(hipMemsetAsync(h->part, 0, part_words * sizeof(unsigned long long), h->stream));
    HIP_TRY(hipMemsetAsync(h->gsum, 0, gsum_words * sizeof(unsigned long long), h->stream));
    HIP_TRY(hipMemsetAsync(h->timeout, 0, sizeof(int), h->stream));
    HIP_TRY(rebk::launch_pipe_solve(a, gs, h->pipe_G, h->pipe_H, h->pipe_Arm, h->panel_dtype, G, h->stream));
    return REBK_OK;
  }
  if (kernel != REBK_KERNEL_GRID) return fail(REBK_ERR_INVALID, "unknown kernel %d", kernel);
  int G = grid_wgs > 0 ? grid_wgs : h->cus;
  // row slabs staged in LDS when they fit, else read from the row panels in HBM
  bool row_lds = true;
  size_t lds = rebk::grid_solve_lds_bytes(a, G, h->panel_dtype, true);
  if (lds > 160 * 1024) {
    row_lds = false;
    lds = rebk::grid_solve_lds_bytes(a, G, h->panel_dtype, false);
  }
  if (lds > 160 * 1024) return fail(REBK_ERR_INVALID, "grid kernel needs %zu bytes of LDS per workgroup", lds);
  int per_cu = 0;
  HIP_TRY(rebk::grid_solve_max_blocks(h->panel_dtype, lds, row_lds, &per_cu));
  if (per_cu <= 0 || G > per_cu * h->cus)
    return fail(REBK_ERR_INVALID, "grid of %d workgroups cannot be co-resident (%d per CU)", G, per_cu);
  if ((h->n + G - 1) / G + 8 > rebk::kGridThreads)  // the most columns a workgroup owns
    return fail(REBK_ERR_INVALID, "too many columns per workgroup; use a larger grid");
  if (h->max_nJ > rebk::kGridThreads)
    return fail(REBK_ERR_INVALID, "column blocks wider than %d columns need the one-workgroup kernel", rebk::kGridThreads);
  rebk::GridSync gs{};
  if (G > 1024) return fail(REBK_ERR_INVALID, "at most 1024 workgroups in the grid kernel");
  gs.stride = ((h->max_nJ + h->max_nI + 1 + 31) / 32) * 32;
  const size_t part_words = (size_t)2 * G * gs.stride * 2;
  const size_t gsum_words = (size_t)rebk::kGridSumRing * rebk::kGridSumCopies * gs.stride * 2;
  if (fixed) {
    // part, gsum and the timeout flag (one 256-byte line) carved from the given words, then cleared
    const size_t need = part_words + gsum_words + 32;
    if (need > fixed->words)
      return fail(REBK_ERR_INVALID, "the grid kernel needs %zu workspace words here; the static workspace holds %zu",
                  need, fixed->words);
    gs.part = fixed->base;
    gs.gsum = fixed->base + part_words;
    gs.timeout = (int*)(fixed->base + part_words + gsum_words);
    HIP_TRY(rebk::launch_fill_zero(fixed->base, need, h->stream));
  } else {
    int rc = ensure_grid_workspace(h, part_words, gsum_words);
    if (rc != REBK_OK) return rc;
    gs.part = h->part;
    gs.gsum = h->gsum;
    gs.timeout = h->timeout;
    // epochs restart at 1 every launch: clear every tag of the previous launch
    HIP_TRY(hipMemsetAsync(h->part, 0, part_words * sizeof(unsigned long long), h->stream));
    HIP_TRY(hipMemsetAsync(h->gsum, 0, gsum_words * sizeof(unsigned long long), h->stream));
    HIP_TRY(hipMemsetAsync(h->timeout, 0, sizeof(int), h->stream));
  }
  HIP_TRY(rebk::launch_grid_solve(a, gs, h->panel_dtype, G, row_lds, h->stream));
  return REBK_OK;
}

}  // namespace

extern "C" {

const char* rebk_last_error(void) { return g_err; }

const char* rebk_version(void) { return "rebk-gfx950 0.1"; }

int rebk_create(rebk_handle_t* out, const void* A_dev, int32_t a_dtype, int32_t panel_dtype, int64_t m, int64_t n,
                int64_t lda, const int64_t* row_offsets, int64_t s, const int64_t* col_offsets, int64_t t,
                double alpha, uint64_t seed, void* stream) {
  g_err[0] = 0;
  if (!out) return fail(REBK_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!A_dev) return fail(REBK_ERR_INVALID, "A is NULL");
  if (a_dtype != REBK_F64 && a_dtype != REBK_F32) return fail(REBK_ERR_INVALID, "A must be FP64 or FP32");
  if (dtype_size(panel_dtype) == 0) return fail(REBK_ERR_INVALID, "unknown panel dtype %d", panel_dtype);
  if (m <= 0 || n <= 0 || lda < n) return fail(REBK_ERR_INVALID, "bad sizes m=%lld n=%lld lda=%lld", (long long)m, (long long)n, (long long)lda);
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(REBK_ERR_INVALID, "alpha must be positive and finite");
  int32_t max_nI = 0, max_nJ = 0;
  int rc = check_offsets(row_offsets, s, m, "row", &max_nI);
  if (rc != REBK_OK) return rc;
  rc = check_offsets(col_offsets, t, n, "column", &max_nJ);
  if (rc != REBK_OK) return rc;

  rebk_handle* h = new (std::nothrow) rebk_handle();
  if (!h) return fail(REBK_ERR_OOM, "host allocation failed");
  h->m = m;
  h->n = n;
  h->s = s;
  h->t = t;
  h->max_nI = max_nI;
  h->max_nJ = max_nJ;
  h->panel_dtype = panel_dtype;
  h->alpha = alpha;
  h->seed = seed;
  h->stream = (hipStream_t)stream;
  h->row_off.assign(row_offsets, row_offsets + s + 1);
  h->col_off.assign(col_offsets, col_offsets + t + 1);

  auto bail = [&](int code) {
    delete h;
    return code;
  };
#define TRY_H(expr)                                                                           \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return bail(fail(REBK_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_))); \
  } while (0)
#define ALLOC_H(ptr, bytes)                                                                    \
  do {                                                                                         \
    if (hipMalloc((void**)&(ptr), (bytes)) != hipSuccess)                                      \
      return bail(fail(REBK_ERR_OOM, "cannot allocate %zu bytes", (size_t)(bytes)));          \
  } while (0)

  TRY_H(hipGetDevice(&h->device));
  TRY_H(hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device));
  TRY_H(hipEventCreate(&h->ev0));
  TRY_H(hipEventCreate(&h->ev1));

  const size_t esz = dtype_size(panel_dtype);
  const size_t elems = (size_t)m * (size_t)n;
  h->ldc = rebk::col_stride(m);
  ALLOC_H(h->Arow, elems * esz);
  ALLOC_H(h->Acol, (size_t)h->ldc * (size_t)n * esz);
  ALLOC_H(h->row_off_d, (s + 1) * sizeof(int64_t));
  ALLOC_H(h->col_off_d, (t + 1) * sizeof(int64_t));
  ALLOC_H(h->T_row, s * sizeof(uint64_t));
  ALLOC_H(h->T_col, t * sizeof(uint64_t));
  ALLOC_H(h->coef_row, s * sizeof(double));
  ALLOC_H(h->coef_col, t * sizeof(double));
  ALLOC_H(h->status_d, sizeof(rebk::DevStatus));
  h->nparts = 512;
  ALLOC_H(h->partials, 2 * (size_t)h->nparts * sizeof(double));

  // scratch for packing and the weights
  std::vector<int32_t> rowblk(m), colblk(n);
  for (int64_t i = 0; i < s; ++i)
    for (int64_t r = row_offsets[i]; r < row_offsets[i + 1]; ++r) rowblk[r] = (int32_t)i;
  for (int64_t j = 0; j < t; ++j)
    for (int64_t c = col_offsets[j]; c < col_offsets[j + 1]; ++c) colblk[c] = (int32_t)j;
  int32_t *rowblk_d = nullptr, *colblk_d = nullptr;
  double *row_sq = nullptr, *colrow_sq = nullptr, *w_d = nullptr;
  int* bad_d = nullptr;
  auto free_scratch = [&]() {
    dfree(rowblk_d);
    dfree(colblk_d);
    dfree(row_sq);
    dfree(colrow_sq);
    dfree(w_d);
    dfree(bad_d);
  };
  auto bail2 = [&](int code) {
    free_scratch();
    return bail(code);
  };
#define TRY_S(expr)                                                                             \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return bail2(fail(REBK_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_))); \
  } while (0)
#define ALLOC_S(ptr, bytes)                                                                      \
  do {                                                                                           \
    if (hipMalloc((void**)&(ptr), (bytes)) != hipSuccess)                                        \
      return bail2(fail(REBK_ERR_OOM, "cannot allocate %zu bytes", (size_t)(bytes)));           \
  } while (0)

  ALLOC_S(rowblk_d, m * sizeof(int32_t));
  ALLOC_S(colblk_d, n * sizeof(int32_t));
  ALLOC_S(row_sq, m * sizeof(double));
  ALLOC_S(colrow_sq, (size_t)m * t * sizeof(double));
  ALLOC_S(w_d, (s + t) * sizeof(double));
  ALLOC_S(bad_d, sizeof(int));
  hipStream_t st = h->stream;
  TRY_S(hipMemcpyAsync(rowblk_d, rowblk.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, st));
  TRY_S(hipMemcpyAsync(colblk_d, colblk.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st));
  TRY_S(hipMemcpyAsync(h->row_off_d, h->row_off.data(), (s + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
  TRY_S(hipMemcpyAsync(h->col_off_d, h->col_off.data(), (t + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
  TRY_S(hipMemsetAsync(bad_d, 0, sizeof(int), st));
  TRY_S(rebk::launch_finite_check(A_dev, a_dtype, lda, m, n, bad_d, st));
  if (h->ldc > m) TRY_S(hipMemsetAsync(h->Acol, 0, (size_t)h->ldc * (size_t)n * esz, st));  // zero pad entries
  TRY_S(rebk::launch_pack(A_dev, a_dtype, lda, panel_dtype, m, n, h->ldc, h->row_off_d, h->col_off_d, rowblk_d,
                          colblk_d, h->Arow, h->Acol, st));
  TRY_S(rebk::launch_block_weights(h->Arow, h->Acol, panel_dtype, m, n, h->ldc, h->row_off_d, (int32_t)s, h->col_off_d,
                                   (int32_t)t, rowblk_d, row_sq, colrow_sq, w_d, w_d + s, st));
  std::vector<double> w(s + t);
  int bad = 0;
  TRY_S(hipMemcpyAsync(w.data(), w_d, (s + t) * sizeof(double), hipMemcpyDeviceToHost, st));
  TRY_S(hipMemcpyAsync(&bad, bad_d, sizeof(int), hipMemcpyDeviceToHost, st));
  TRY_S(hipStreamSynchronize(st));
  free_scratch();
  if (bad) return bail(fail(REBK_ERR_INVALID, "A has a non-finite entry"));
  h->w_row.assign(w.begin(), w.begin() + s);
  h->w_col.assign(w.begin() + s, w.end());
  if (!build_thresholds(h->w_row, h->T_row_h) || !build_thresholds(h->w_col, h->T_col_h))
    return bail(fail(REBK_ERR_INVALID, "||A||_F is zero or not finite"));
  h->fro2 = 0.0;
  for (double x : h->w_row) h->fro2 += x;
  std::vector<double> cr(s), cc(t);
  for (int64_t i = 0; i < s; ++i) cr[i] = h->w_row[i] > 0.0 ? alpha / h->w_row[i] : 0.0;
  for (int64_t j = 0; j < t; ++j) cc[j] = h->w_col[j] > 0.0 ? alpha / h->w_col[j] : 0.0;
  TRY_H(hipMemcpyAsync(h->T_row, h->T_row_h.data(), s * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  TRY_H(hipMemcpyAsync(h->T_col, h->T_col_h.data(), t * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  TRY_H(hipMemcpyAsync(h->coef_row, cr.data(), s * sizeof(double), hipMemcpyHostToDevice, st));
  TRY_H(hipMemcpyAsync(h->coef_col, cc.data(), t * sizeof(double), hipMemcpyHostToDevice, st));
  TRY_H(hipStreamSynchronize(st));
  *out = h;
  return REBK_OK;
#undef TRY_H
#undef ALLOC_H
#undef TRY_S
#undef ALLOC_S
}

void rebk_destroy(rebk_handle_t h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

int rebk_get_info(rebk_handle_t h, int64_t* m, int64_t* n, int64_t* s, int64_t* t, int64_t* max_row_block,
                  int64_t* max_col_block) {
  if (!h) return fail(REBK_ERR_INVALID, "handle is NULL");
  if (m) *m = h->m;
  if (n) *n = h->n;
  if (s) *s = h->s;
  if (t) *t = h->t;
  if (max_row_block) *max_row_block = h->max_nI;
  if (max_col_block) *max_col_block = h->max_nJ;
  return REBK_OK;
}

int rebk_get_weights(rebk_handle_t h, double* w_row, double* w_col) {
  if (!h) return fail(REBK_ERR_INVALID, "handle is NULL");
  if (w_row) std::memcpy(w_row, h->w_row.data(), h->s * sizeof(double));
  if (w_col) std::memcpy(w_col, h->w_col.data(), h->t * sizeof(double));
  return REBK_OK;
}

int rebk_get_thresholds(rebk_handle_t h, uint64_t* T_row, uint64_t* T_col) {
  if (!h) return fail(REBK_ERR_INVALID, "handle is NULL");
  if (T_row) std::memcpy(T_row, h->T_row_h.data(), h->s * sizeof(uint64_t));
  if (T_col) std::memcpy(T_col, h->T_col_h.data(), h->t * sizeof(uint64_t));
  return REBK_OK;
}

int rebk_sample_blocks(rebk_handle_t h, uint64_t system, int64_t k0, int64_t count, int32_t* j_out_dev,
                       int32_t* i_out_dev) {
  if (!h) return fail(REBK_ERR_INVALID, "handle is NULL");
  if (count < 0 || k0 < 0 || (count > 0 && (!j_out_dev || !i_out_dev)))
    return fail(REBK_ERR_INVALID, "bad sampler arguments");
  if (count == 0) return REBK_OK;
  HIP_TRY(rebk::launch_sample(h->T_row, (int32_t)h->s, h->T_col, (int32_t)h->t, h->seed, system, k0, count, j_out_dev,
                              i_out_dev, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return REBK_OK;
}

int rebk_philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1, int64_t count,
                       uint64_t* out_dev, void* stream) {
  if (count < 0 || (count > 0 && !out_dev)) return fail(REBK_ERR_INVALID, "bad Philox arguments");
  if (count == 0) return REBK_OK;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(rebk::launch_philox(c0, c1, c2, c3, k0, k1, count, out_dev, st));
  HIP_TRY(hipStreamSynchronize(st));
  return REBK_OK;
}

int rebk_solve_ex(rebk_handle_t h, const rebk_solve_opts_t* o, rebk_result_t* res) {
  g_err[0] = 0;
  if (!h) return fail(REBK_ERR_INVALID, "handle is NULL");
  if (!o) return fail(REBK_ERR_INVALID, "opts is NULL");
  if (!o->b_dev || !o->x_out_dev) return fail(REBK_ERR_INVALID, "b and x_out are required");
  if (o->max_iter <= 0) return fail(REBK_ERR_INVALID, "max_iter must be positive");
  if (o->k0 < 0) return fail(REBK_ERR_INVALID, "k0 must be non-negative");
  if (o->check_every < 0) return fail(REBK_ERR_INVALID, "check_every must be non-negative");
  if (!(o->tol == o->tol)) return fail(REBK_ERR_INVALID, "tol is NaN");
  if (o->kernel < REBK_KERNEL_AUTO || o->kernel > REBK_KERNEL_PIPE) return fail(REBK_ERR_INVALID, "unknown kernel");
  const bool ref_mode = o->x_ref_dev != nullptr;
  const bool residual_mode = !ref_mode && o->tol > 0.0;
  rebk::SolveArgs a = base_args(h);
  a.b = o->b_dev;
  a.x_in = o->x0_dev;
  a.z_in = o->z0_dev;
  a.x_out = o->x_out_dev;
  a.z_out = o->z_out_dev;
  a.x_ref = o->x_ref_dev;
  a.tol = o->tol;
  a.k0 = o->k0;
  a.trace_j = o->trace_j_dev;
  a.trace_i = o->trace_i_dev;
  if ((a.trace_j == nullptr) != (a.trace_i == nullptr)) return fail(REBK_ERR_INVALID, "give both trace buffers or none");

  if (ref_mode) {
    double xr2 = 0.0;
    // ||x_ref||^2, summed on the host from a copy
    std::vector<double> xr(h->n);
    HIP_TRY(hipMemcpyAsync(xr.data(), o->x_ref_dev, h->n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (double v : xr) xr2 += v * v;
    if (!(xr2 > 0.0) || !std::isfinite(xr2)) return fail(REBK_ERR_INVALID, "x_ref must be non-zero and finite");
    a.xref_sq = xr2;
  }

  if (o->kernel == REBK_KERNEL_PIPE) {  // the Gram matrices are built outside the timed region
    int rc = ensure_pipe(h, nullptr);
    if (rc != REBK_OK) return rc;
  }

  rebk_result_t r{};
  r.rel_err = -1.0;
  int used = 0;
  float ms_total = 0.0f;
  if (!residual_mode) {
    a.max_iter = o->max_iter;
    a.check_every = o->check_every > 0 ? o->check_every : 1;
    HIP_TRY(hipEventRecord(h->ev0, h->stream));
    int rc = run_iterations(h, a, o->kernel, o->grid_wgs, &used);
    if (rc != REBK_OK) return rc;
    HIP_TRY(hipEventRecord(h->ev1, h->stream));
    rebk::DevStatus ds{};
    HIP_TRY(hipMemcpyAsync(&ds, h->status_d, sizeof(ds), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipEventElapsedTime(&ms_total, h->ev0, h->ev1));
    if (ds.status == REBK_ERR_TIMEOUT) return fail(REBK_ERR_TIMEOUT, "grid barrier spin limit exceeded");
    r.status = ref_mode ? ds.status : REBK_OK;
    r.iterations = ds.last_k - o->k0;
    if (ref_mode && ds.err2 >= 0.0) r.rel_err = std::sqrt(ds.err2) / std::sqrt(a.xref_sq);
  } else {
    // residual stop rule: chunks of check_every iterations, norms of b - z - A x and A^T z between chunks
    const int64_t ce = o->check_every > 0 ? o->check_every : 256;
    const bool have_z_out = o->z_out_dev != nullptr;
    double* zbuf = o->z_out_dev;
    if (!have_z_out && hipMalloc((void**)&zbuf, h->m * sizeof(double)) != hipSuccess)
      return fail(REBK_ERR_OOM, "cannot allocate z");
    double bnorm2 = 0.0;
    {
      std::vector<double> bh(h->m);
      hipError_t e = hipMemcpyAsync(bh.data(), o->b_dev, h->m * sizeof(double), hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) {
        if (!have_z_out) (void)hipFree(zbuf);
        return fail(REBK_ERR_HIP, "copy of b: %s", hipGetErrorString(e));
      }
      for (double v : bh) bnorm2 += v * v;
    }
    const double bnorm = std::sqrt(bnorm2), anorm = std::sqrt(h->fro2);
    int64_t done = 0;
    int status = REBK_NOT_CONVERGED;
    int rc = REBK_OK;
    while (done < o->max_iter) {
      const int64_t chunk = (o->max_iter - done) < ce ? (o->max_iter - done) : ce;
      rebk::SolveArgs c = a;
      c.k0 = o->k0 + done;
      c.max_iter = chunk;
      c.check_every = chunk;
      c.x_in = done == 0 ? o->x0_dev : o->x_out_dev;
      c.z_in = done == 0 ? o->z0_dev : zbuf;
      c.z_out = zbuf;
      c.x_ref = nullptr;
      c.tol = 0.0;
      c.trace_j = o->trace_j_dev ? o->trace_j_dev + done : nullptr;
      c.trace_i = o->trace_i_dev ? o->trace_i_dev + done : nullptr;
      float ms = 0.0f;
      if (hipEventRecord(h->ev0, h->stream) != hipSuccess) { rc = fail(REBK_ERR_HIP, "event record failed"); break; }
      rc = run_iterations(h, c, o->kernel, o->grid_wgs, &used);
      if (rc != REBK_OK) break;
      if (hipEventRecord(h->ev1, h->stream) != hipSuccess) { rc = fail(REBK_ERR_HIP, "event record failed"); break; }
      done += chunk;
      hipError_t e = rebk::launch_residual(h->Arow, h->Acol, h->panel_dtype, c, o->x_out_dev, zbuf, h->partials,
                                           h->nparts, h->stream);
      if (e != hipSuccess) { rc = fail(REBK_ERR_HIP, "residual kernel: %s", hipGetErrorString(e)); break; }
      std::vector<double> parts(2 * h->nparts);
      e = hipMemcpyAsync(parts.data(), h->partials, parts.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, h->ev0, h->ev1);
      if (e != hipSuccess) { rc = fail(REBK_ERR_HIP, "residual readback: %s", hipGetErrorString(e)); break; }
      ms_total += ms;
      double f2 = 0.0, g2 = 0.0;
      for (int q = 0; q < h->nparts; ++q) f2 += parts[q];
      for (int q = 0; q < h->nparts; ++q) g2 += parts[h->nparts + q];
      const double rf = std::sqrt(f2) / (bnorm > 0 ? bnorm : 1.0);
      const double rg = std::sqrt(g2) / ((anorm * bnorm) > 0 ? anorm * bnorm : 1.0);
      r.rel_err = rf > rg ? rf : rg;
      if (!std::isfinite(f2) || !std::isfinite(g2) || r.rel_err > 1e6) { status = REBK_DIVERGED; break; }
      if (rf <= o->tol && rg <= o->tol) { status = REBK_OK; break; }
    }
    if (!have_z_out) (void)hipFree(zbuf);
    if (rc != REBK_OK) return rc;
    r.status = status;
    r.iterations = done;
  }
  r.kernel = used;
  r.time_ms = ms_total;
  if (res) *res = r;
  return r.status;
}

int rebk_solve_ex_static(rebk_handle_t h, const rebk_solve_opts_t* o, rebk_result_t* res) {
  g_err[0] = 0;
  if (!h) return fail(REBK_ERR_INVALID, "handle is NULL");
  if (!o) return fail(REBK_ERR_INVALID, "opts is NULL");
  if (!o->b_dev || !o->x_out_dev) return fail(REBK_ERR_INVALID, "b and x_out are required");
  if (o->max_iter <= 0) return fail(REBK_ERR_INVALID, "max_iter must be positive");
  if (o->k0 < 0) return fail(REBK_ERR_INVALID, "k0 must be non-negative");
  if (o->check_every < 0) return fail(REBK_ERR_INVALID, "check_every must be non-negative");
  if (!(o->tol == o->tol)) return fail(REBK_ERR_INVALID, "tol is NaN");
  if (o->kernel < REBK_KERNEL_AUTO || o->kernel > REBK_KERNEL_PIPE) return fail(REBK_ERR_INVALID, "unknown kernel");
  if (!o->x_ref_dev && o->tol > 0.0)
    return fail(REBK_ERR_INVALID, "the residual stop rule is not available without allocation; give x_ref or tol <= 0");
  if ((o->trace_j_dev == nullptr) != (o->trace_i_dev == nullptr))
    return fail(REBK_ERR_INVALID, "give both trace buffers or none");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != h->device) return fail(REBK_ERR_INVALID, "the handle's device (%d) is not the current device (%d)", h->device, dev);
  unsigned long long* ws = nullptr;
  HIP_TRY(rebk::static_scratch(dev, &ws));
  // the last 32 words hold ||x_ref||^2; the rest is the grid workspace
  const FixedWorkspace fixed{ws, rebk::kStaticScratchWords - 32};
  double* xr2_dev = (double*)(ws + rebk::kStaticScratchWords - 32);

  rebk::SolveArgs a = base_args(h);
  a.b = o->b_dev;
  a.x_in = o->x0_dev;
  a.z_in = o->z0_dev;
  a.x_out = o->x_out_dev;
  a.z_out = o->z_out_dev;
  a.x_ref = o->x_ref_dev;
  a.tol = o->tol;
  a.k0 = o->k0;
  a.trace_j = o->trace_j_dev;
  a.trace_i = o->trace_i_dev;
  a.max_iter = o->max_iter;
  a.check_every = o->check_every > 0 ? o->check_every : 1;
  if (a.x_ref) {
    double xr2 = 0.0;
    HIP_TRY(rebk::launch_sumsq_in_order(o->x_ref_dev, h->n, xr2_dev, h->stream));
    HIP_TRY(hipMemcpyAsync(&xr2, xr2_dev, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (!(xr2 > 0.0) || !std::isfinite(xr2)) return fail(REBK_ERR_INVALID, "x_ref must be non-zero and finite");
    a.xref_sq = xr2;
  }
  rebk_result_t r{};
  r.rel_err = -1.0;
  int used = 0;
  float ms = 0.0f;
  HIP_TRY(hipEventRecord(h->ev0, h->stream));
  int rc = run_iterations(h, a, o->kernel, o->grid_wgs, &used, &fixed);
  if (rc != REBK_OK) return rc;
  HIP_TRY(hipEventRecord(h->ev1, h->stream));
  rebk::DevStatus ds{};
  HIP_TRY(hipMemcpyAsync(&ds, h->status_d, sizeof(ds), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  if (ds.status == REBK_ERR_TIMEOUT) return fail(REBK_ERR_TIMEOUT, "grid barrier spin limit exceeded");
  r.status = a.x_ref ? ds.status : REBK_OK;
  r.iterations = ds.last_k - o->k0;
  if (a.x_ref && ds.err2 >= 0.0) r.rel_err = std::sqrt(ds.err2) / std::sqrt(a.xref_sq);
  r.kernel = used;
  r.time_ms = ms;
  if (res) *res = r;
  return r.status;
}

int rebk_pipe_prepare(rebk_handle_t h, double* build_ms) {
  g_err[0] = 0;
  if (build_ms) *build_ms = 0.0;
  if (!h) return fail(REBK_ERR_INVALID, "handle is NULL");
  return ensure_pipe(h, build_ms);
}

void rebk_pipe_release(rebk_handle_t h) {
  if (h) h->release_pipe();
}

int rebk_solve(rebk_handle_t h, const double* b_dev, const double* x0_dev, double* x_out_dev, double tol,
               int64_t max_iter, rebk_result_t* res) {
  rebk_solve_opts_t o{};
  o.b_dev = b_dev;
  o.x0_dev = x0_dev;
  o.max_iter = max_iter;
  o.tol = tol;
  o.x_out_dev = x_out_dev;
  o.kernel = REBK_KERNEL_AUTO;
  return rebk_solve_ex(h, &o, res);
}

}  // extern "C"

// ------------------------------------------------------------------ batched solves

struct rebk_batch {
  int32_t nsys = 0;
  int panel_dtype = 0;
  hipStream_t stream = nullptr;
  int cus = 0;
  int32_t max_nJ = 0, max_nI = 0;
  std::vector<rebk_handle*> hs;
  std::vector<int64_t> last_iters;  // per system, from the previous solve (longest-first order)
  std::vector<int> team_P;          // per system: workgroups per team tile of this solve (0: none)
  rebk::BatchSys* sys_d = nullptr;
  // choices of rebk_batch_autotune (0 / -1: not tuned)
  int32_t tuned_threads = 0, tuned_lds = 0, tuned_tile = 0, tuned_xcd = -1;
  // launch buffers, grown as needed
  rebk::BatchTask* tasks_d = nullptr;
  int64_t* iters_d = nullptr;
  int32_t* status_d = nullptr;
  double* err2_d = nullptr;
  double* xref2_d = nullptr;
  size_t tasks_cap = 0, iters_cap = 0, status_cap = 0, err2_cap = 0, xref2_cap = 0;
  // teams: their table, the team of every workgroup of the launch, the reduction words
  rebk::TeamTask* teams_d = nullptr;
  int32_t* team_of_wg_d = nullptr;
  unsigned long long* tsync_d = nullptr;
  size_t teams_cap = 0, twg_cap = 0, tsync_cap = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // the tile widths run as separate kernels at the same time: two more streams, forked from and
  // joined back into `stream` with events
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};

  ~rebk_batch() {
    dfree(sys_d);
    dfree(tasks_d);
    dfree(iters_d);
    dfree(status_d);
    dfree(err2_d);
    dfree(xref2_d);
    dfree(teams_d);
    dfree(team_of_wg_d);
    dfree(tsync_d);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (fork) (void)hipEventDestroy(fork);
    for (int q = 0; q < 2; ++q) {
      if (join[q]) (void)hipEventDestroy(join[q]);
      if (side[q]) (void)hipStreamDestroy(side[q]);
    }
  }
};

namespace {

constexpr int kLdsMax = 160 * 1024 - 1024;  // per workgroup, leaving room for static shared memory

struct BatchConfig {
  int threads, lds_budget, max_tile, xcd_order;
};

BatchConfig batch_config(const rebk_batch* b, const rebk_batch_opts_t* o) {
  BatchConfig c;
  c.threads = o->threads ? o->threads : (b->tuned_threads ? b->tuned_threads : 512);
  c.lds_budget = o->lds_budget ? o->lds_budget : (b->tuned_lds ? b->tuned_lds : kLdsMax);
  c.max_tile = o->max_tile ? o->max_tile : (b->tuned_tile ? b->tuned_tile : 4);
  c.xcd_order = o->xcd_order >= 0 ? o->xcd_order : (b->tuned_xcd >= 0 ? b->tuned_xcd : 1);
  return c;
}

template <typename T>
int grow(T*& p, size_t& cap, size_t need) {
  if (need <= cap) return REBK_OK;
  dfree(p);
  if (hipMalloc((void**)&p, need * sizeof(T)) != hipSuccess) return fail(REBK_ERR_OOM, "cannot allocate %zu bytes", need * sizeof(T));
  cap = need;
  return REBK_OK;
}

// Teams (rebk_batch_solve): sets b->team_P[s], the workgroups of each team tile of system s (0:
// ordinary tiles), and removes the team systems' cost from *total, the summed tile cost of the
// batch (in the units of batch_run: panel entries per iteration x iterations x (1 + R / 4)).
constexpr int kTeamMaxWgs = 256;
constexpr int kTeamLdsMax = 152 * 1024;  // dynamic LDS of a team workgroup (the kernel has ~6 KB static)
// A team pays off when a single compute unit's iteration (its panel stream at about 33 GB/s)
// takes at least twice a team's iteration (about 25 us: slab copies, four block products on the
// matrix cores and the two reduction hops).
constexpr double kCuBytesPerSec = 33e9;
constexpr double kTeamIterSec = 25e-6;

int plan_teams(rebk_batch* b, const rebk_batch_opts_t* o, const std::vector<int>& Rsys, double* total) {
  const int32_t ns = b->nsys;
  b->team_P.assign(ns, 0);
  if (o->team < 0) return REBK_OK;
  const int cus = b->cus > 0 ? b->cus : 1;
  auto min_P = [&](int32_t s) -> int {  // smallest team whose workgroups fit the LDS
    const rebk_handle* h = b->hs[s];
    for (int P = 2; P <= kTeamMaxWgs; ++P)
      if (rebk::team_lds_bytes(h->m, h->n, P, b->max_nJ, b->max_nI, b->panel_dtype) <= (size_t)kTeamLdsMax) return P;
    return 0;
  };
  auto team_tiles = [&](int32_t s) { return (o->nrhs[s] + rebk::kTeamR - 1) / rebk::kTeamR; };
  if (o->team > 0) {
    if (o->team > kTeamMaxWgs) return fail(REBK_ERR_INVALID, "team must be at most %d workgroups", kTeamMaxWgs);
    if (o->z0_from_x0) return fail(REBK_ERR_INVALID, "teams do not take z0_from_x0");
    for (int32_t s = 0; s < ns; ++s) {
      const int pm = min_P(s);
      if (pm == 0 || pm > o->team)
        return fail(REBK_ERR_INVALID, "system %d needs teams of %s %d workgroups", s, pm ? "at least" : "more than",
                    pm ? pm : kTeamMaxWgs);
      b->team_P[s] = o->team;
    }
    *total = 0.0;
    return REBK_OK;
  }
  if (o->z0_from_x0) return REBK_OK;
  const double esz = b->panel_dtype == 0 ? 8.0 : (b->panel_dtype == 1 ? 4.0 : 2.0);
  std::vector<double> load(ns), single(ns), work(ns), per_iter(ns);
  for (int32_t s = 0; s < ns; ++s) {
    const rebk_handle* h = b->hs[s];
    per_iter[s] = (double)h->m * h->max_nJ + (double)h->max_nI * h->n;
    const double iters = b->last_iters[s] > 0 ? (double)b->last_iters[s] : 1.0;
    load[s] = per_iter[s] * iters * (1.0 + 0.25 * Rsys[s]) * ((o->nrhs[s] + Rsys[s] - 1) / Rsys[s]);
    single[s] = per_iter[s] * iters * 1.25;
    work[s] = per_iter[s] * iters * team_tiles(s);
  }
  std::vector<int32_t> by(ns);
  for (int32_t s = 0; s < ns; ++s) by[s] = s;
  std::stable_sort(by.begin(), by.end(), [&](int32_t p, int32_t q) { return single[p] > single[q]; });
  // heaviest first: a system becomes a team while its single tile outlasts the average load of a
  // compute unit over the other ordinary tiles
  double rest = *total;
  std::vector<int32_t> chosen;
  std::vector<int> pmin(ns, 0);
  for (int32_t s : by) {
    if (b->last_iters[s] <= 0) continue;
    if (single[s] <= (rest - load[s]) / cus) break;
    if (2.0 * per_iter[s] * esz / kCuBytesPerSec < 2.0 * kTeamIterSec) continue;
    pmin[s] = min_P(s);
    if (pmin[s] == 0) continue;
    chosen.push_back(s);
    rest -= load[s];
    if ((int)chosen.size() >= cus / 8) break;
  }
  // workgroups in proportion to the work, at least the LDS minimum each, all compute units in
  // total; the lightest teams go back to ordinary tiles while the minimum sizes do not fit
  while (!chosen.empty()) {
    int need = 0;
    double W = 0.0;
    for (int32_t s : chosen) {
      need += pmin[s] * team_tiles(s);
      W += work[s];
    }
    if (need > cus) {
      rest += load[chosen.back()];
      chosen.pop_back();
      continue;
    }
    int used = 0;
    for (int32_t s : chosen) {
      int P = (int)((double)cus * work[s] / W / team_tiles(s));
      P = P < pmin[s] ? pmin[s] : (P > kTeamMaxWgs ? kTeamMaxWgs : P);
      b->team_P[s] = P;
      used += P * team_tiles(s);
    }
    while (used > cus) {  // trim the largest teams
      int32_t big = -1;
      for (int32_t s : chosen)
        if (b->team_P[s] > pmin[s] && (big < 0 || b->team_P[s] > b->team_P[big])) big = s;
      if (big < 0) break;
      --b->team_P[big];
      used -= team_tiles(big);
    }
    break;
  }
  *total = rest;
  return REBK_OK;
}

// Run the batch once with configuration c.  Fills out (may be NULL) and *ms.
int batch_run(rebk_batch* b, const rebk_batch_opts_t* o, const BatchConfig& c, rebk_batch_rhs_t* out, double* ms,
              int* overall) {
  if (c.threads != 256 && c.threads != 512 && c.threads != 1024)
    return fail(REBK_ERR_INVALID, "threads must be 256, 512 or 1024");
  if (c.max_tile != 1 && c.max_tile != 2 && c.max_tile != 4) return fail(REBK_ERR_INVALID, "max_tile must be 1, 2 or 4");
  if (c.lds_budget <= 0 || c.lds_budget > kLdsMax) return fail(REBK_ERR_INVALID, "lds_budget out of range");
  const int32_t ns = b->nsys;
  // tiles: per system the widest tile that fits the LDS budget (narrower for the longest systems,
  // below), remainder in smaller tiles
  struct Tile {
    int32_t sys, rhs0, R;
    int64_t rhs_index;  // global index of the tile's first right-hand side
    double cost;
    int32_t P;          // workgroups of its team (0: one workgroup)
  };
  std::vector<Tile> tiles;
  std::vector<int64_t> rhs_base(ns + 1, 0);
  for (int32_t s = 0; s < ns; ++s) rhs_base[s + 1] = rhs_base[s] + o->nrhs[s];
  // A tile of width R costs about (panel entries per iteration) x (iterations of the previous
  // solve) x (1 + R / 4): the panel stream is shared by the R right-hand sides, the LDS traffic and
  // arithmetic grow with R.  Wide tiles cost less in total, but a system whose single tile would
  // run longer than the average load of a compute unit sets the time of the whole batch: such a
  // system gets narrower tiles (more of them run at once).
  std::vector<int> Rsys(ns, 0);
  double total = 0.0;
  for (int32_t s = 0; s < ns; ++s) {
    const rebk_handle* h = b->hs[s];
    for (int R = c.max_tile; R >= 1; R >>= 1)
      if (rebk::batch_lds_bytes(h->m, h->n, R, b->max_nJ, b->max_nI, c.threads) <= (size_t)c.lds_budget) {
        Rsys[s] = R;
        break;
      }
    if (Rsys[s] == 0)
      return fail(REBK_ERR_INVALID, "system %d (%lld x %lld) does not fit %d bytes of LDS", s, (long long)h->m,
                  (long long)h->n, c.lds_budget);
    const double per_iter = (double)h->m * h->max_nJ + (double)h->max_nI * h->n;
    const double iters = b->last_iters[s] > 0 ? (double)b->last_iters[s] : 1.0;
    total += per_iter * iters * (1.0 + 0.25 * Rsys[s]) * ((o->nrhs[s] + Rsys[s] - 1) / Rsys[s]);
  }
  int rc = plan_teams(b, o, Rsys, &total);
  if (rc != REBK_OK) return rc;
  const double per_cu_load = total / (b->cus > 0 ? b->cus : 1);
  for (int32_t s = 0; s < ns; ++s) {
    if (b->team_P[s] > 0) continue;
    if (b->last_iters[s] <= 0) continue;  // no previous solve: nothing to go by
    const rebk_handle* h = b->hs[s];
    const double per_iter = (double)h->m * h->max_nJ + (double)h->max_nI * h->n;
    const double iters = (double)b->last_iters[s];
    while (Rsys[s] > 1 && per_iter * iters * (1.0 + 0.25 * Rsys[s]) > per_cu_load) Rsys[s] >>= 1;
  }
  for (int32_t s = 0; s < ns; ++s) {
    const rebk_handle* h = b->hs[s];
    const int Rfit = Rsys[s];
    const double per_iter = (double)h->m * h->max_nJ + (double)h->max_nI * h->n;
    const double iters = b->last_iters[s] > 0 ? (double)b->last_iters[s] : 1.0;
    int32_t done = 0;
    while (done < o->nrhs[s]) {
      if (b->team_P[s] > 0) {  // team tiles of up to kTeamR right-hand sides
        const int R = o->nrhs[s] - done < rebk::kTeamR ? o->nrhs[s] - done : rebk::kTeamR;
        tiles.push_back({s, done, R, rhs_base[s] + done, per_iter * iters, b->team_P[s]});
        done += R;
        continue;
      }
      int R = Rfit;
      while (R > o->nrhs[s] - done) R >>= 1;
      tiles.push_back({s, done, R, rhs_base[s] + done, per_iter * iters * (1.0 + 0.25 * R), 0});
      done += R;
    }
  }
  // Order, per tile width (each width is its own kernel): longest first; with xcd_order, the tiles
  // of a system are cut into groups of at most one XCD's worth of compute units (so a system with
  // many right-hand sides still spreads over the chip), groups go to the least loaded of the 8
  // XCDs, and workgroup 8*slot + x of the launch runs slot `slot` of XCD x.
  auto make_order = [&](const std::vector<int32_t>& idx) -> std::vector<int32_t> {
    std::vector<int32_t> ord;  // tile index per workgroup, -1 for an empty slot
    if (c.xcd_order) {
      const size_t per_xcd = (size_t)(b->cus >= 8 ? b->cus / 8 : 1);
      std::vector<std::vector<int32_t>> by_sys(ns);
      for (int32_t q : idx) by_sys[tiles[q].sys].push_back(q);
      std::vector<std::vector<int32_t>> groups;
      std::vector<double> gcost;
      for (int32_t s_ = 0; s_ < ns; ++s_)
        for (size_t q0 = 0; q0 < by_sys[s_].size(); q0 += per_xcd) {
          groups.emplace_back();
          double cst = 0.0;
          for (size_t q = q0; q < by_sys[s_].size() && q < q0 + per_xcd; ++q) {
            groups.back().push_back(by_sys[s_][q]);
            cst += tiles[by_sys[s_][q]].cost;
          }
          gcost.push_back(cst);
        }
      std::vector<int32_t> gidx(groups.size());
      for (size_t g = 0; g < gidx.size(); ++g) gidx[g] = (int32_t)g;
      std::stable_sort(gidx.begin(), gidx.end(), [&](int32_t p, int32_t q) { return gcost[p] > gcost[q]; });
      std::vector<std::vector<int32_t>> lists(8);
      std::vector<double> load(8, 0.0);
      for (int32_t g : gidx) {
        int best = 0;
        for (int x = 1; x < 8; ++x)
          if (load[x] < load[best]) best = x;
        for (int32_t q : groups[g]) lists[best].push_back(q);
        load[best] += gcost[g];
      }
      size_t slots = 0;
      for (auto& l : lists) slots = l.size() > slots ? l.size() : slots;
      ord.assign(slots * 8, -1);
      for (int x = 0; x < 8; ++x)
        for (size_t q = 0; q < lists[x].size(); ++q) ord[q * 8 + x] = lists[x][q];
    } else {
      ord = idx;
      std::stable_sort(ord.begin(), ord.end(), [&](int32_t p, int32_t q) { return tiles[p].cost > tiles[q].cost; });
    }
    return ord;
  };
  static constexpr int kWidths[3] = {4, 2, 1};
  std::vector<int32_t> order;
  size_t seg_off[3] = {0, 0, 0}, seg_len[3] = {0, 0, 0}, seg_lds[3] = {0, 0, 0};
  for (int wi = 0; wi < 3; ++wi) {
    std::vector<int32_t> idx;
    for (size_t q = 0; q < tiles.size(); ++q)
      if (tiles[q].P == 0 && tiles[q].R == kWidths[wi]) {
        idx.push_back((int32_t)q);
        const rebk_handle* h = b->hs[tiles[q].sys];
        const size_t lds = rebk::batch_lds_bytes(h->m, h->n, kWidths[wi], b->max_nJ, b->max_nI, c.threads);
        if (lds > seg_lds[wi]) seg_lds[wi] = lds;
      }
    const std::vector<int32_t> ord = make_order(idx);
    seg_off[wi] = order.size();
    seg_len[wi] = ord.size();
    order.insert(order.end(), ord.begin(), ord.end());
  }
  // the team tiles, after the others
  const size_t team_off = order.size();
  for (size_t q = 0; q < tiles.size(); ++q)
    if (tiles[q].P > 0) order.push_back((int32_t)q);
  const size_t nteam = order.size() - team_off;
  const size_t ntask = order.size();
  if (ntask > (size_t)INT32_MAX) return fail(REBK_ERR_INVALID, "too many tasks");
  const size_t nrhs_total = (size_t)rhs_base[ns];
  rc = grow(b->tasks_d, b->tasks_cap, ntask);
  if (rc == REBK_OK) rc = grow(b->iters_d, b->iters_cap, ntask);
  if (rc == REBK_OK) rc = grow(b->status_d, b->status_cap, ntask);
  if (rc == REBK_OK) rc = grow(b->err2_d, b->err2_cap, nrhs_total);
  if (rc == REBK_OK) rc = grow(b->xref2_d, b->xref2_cap, nrhs_total);
  if (rc != REBK_OK) return rc;
  std::vector<rebk::BatchTask> tasks(ntask);
  for (size_t w = 0; w < ntask; ++w) {
    rebk::BatchTask& t = tasks[w];
    t = rebk::BatchTask{};
    t.sys = -1;
    if (order[w] < 0) continue;
    const Tile& tl = tiles[order[w]];
    const rebk_handle* h = b->hs[tl.sys];
    t.sys = tl.sys;
    t.R = tl.R;
    t.b = o->b_dev[tl.sys] + (int64_t)tl.rhs0 * h->m;
    t.x_in = (o->x0_dev && o->x0_dev[tl.sys]) ? o->x0_dev[tl.sys] + (int64_t)tl.rhs0 * h->n : nullptr;
    t.x_ref = o->x_ref_dev ? o->x_ref_dev[tl.sys] + (int64_t)tl.rhs0 * h->n : nullptr;
    t.x_out = o->x_out_dev[tl.sys] + (int64_t)tl.rhs0 * h->n;
    t.z_out = o->z_out_dev ? o->z_out_dev[tl.sys] + (int64_t)tl.rhs0 * h->m : nullptr;
    t.iters_out = b->iters_d + w;
    t.status_out = b->status_d + w;
    t.err2_out = b->err2_d + tl.rhs_index;
    t.xref2_out = b->xref2_d + tl.rhs_index;
  }
  rebk::BatchArgs a{};
  a.sys = b->sys_d;
  a.tasks = b->tasks_d;
  a.max_nJ = b->max_nJ;
  a.max_nI = b->max_nI;
  a.max_iter = o->max_iter;
  a.tol = o->tol;
  a.check_every = o->check_every > 0 ? o->check_every : 16;
  a.z0_from_x0 = o->z0_from_x0 ? 1 : 0;
  for (int wi = 0; wi < 3; ++wi) {
    if (seg_len[wi] == 0) continue;
    int per_cu = 0;
    HIP_TRY(rebk::batch_max_blocks(b->panel_dtype, c.threads, kWidths[wi], seg_lds[wi], &per_cu));
    if (per_cu <= 0)
      return fail(REBK_ERR_INVALID, "batch kernel cannot run with %zu bytes of LDS and %d threads", seg_lds[wi],
                  c.threads);
  }
  // teams: workgroups [wg0, wg0 + P) of one cooperative launch per team tile; each team's
  // reduction words (2 P partial vectors and 2 reduced vectors of E tagged pairs) in one zeroed
  // buffer that ends with the timeout flag
  const int32_t E = rebk::kTeamR * (b->max_nJ + b->max_nI + 1);
  std::vector<rebk::TeamTask> teams(nteam);
  std::vector<int32_t> team_of_wg;
  size_t team_lds = 0, tsync_words = 0;
  for (size_t q = 0; q < nteam; ++q) {
    const Tile& tl = tiles[order[team_off + q]];
    const rebk_handle* h = b->hs[tl.sys];
    const size_t lds = rebk::team_lds_bytes(h->m, h->n, tl.P, b->max_nJ, b->max_nI, b->panel_dtype);
    if (lds > team_lds) team_lds = lds;
    teams[q].task = (int32_t)(team_off + q);
    teams[q].P = tl.P;
    teams[q].wg0 = (int32_t)team_of_wg.size();
    teams[q].E = E;
    team_of_wg.insert(team_of_wg.end(), (size_t)tl.P, (int32_t)q);
    tsync_words += (2 * (size_t)tl.P + 2) * E * 2;
  }
  if (nteam > 0) {
    int per_cu = 0;
    HIP_TRY(rebk::team_max_blocks(b->panel_dtype, team_lds, &per_cu));
    if (per_cu <= 0 || team_of_wg.size() > (size_t)per_cu * (size_t)(b->cus > 0 ? b->cus : 1))
      return fail(REBK_ERR_INVALID, "teams need %zu workgroups at once; the device holds %d with %zu bytes of LDS",
                  team_of_wg.size(), per_cu * b->cus, team_lds);
    rc = grow(b->teams_d, b->teams_cap, nteam);
    if (rc == REBK_OK) rc = grow(b->team_of_wg_d, b->twg_cap, team_of_wg.size());
    if (rc == REBK_OK) rc = grow(b->tsync_d, b->tsync_cap, tsync_words + 1);
    if (rc != REBK_OK) return rc;
    size_t off = 0;
    for (size_t q = 0; q < nteam; ++q) {
      teams[q].part = b->tsync_d + off;
      off += 2 * (size_t)teams[q].P * E * 2;
      teams[q].sum = b->tsync_d + off;
      off += 2 * (size_t)E * 2;
    }
  }
  hipStream_t st = b->stream;
  HIP_TRY(hipMemcpyAsync(b->tasks_d, tasks.data(), ntask * sizeof(rebk::BatchTask), hipMemcpyHostToDevice, st));
  if (nteam > 0) {
    HIP_TRY(hipMemcpyAsync(b->teams_d, teams.data(), nteam * sizeof(rebk::TeamTask), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(b->team_of_wg_d, team_of_wg.data(), team_of_wg.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(b->tsync_d, 0, (tsync_words + 1) * sizeof(unsigned long long), st));
  }
  HIP_TRY(hipEventRecord(b->ev0, st));
  if (nteam > 0) {  // the teams first, on the batch's stream; the other tiles start after them
    rebk::TeamArgs ta{};
    ta.teams = b->teams_d;
    ta.team_of_wg = b->team_of_wg_d;
    ta.timeout = (int*)(b->tsync_d + tsync_words);
    HIP_TRY(rebk::launch_team_solve(a, ta, (int)team_of_wg.size(), b->panel_dtype, team_lds, st));
  }
  // the first non-empty width runs on the caller's stream, the others on the side streams, all at
  // the same time; the caller's stream then waits for them.  The fork is recorded before the
  // first width is queued (after the teams), so the side streams do not wait for that kernel.
  int nside = 0;
  bool first = true;
  HIP_TRY(hipEventRecord(b->fork, st));
  for (int wi = 0; wi < 3; ++wi) {
    if (seg_len[wi] == 0) continue;
    hipStream_t ls = st;
    if (!first) {
      ls = b->side[nside];
      HIP_TRY(hipStreamWaitEvent(ls, b->fork, 0));
    }
    rebk::BatchArgs aw = a;
    aw.tasks = b->tasks_d + seg_off[wi];
    aw.ntasks = (int32_t)seg_len[wi];
    HIP_TRY(rebk::launch_batch_solve(aw, b->panel_dtype, c.threads, kWidths[wi], seg_lds[wi], ls));
    if (!first) {
      HIP_TRY(hipEventRecord(b->join[nside], ls));
      ++nside;
    }
    first = false;
  }
  for (int q = 0; q < nside; ++q) HIP_TRY(hipStreamWaitEvent(st, b->join[q], 0));
  HIP_TRY(hipEventRecord(b->ev1, st));
  std::vector<int64_t> it(ntask);
  std::vector<int32_t> stt(ntask);
  std::vector<double> e2(nrhs_total), x2(nrhs_total);
  HIP_TRY(hipMemcpyAsync(it.data(), b->iters_d, ntask * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(stt.data(), b->status_d, ntask * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(e2.data(), b->err2_d, nrhs_total * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(x2.data(), b->xref2_d, nrhs_total * sizeof(double), hipMemcpyDeviceToHost, st));
  int timed_out = 0;
  if (nteam > 0)
    HIP_TRY(hipMemcpyAsync(&timed_out, b->tsync_d + tsync_words, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (timed_out) return fail(REBK_ERR_TIMEOUT, "a team reduction exceeded its spin limit");
  float fms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&fms, b->ev0, b->ev1));
  if (ms) *ms = fms;
  int worst = REBK_OK;
  std::vector<int64_t> sys_iters(ns, 0);
  for (size_t w = 0; w < ntask; ++w) {
    if (order[w] < 0) continue;
    const Tile& tl = tiles[order[w]];
    if (it[w] > sys_iters[tl.sys]) sys_iters[tl.sys] = it[w];
    const int s_ = stt[w];
    if (s_ == REBK_DIVERGED) worst = REBK_DIVERGED;
    else if (s_ == REBK_NOT_CONVERGED && worst == REBK_OK) worst = REBK_NOT_CONVERGED;
    if (out) {
      for (int k = 0; k < tl.R; ++k) {
        rebk_batch_rhs_t& r = out[tl.rhs_index + k];
        r.iterations = it[w];
        r.status = s_;
        r.tile = tl.R;
        r.team = tl.P;
        const double ee = e2[tl.rhs_index + k], xx = x2[tl.rhs_index + k];
        r.rel_err = (o->x_ref_dev && ee >= 0.0 && xx > 0.0) ? std::sqrt(ee) / std::sqrt(xx) : -1.0;
      }
    }
  }
  b->last_iters = sys_iters;
  *overall = worst;
  return REBK_OK;
}

int check_batch_opts(const rebk_batch* b, const rebk_batch_opts_t* o) {
  if (!o) return fail(REBK_ERR_INVALID, "opts is NULL");
  if (!o->nrhs || !o->b_dev || !o->x_out_dev) return fail(REBK_ERR_INVALID, "nrhs, b and x_out are required");
  if (o->max_iter <= 0) return fail(REBK_ERR_INVALID, "max_iter must be positive");
  if (o->check_every < 0) return fail(REBK_ERR_INVALID, "check_every must be non-negative");
  if (!(o->tol == o->tol)) return fail(REBK_ERR_INVALID, "tol is NaN");
  if (o->tol > 0.0 && !o->x_ref_dev) return fail(REBK_ERR_INVALID, "a tolerance needs x_ref");
  for (int32_t s = 0; s < b->nsys; ++s) {
    if (o->nrhs[s] < 1 || o->nrhs[s] > (1 << 20)) return fail(REBK_ERR_INVALID, "nrhs[%d] must be in 1..2^20", s);
    if (!o->b_dev[s] || !o->x_out_dev[s]) return fail(REBK_ERR_INVALID, "b and x_out of system %d are NULL", s);
    if (o->x_ref_dev && !o->x_ref_dev[s]) return fail(REBK_ERR_INVALID, "x_ref of system %d is NULL", s);
    if (o->z_out_dev && !o->z_out_dev[s]) return fail(REBK_ERR_INVALID, "z_out of system %d is NULL", s);
  }
  return REBK_OK;
}

}  // namespace

extern "C" {

int rebk_batch_create(rebk_batch_t* out, int32_t nsys, const rebk_handle_t* systems, const uint64_t* sys_ids,
                      void* stream) {
  g_err[0] = 0;
  if (!out) return fail(REBK_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (nsys < 1 || !systems) return fail(REBK_ERR_INVALID, "need at least one system");
  for (int32_t s = 0; s < nsys; ++s) {
    if (!systems[s]) return fail(REBK_ERR_INVALID, "system %d is NULL", s);
    if (systems[s]->panel_dtype != systems[0]->panel_dtype) return fail(REBK_ERR_INVALID, "mixed panel types");
    if (systems[s]->device != systems[0]->device) return fail(REBK_ERR_INVALID, "systems on different devices");
  }
  rebk_batch* b = new (std::nothrow) rebk_batch();
  if (!b) return fail(REBK_ERR_OOM, "host allocation failed");
  b->nsys = nsys;
  b->panel_dtype = systems[0]->panel_dtype;
  b->stream = (hipStream_t)stream;
  b->cus = systems[0]->cus;
  b->hs.assign(systems, systems + nsys);
  b->last_iters.assign(nsys, 0);
  b->team_P.assign(nsys, 0);
  std::vector<rebk::BatchSys> S(nsys);
  for (int32_t s = 0; s < nsys; ++s) {
    const rebk_handle* h = systems[s];
    rebk::BatchSys& d = S[s];
    d.Arow = h->Arow;
    d.Acol = h->Acol;
    d.row_off = h->row_off_d;
    d.col_off = h->col_off_d;
    d.T_row = h->T_row;
    d.T_col = h->T_col;
    d.coef_row = h->coef_row;
    d.coef_col = h->coef_col;
    d.m = h->m;
    d.n = h->n;
    d.ldc = h->ldc;
    d.s = (int32_t)h->s;
    d.t = (int32_t)h->t;
    d.max_nI = h->max_nI;
    d.max_nJ = h->max_nJ;
    d.seed = h->seed;
    d.sys = sys_ids ? sys_ids[s] : (uint64_t)s;
    if (h->max_nJ > b->max_nJ) b->max_nJ = h->max_nJ;
    if (h->max_nI > b->max_nI) b->max_nI = h->max_nI;
  }
  auto bail = [&](int code) {
    delete b;
    return code;
  };
  if (hipMalloc((void**)&b->sys_d, nsys * sizeof(rebk::BatchSys)) != hipSuccess)
    return bail(fail(REBK_ERR_OOM, "cannot allocate the system table"));
  hipError_t e = hipMemcpyAsync(b->sys_d, S.data(), nsys * sizeof(rebk::BatchSys), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) e = hipEventCreate(&b->ev0);
  if (e == hipSuccess) e = hipEventCreate(&b->ev1);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int q = 0; q < 2 && e == hipSuccess; ++q) {
    e = hipEventCreateWithFlags(&b->join[q], hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side[q], hipStreamNonBlocking);
  }
  if (e != hipSuccess) return bail(fail(REBK_ERR_HIP, "batch setup: %s", hipGetErrorString(e)));
  *out = b;
  return REBK_OK;
}

void rebk_batch_destroy(rebk_batch_t b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  delete b;
}

int rebk_batch_solve(rebk_batch_t b, const rebk_batch_opts_t* o, rebk_batch_rhs_t* out, double* time_ms) {
  g_err[0] = 0;
  if (!b) return fail(REBK_ERR_INVALID, "batch is NULL");
  int rc = check_batch_opts(b, o);
  if (rc != REBK_OK) return rc;
  double ms = 0.0;
  int overall = REBK_OK;
  rc = batch_run(b, o, batch_config(b, o), out, &ms, &overall);
  if (rc != REBK_OK) return rc;
  if (time_ms) *time_ms = ms;
  return overall;
}

int rebk_batch_autotune(rebk_batch_t b, const rebk_batch_opts_t* o, int64_t probe_iters, int32_t* threads,
                        int32_t* lds_budget, int32_t* max_tile, int32_t* xcd_order, double* best_ms) {
  g_err[0] = 0;
  if (!b) return fail(REBK_ERR_INVALID, "batch is NULL");
  int rc = check_batch_opts(b, o);
  if (rc != REBK_OK) return rc;
  if (probe_iters <= 0) return fail(REBK_ERR_INVALID, "probe_iters must be positive");
  rebk_batch_opts_t p = *o;
  p.max_iter = probe_iters;
  p.tol = 0.0;
  const int cand_threads[] = {256, 512, 1024};
  const int cand_tile[] = {1, 2, 4};
  const int cand_lds[] = {kLdsMax, 80 * 1024 - 512};
  BatchConfig best{0, 0, 0, 1};
  double best_t = 1e300;
  for (int xo = 1; xo >= 0; --xo)
    for (int th : cand_threads)
      for (int tl : cand_tile)
        for (int ld : cand_lds) {
          BatchConfig c{th, ld, tl, xo};
          double ms = 0.0;
          int overall = 0;
          const std::vector<int64_t> keep = b->last_iters;
          int r = batch_run(b, &p, c, nullptr, &ms, &overall);
          b->last_iters = keep;
          if (r == REBK_ERR_INVALID) continue;  // this candidate does not fit
          if (r != REBK_OK) return r;
          if (ms < best_t) {
            best_t = ms;
            best = c;
          }
        }
  if (best.threads == 0) return fail(REBK_ERR_INVALID, "no configuration fits the batch");
  g_err[0] = 0;
  b->tuned_threads = best.threads;
  b->tuned_lds = best.lds_budget;
  b->tuned_tile = best.max_tile;
  b->tuned_xcd = best.xcd_order;
  if (threads) *threads = best.threads;
  if (lds_budget) *lds_budget = best.lds_budget;
  if (max_tile) *max_tile = best.max_tile;
  if (xcd_order) *xcd_order = best.xcd_order;
  if (best_ms) *best_ms = best_t;
  return REBK_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ FP64 refinement around REBK

namespace {

struct DevBuffers {  // device scratch of one call, freed on every return path
  std::vector<void*> ptrs;
  ~DevBuffers() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  double* get(size_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, (count > 0 ? count : 1) * sizeof(double)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return (double*)p;
  }
};

// sum of squares of v (len entries) on the device, partial sums added on the host in order
int dev_sumsq(rebk_handle* h, const double* v, int64_t len, double* out) {
  HIP_TRY(rebk::launch_sumsq(v, len, h->partials, h->nparts, h->stream));
  return host_sum(h, h->partials, h->nparts, out);
}

}  // namespace

extern "C" int rebk_solve_refined(rebk_handle_t h, const rebk_refine_opts_t* o, rebk_result_t* res) {
  g_err[0] = 0;
  if (!h) return fail(REBK_ERR_INVALID, "handle is NULL");
  if (!o) return fail(REBK_ERR_INVALID, "opts is NULL");
  if (!o->A_dev || !o->b_dev || !o->x_out_dev) return fail(REBK_ERR_INVALID, "A, b and x_out are required");
  if (o->lda < h->n) return fail(REBK_ERR_INVALID, "lda must be at least n");
  if (o->inner_iters <= 0) return fail(REBK_ERR_INVALID, "inner_iters must be positive");
  if (o->max_outer < 0) return fail(REBK_ERR_INVALID, "max_outer must be non-negative");
  if (!(o->tol == o->tol)) return fail(REBK_ERR_INVALID, "tol is NaN");
  if (o->kernel < REBK_KERNEL_AUTO || o->kernel > REBK_KERNEL_PIPE) return fail(REBK_ERR_INVALID, "unknown kernel");
  const int64_t m = h->m, n = h->n;
  hipStream_t st = h->stream;
  DevBuffers buf;
  double* f = buf.get(m);
  double* g = buf.get(n);
  double* dz = buf.get(m);
  double* dx = buf.get(n);
  double* dy = buf.get(m);
  double* partial = buf.get((size_t)rebk::refine_chunks(m) * n);
  double* z = o->z_out_dev ? o->z_out_dev : buf.get(m);
  if (!f || !g || !dz || !dx || !dy || !partial || !z) return fail(REBK_ERR_OOM, "cannot allocate refinement scratch");
  double* x = o->x_out_dev;

  double b2 = 0.0, a2 = 0.0, xr2 = 0.0;
  int rc = dev_sumsq(h, o->b_dev, m, &b2);
  if (rc != REBK_OK) return rc;
  HIP_TRY(rebk::launch_sumsq_matrix(o->A_dev, o->lda, m, n, h->partials, h->nparts, st));
  rc = host_sum(h, h->partials, h->nparts, &a2);
  if (rc != REBK_OK) return rc;
  if (o->x_ref_dev) {
    rc = dev_sumsq(h, o->x_ref_dev, n, &xr2);
    if (rc != REBK_OK) return rc;
    if (!(xr2 > 0.0) || !std::isfinite(xr2)) return fail(REBK_ERR_INVALID, "x_ref must be non-zero and finite");
  }
  const double bn = std::sqrt(b2), an = std::sqrt(a2);
  if (o->x0_dev) {
    if (o->x0_dev != x) HIP_TRY(hipMemcpyAsync(x, o->x0_dev, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  } else {
    HIP_TRY(hipMemsetAsync(x, 0, n * sizeof(double), st));
  }
  HIP_TRY(hipMemcpyAsync(z, o->b_dev, m * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipEventRecord(h->ev0, st));

  rebk_result_t r{};
  r.status = REBK_NOT_CONVERGED;
  int used = 0;
  for (int64_t q = 0;; ++q) {
    // residuals of the augmented system: f = b - z - A x, g = -A^T z
    HIP_TRY(rebk::launch_resid_f(o->A_dev, o->lda, m, n, o->b_dev, z, x, f, st));
    HIP_TRY(rebk::launch_gemv_t(o->A_dev, o->lda, m, n, z, -1.0, 0.0, g, nullptr, partial, st));
    double e = 0.0;
    bool ok = false;
    if (o->x_ref_dev) {
      double e2 = 0.0;
      HIP_TRY(rebk::launch_err2(x, o->x_ref_dev, n, h->partials, h->nparts, st));
      rc = host_sum(h, h->partials, h->nparts, &e2);
      if (rc != REBK_OK) return rc;
      e = std::sqrt(e2) / std::sqrt(xr2);
      ok = e < o->tol;
    } else {
      double f2 = 0.0, g2 = 0.0;
      rc = dev_sumsq(h, f, m, &f2);
      if (rc == REBK_OK) rc = dev_sumsq(h, g, n, &g2);
      if (rc != REBK_OK) return rc;
      const double rf = std::sqrt(f2) / (bn > 0.0 ? bn : 1.0);
      const double rg = std::sqrt(g2) / (an * bn > 0.0 ? an * bn : 1.0);
      e = rf > rg ? rf : rg;
      ok = rf <= o->tol && rg <= o->tol;
    }
    if (o->err_trace) o->err_trace[q] = e;
    r.rel_err = e;
    if (!std::isfinite(e)) {
      r.status = REBK_DIVERGED;
      break;
    }
    if (ok) {
      r.status = REBK_OK;
      break;
    }
    if (q >= o->max_outer) break;
    // correction: REBK on (f, g) from dz = f, dx = 0, the Philox stream continuing at q * inner
    rebk::SolveArgs a = base_args(h);
    a.b = f;
    a.z_in = f;
    a.x_in = nullptr;
    a.x_out = dx;
    a.z_out = dz;
    a.g = g;
    a.y_out = dy;
    a.x_ref = nullptr;
    a.tol = 0.0;
    a.k0 = q * o->inner_iters;
    a.max_iter = o->inner_iters;
    a.check_every = o->inner_iters;
    rc = run_iterations(h, a, o->kernel, o->grid_wgs, &used);
    if (rc != REBK_OK) return rc;
    rebk::DevStatus ds{};
    HIP_TRY(hipMemcpyAsync(&ds, h->status_d, sizeof(ds), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (ds.status == REBK_ERR_TIMEOUT) return fail(REBK_ERR_TIMEOUT, "grid barrier spin limit exceeded");
    r.iterations += o->inner_iters;
    // z += dz, x += A^T y
    HIP_TRY(rebk::launch_axpy(z, dz, m, st));
    HIP_TRY(rebk::launch_gemv_t(o->A_dev, o->lda, m, n, dy, 1.0, 1.0, x, nullptr, partial, st));
  }
  HIP_TRY(hipEventRecord(h->ev1, st));
  HIP_TRY(hipStreamSynchronize(st));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  r.kernel = used;
  r.time_ms = ms;
  if (res) *res = r;
  return r.status;
}

// ------------------------------------------------------------------ block constants beta

extern "C" int rebk_block_betas(rebk_handle_t h, int32_t max_steps, double rtol, double* beta_row, double* beta_col,
                                double* beta_max, int32_t* steps_max) {
  g_err[0] = 0;
  if (!h) return fail(REBK_ERR_INVALID, "handle is NULL");
  if (max_steps <= 0) return fail(REBK_ERR_INVALID, "max_steps must be positive");
  if (!(rtol >= 0.0)) return fail(REBK_ERR_INVALID, "rtol must be non-negative");
  const int64_t m = h->m, n = h->n;
  // one pass per panel layout: row blocks (Arow: entry (l, c) of block i at n*r0 + c*nI + l),
  // column blocks (Acol: entry (r, c) of block j at ldc*c0 + c*ldc + r)
  struct Pass {
    const void* P;
    std::vector<rebk::GramDesc> desc;
    double* out;
  };
  std::vector<Pass> passes(2);
  passes[0].P = h->Arow;
  passes[0].out = beta_row;
  passes[1].P = h->Acol;
  passes[1].out = beta_col;
  int64_t gram_total = 0;
  int32_t max_d = 0;
  auto add = [&](Pass& p, int64_t base, int64_t rows, int64_t cols, int64_t s_row, int64_t s_col) {
    // block of rows x cols with entry (r, c) at base + r * s_row + c * s_col; Gram of the shorter side
    rebk::GramDesc d{};
    d.base = base;
    if (rows <= cols) {
      d.d = (int32_t)rows; d.L = cols; d.sa = s_row; d.st = s_col;
    } else {
      d.d = (int32_t)cols; d.L = rows; d.sa = s_col; d.st = s_row;
    }
    d.gram = gram_total;
    gram_total += (int64_t)d.d * d.d;
    if (d.d > max_d) max_d = d.d;
    p.desc.push_back(d);
  };
  for (int64_t i = 0; i < h->s; ++i) {
    const int64_t r0 = h->row_off[i], nI = h->row_off[i + 1] - r0;
    add(passes[0], n * r0, nI, n, 1, nI);
  }
  for (int64_t j = 0; j < h->t; ++j) {
    const int64_t c0 = h->col_off[j], nJ = h->col_off[j + 1] - c0;
    add(passes[1], h->ldc * c0, m, nJ, 1, h->ldc);
  }
  if (max_d > 8192) return fail(REBK_ERR_INVALID, "blocks whose shorter side exceeds 8192 are not supported");
  DevBuffers buf;
  double* gram = buf.get((size_t)gram_total);
  if (!gram) return fail(REBK_ERR_OOM, "cannot allocate %lld Gram entries", (long long)gram_total);
  hipStream_t st = h->stream;
  double bmax = 0.0;
  int32_t smax = 0;
  for (Pass& p : passes) {
    const int nb = (int)p.desc.size();
    std::vector<int32_t> tb, ta1, ta2;
    for (int b = 0; b < nb; ++b) {
      const int D = p.desc[b].d;
      for (int a1 = 0; a1 < D; a1 += 16)
        for (int a2 = 0; a2 < D; a2 += 16) {
          tb.push_back(b);
          ta1.push_back(a1);
          ta2.push_back(a2);
        }
    }
    const size_t nt = tb.size();
    rebk::GramDesc* desc_d = (rebk::GramDesc*)buf.get((nb * sizeof(rebk::GramDesc) + 7) / 8);
    int32_t* tiles_d = (int32_t*)buf.get((3 * nt * sizeof(int32_t) + 7) / 8);
    double* lam_d = buf.get(nb);
    double* tr_d = buf.get(nb);
    int32_t* steps_d = (int32_t*)buf.get((nb * sizeof(int32_t) + 7) / 8);
    if (!desc_d || !tiles_d || !lam_d || !tr_d || !steps_d) return fail(REBK_ERR_OOM, "cannot allocate beta scratch");
    HIP_TRY(hipMemcpyAsync(desc_d, p.desc.data(), nb * sizeof(rebk::GramDesc), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(tiles_d, tb.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(tiles_d + nt, ta1.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(tiles_d + 2 * nt, ta2.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(rebk::launch_gram(p.P, h->panel_dtype, desc_d, (int)nt, tiles_d, tiles_d + nt, tiles_d + 2 * nt, gram, st));
    HIP_TRY(rebk::launch_power(desc_d, nb, max_d, gram, max_steps, rtol, lam_d, tr_d, steps_d, st));
    std::vector<double> lam(nb), tr(nb);
    std::vector<int32_t> steps(nb);
    HIP_TRY(hipMemcpyAsync(lam.data(), lam_d, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(tr.data(), tr_d, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(steps.data(), steps_d, nb * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int b = 0; b < nb; ++b) {
      const double beta = tr[b] > 0.0 ? lam[b] / tr[b] : 0.0;
      if (p.out) p.out[b] = beta;
      if (beta > bmax) bmax = beta;
      if (steps[b] > smax) smax = steps[b];
    }
  }
  if (beta_max) *beta_max = bmax;
  if (steps_max) *steps_max = smax;
  return REBK_OK;
}

// ------------------------------------------------------------------ learned warm start

struct rebk_mlp {
  int32_t in = 0, hid = 0, max_batch = 0;
  double out_scale = 1.0;  // x0 = out_scale A^T y
  int64_t out = 0, n = 0;
  hipStream_t stream = nullptr;
  int64_t t = 0;  // Adam steps taken
  bool have_grads = false;
  // parameters W1 (hid x in), c1, W2 (hid x hid), c2, W3 (out x hid), c3: FP32 masters,
  // gradients, Adam moments; half copies of the three weight matrices
  float* p[6] = {};
  float* g[6] = {};
  float* m1[6] = {};
  float* m2[6] = {};
  int64_t cnt[6] = {};
  _Float16* w16[3] = {};
  _Float16* A16 = nullptr;  // out x n
  double* A64 = nullptr;    // out x n, for x0 = out_scale A^T y in FP64 at inference
  double* Y64 = nullptr;    // max_batch x out
  // activations and signals for max_batch rows
  _Float16 *B16 = nullptr, *H1 = nullptr, *H2 = nullptr, *Y16 = nullptr, *R16 = nullptr, *DY16 = nullptr,
           *D2 = nullptr, *D1 = nullptr;
  float *C = nullptr, *Y = nullptr, *X0 = nullptr, *R = nullptr, *DY = nullptr, *DH = nullptr, *pmax = nullptr;
  double* psq = nullptr;
  int nparts = 256;
  std::vector<void*> owned;

  ~rebk_mlp() {
    for (void* q : owned) (void)hipFree(q);
  }
  template <typename T>
  bool alloc(T*& q, size_t count) {
    if (hipMalloc((void**)&q, (count > 0 ? count : 1) * sizeof(T)) != hipSuccess) return false;
    owned.push_back((void*)q);
    return true;
  }
};

namespace {

int mlp_forward_impl(rebk_mlp* w, const double* B, int32_t batch, double b_scale) {
  hipStream_t st = w->stream;
  const int in = w->in, hid = w->hid, out = (int)w->out, n = (int)w->n;
  HIP_TRY(rebk::launch_to_half_f64(B, (int64_t)batch * in, b_scale, w->B16, st));
  HIP_TRY(rebk::launch_gemm_f16(false, true, batch, hid, in, 1.f, w->B16, in, w->w16[0], in, 0.f, w->C, hid, st));
  HIP_TRY(rebk::launch_bias_act(w->C, w->p[1], batch, hid, 1, w->H1, nullptr, st));
  HIP_TRY(rebk::launch_gemm_f16(false, true, batch, hid, hid, 1.f, w->H1, hid, w->w16[1], hid, 0.f, w->C, hid, st));
  HIP_TRY(rebk::launch_bias_act(w->C, w->p[3], batch, hid, 1, w->H2, nullptr, st));
  HIP_TRY(rebk::launch_gemm_f16(false, true, batch, out, hid, 1.f, w->H2, hid, w->w16[2], hid, 0.f, w->Y, out, st));
  HIP_TRY(rebk::launch_bias_act(w->Y, w->p[5], batch, out, 0, w->Y16, w->Y, st));
  // x0 = A^T y for every row: X0 = Y A
  HIP_TRY(rebk::launch_gemm_f16(false, false, batch, n, out, (float)w->out_scale, w->Y16, out, w->A16, n, 0.f, w->X0, n,
                                st));
  return REBK_OK;
}

int mlp_check_batch(const rebk_mlp* w, int32_t batch) {
  if (batch <= 0 || batch > w->max_batch || batch % 64)
    return fail(REBK_ERR_INVALID, "batch must be a positive multiple of 64 up to %d", w->max_batch);
  return REBK_OK;
}

}  // namespace

extern "C" {

int rebk_mlp_create(rebk_mlp_t* out, int32_t in_dim, int32_t hidden, const double* A_dev, int64_t out_dim, int64_t n,
                    double out_scale, int32_t max_batch, uint64_t seed, void* stream) {
  g_err[0] = 0;
  if (!out) return fail(REBK_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!A_dev) return fail(REBK_ERR_INVALID, "A is NULL");
  if (in_dim <= 0 || hidden <= 0 || out_dim <= 0 || n <= 0 || max_batch <= 0 || in_dim % 64 || hidden % 64 ||
      out_dim % 64 || n % 64 || max_batch % 64)
    return fail(REBK_ERR_INVALID, "in_dim, hidden, out_dim, n and max_batch must be positive multiples of 64");
  if (out_dim > (1 << 26) || in_dim > (1 << 26)) return fail(REBK_ERR_INVALID, "dimensions too large");
  if (!(out_scale > 0.0) || !std::isfinite(out_scale)) return fail(REBK_ERR_INVALID, "out_scale must be positive");
  rebk_mlp* w = new (std::nothrow) rebk_mlp();
  if (!w) return fail(REBK_ERR_OOM, "host allocation failed");
  w->in = in_dim;
  w->hid = hidden;
  w->out = out_dim;
  w->n = n;
  w->max_batch = max_batch;
  w->out_scale = out_scale;
  w->stream = (hipStream_t)stream;
  const int64_t cnt[6] = {(int64_t)hidden * in_dim, hidden, (int64_t)hidden * hidden, hidden, out_dim * hidden, out_dim};
  bool ok = true;
  for (int q = 0; q < 6; ++q) {
    w->cnt[q] = cnt[q];
    ok = ok && w->alloc(w->p[q], cnt[q]) && w->alloc(w->g[q], cnt[q]) && w->alloc(w->m1[q], cnt[q]) &&
         w->alloc(w->m2[q], cnt[q]);
  }
  for (int q = 0; q < 3; ++q) ok = ok && w->alloc(w->w16[q], cnt[2 * q]);
  const int64_t B = max_batch;
  ok = ok && w->alloc(w->A16, out_dim * n) && w->alloc(w->A64, out_dim * n) && w->alloc(w->Y64, B * out_dim) &&
       w->alloc(w->B16, B * in_dim) && w->alloc(w->H1, B * hidden) &&
       w->alloc(w->H2, B * hidden) && w->alloc(w->Y16, B * out_dim) && w->alloc(w->R16, B * n) &&
       w->alloc(w->DY16, B * out_dim) && w->alloc(w->D2, B * hidden) && w->alloc(w->D1, B * hidden) &&
       w->alloc(w->C, B * hidden) && w->alloc(w->Y, B * out_dim) && w->alloc(w->X0, B * n) && w->alloc(w->R, B * n) &&
       w->alloc(w->DY, B * out_dim) && w->alloc(w->DH, B * hidden) && w->alloc(w->pmax, w->nparts) &&
       w->alloc(w->psq, w->nparts);
  if (!ok) {
    delete w;
    return fail(REBK_ERR_OOM, "cannot allocate the network");
  }
  hipStream_t st = w->stream;
  hipError_t e = rebk::launch_to_half_f64(A_dev, out_dim * n, 1.0, w->A16, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w->A64, A_dev, out_dim * n * sizeof(double), hipMemcpyDeviceToDevice, st);
  // weights uniform in +-1/sqrt(fan_in) (Philox, seed), biases and moments zero
  const int fan[3] = {in_dim, hidden, hidden};
  for (int q = 0; q < 3 && e == hipSuccess; ++q) {
    e = rebk::launch_init_uniform(w->p[2 * q], cnt[2 * q], (float)(1.0 / std::sqrt((double)fan[q])), seed,
                                  (uint64_t)q, st);
    if (e == hipSuccess) e = rebk::launch_to_half_f32(w->p[2 * q], cnt[2 * q], w->w16[q], st);
  }
  for (int q = 0; q < 6 && e == hipSuccess; ++q) {
    if (q % 2 == 1) e = hipMemsetAsync(w->p[q], 0, cnt[q] * sizeof(float), st);
    if (e == hipSuccess) e = hipMemsetAsync(w->m1[q], 0, cnt[q] * sizeof(float), st);
    if (e == hipSuccess) e = hipMemsetAsync(w->m2[q], 0, cnt[q] * sizeof(float), st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete w;
    return fail(REBK_ERR_HIP, "network setup: %s", hipGetErrorString(e));
  }
  *out = w;
  return REBK_OK;
}

void rebk_mlp_destroy(rebk_mlp_t w) {
  if (!w) return;
  (void)hipStreamSynchronize(w->stream);
  delete w;
}

int rebk_mlp_set_params(rebk_mlp_t w, const float* W1, const float* c1, const float* W2, const float* c2,
                        const float* W3, const float* c3) {
  if (!w) return fail(REBK_ERR_INVALID, "network is NULL");
  const float* src[6] = {W1, c1, W2, c2, W3, c3};
  for (int q = 0; q < 6; ++q) {
    if (!src[q]) continue;
    HIP_TRY(hipMemcpyAsync(w->p[q], src[q], w->cnt[q] * sizeof(float), hipMemcpyHostToDevice, w->stream));
    if (q % 2 == 0) HIP_TRY(rebk::launch_to_half_f32(w->p[q], w->cnt[q], w->w16[q / 2], w->stream));
  }
  HIP_TRY(hipStreamSynchronize(w->stream));
  return REBK_OK;
}

int rebk_mlp_get_params(rebk_mlp_t w, float* W1, float* c1, float* W2, float* c2, float* W3, float* c3) {
  if (!w) return fail(REBK_ERR_INVALID, "network is NULL");
  float* dst[6] = {W1, c1, W2, c2, W3, c3};
  for (int q = 0; q < 6; ++q)
    if (dst[q]) HIP_TRY(hipMemcpyAsync(dst[q], w->p[q], w->cnt[q] * sizeof(float), hipMemcpyDeviceToHost, w->stream));
  HIP_TRY(hipStreamSynchronize(w->stream));
  return REBK_OK;
}

int rebk_mlp_forward(rebk_mlp_t w, const double* B_dev, int32_t batch, double b_scale, double* X0_dev, double* Y_dev) {
  g_err[0] = 0;
  if (!w) return fail(REBK_ERR_INVALID, "network is NULL");
  if (!B_dev || !X0_dev) return fail(REBK_ERR_INVALID, "B and X0 are required");
  int rc = mlp_check_batch(w, batch);
  if (rc != REBK_OK) return rc;
  rc = mlp_forward_impl(w, B_dev, batch, b_scale);
  if (rc != REBK_OK) return rc;
  // x0 = out_scale A^T y in FP64 from the FP64 A: inside range(A^T) to FP64 rounding, which REBK
  // needs to reach A^+ b (its x-steps never remove a component outside range(A^T))
  double* Y64 = Y_dev ? Y_dev : w->Y64;
  HIP_TRY(rebk::launch_widen(w->Y, (int64_t)batch * w->out, Y64, w->stream));
  HIP_TRY(rebk::launch_gemm_f64(batch, (int)w->n, (int)w->out, w->out_scale, Y64, (int)w->out, w->A64, (int)w->n, X0_dev,
                                (int)w->n, w->stream));
  HIP_TRY(hipStreamSynchronize(w->stream));
  return REBK_OK;
}

int rebk_mlp_grad(rebk_mlp_t w, const double* B_dev, const double* Xt_dev, int32_t batch, double b_scale,
                  double* loss) {
  g_err[0] = 0;
  if (!w) return fail(REBK_ERR_INVALID, "network is NULL");
  if (!B_dev || !Xt_dev) return fail(REBK_ERR_INVALID, "B and Xt are required");
  int rc = mlp_check_batch(w, batch);
  if (rc != REBK_OK) return rc;
  rc = mlp_forward_impl(w, B_dev, batch, b_scale);
  if (rc != REBK_OK) return rc;
  hipStream_t st = w->stream;
  const int in = w->in, hid = w->hid, out = (int)w->out, n = (int)w->n;
  const int64_t rn = (int64_t)batch * n;
  HIP_TRY(rebk::launch_mlp_residual(w->X0, Xt_dev, rn, w->R, w->psq, w->pmax, w->nparts, st));
  std::vector<double> sq(w->nparts);
  std::vector<float> mx(w->nparts);
  HIP_TRY(hipMemcpyAsync(sq.data(), w->psq, w->nparts * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(mx.data(), w->pmax, w->nparts * sizeof(float), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double total = 0.0, rmax = 0.0;
  for (int q = 0; q < w->nparts; ++q) {
    total += sq[q];
    rmax = mx[q] > rmax ? mx[q] : rmax;
  }
  if (loss) *loss = total / (2.0 * batch);
  if (!std::isfinite(total)) return fail(REBK_ERR_INVALID, "the loss is not finite");
  // residual scaled by a power of two (largest magnitude in [4, 8]) before half rounding
  const double s = rmax > 0.0 ? std::ldexp(1.0, 3 - (int)std::ceil(std::log2(rmax))) : 1.0;
  const float k = (float)(w->out_scale / (s * batch));
  HIP_TRY(rebk::launch_scale_half(w->R, rn, (float)s, w->R16, st));
  // dY = (s R) A^T
  HIP_TRY(rebk::launch_gemm_f16(false, true, batch, out, n, 1.f, w->R16, n, w->A16, n, 0.f, w->DY, out, st));
  HIP_TRY(rebk::launch_to_half_f32(w->DY, (int64_t)batch * out, w->DY16, st));
  // layer 3
  HIP_TRY(rebk::launch_gemm_f16(true, false, out, hid, batch, k, w->DY16, out, w->H2, hid, 0.f, w->g[4], hid, st));
  HIP_TRY(rebk::launch_colsum_half(w->DY16, batch, out, k, w->g[5], st));
  HIP_TRY(rebk::launch_gemm_f16(false, false, batch, hid, out, 1.f, w->DY16, out, w->w16[2], hid, 0.f, w->DH, hid, st));
  HIP_TRY(rebk::launch_relu_back(w->DH, w->H2, (int64_t)batch * hid, w->D2, st));
  // layer 2
  HIP_TRY(rebk::launch_gemm_f16(true, false, hid, hid, batch, k, w->D2, hid, w->H1, hid, 0.f, w->g[2], hid, st));
  HIP_TRY(rebk::launch_colsum_half(w->D2, batch, hid, k, w->g[3], st));
  HIP_TRY(rebk::launch_gemm_f16(false, false, batch, hid, hid, 1.f, w->D2, hid, w->w16[1], hid, 0.f, w->DH, hid, st));
  HIP_TRY(rebk::launch_relu_back(w->DH, w->H1, (int64_t)batch * hid, w->D1, st));
  // layer 1
  HIP_TRY(rebk::launch_gemm_f16(true, false, hid, in, batch, k, w->D1, hid, w->B16, in, 0.f, w->g[0], in, st));
  HIP_TRY(rebk::launch_colsum_half(w->D1, batch, hid, k, w->g[1], st));
  w->have_grads = true;
  return REBK_OK;
}

int rebk_mlp_get_grads(rebk_mlp_t w, float* gW1, float* gc1, float* gW2, float* gc2, float* gW3, float* gc3) {
  if (!w) return fail(REBK_ERR_INVALID, "network is NULL");
  if (!w->have_grads) return fail(REBK_ERR_INVALID, "no gradients computed yet");
  float* dst[6] = {gW1, gc1, gW2, gc2, gW3, gc3};
  for (int q = 0; q < 6; ++q)
    if (dst[q]) HIP_TRY(hipMemcpyAsync(dst[q], w->g[q], w->cnt[q] * sizeof(float), hipMemcpyDeviceToHost, w->stream));
  HIP_TRY(hipStreamSynchronize(w->stream));
  return REBK_OK;
}

int rebk_mlp_adam(rebk_mlp_t w, double lr, double beta1, double beta2, double eps) {
  if (!w) return fail(REBK_ERR_INVALID, "network is NULL");
  if (!w->have_grads) return fail(REBK_ERR_INVALID, "no gradients computed yet");
  if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return fail(REBK_ERR_INVALID, "bad Adam hyper-parameters");
  w->t += 1;
  const float c1 = (float)(1.0 - std::pow(beta1, (double)w->t)), c2 = (float)(1.0 - std::pow(beta2, (double)w->t));
  for (int q = 0; q < 6; ++q)
    HIP_TRY(rebk::launch_adam(w->p[q], w->g[q], w->m1[q], w->m2[q], w->cnt[q], (float)lr, (float)beta1,
                              (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2), (float)eps, c1, c2,
                              q % 2 == 0 ? w->w16[q / 2] : nullptr, w->stream));
  return REBK_OK;
}

int rebk_mlp_train_step(rebk_mlp_t w, const double* B_dev, const double* Xt_dev, int32_t batch, double b_scale,
                        double lr, double* loss) {
  int rc = rebk_mlp_grad(w, B_dev, Xt_dev, batch, b_scale, loss);
  if (rc != REBK_OK) return rc;
  return rebk_mlp_adam(w, lr, 0.9, 0.999, 1e-8);
}

}  // extern "C"
