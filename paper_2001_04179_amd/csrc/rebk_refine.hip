// FP64 kernels of the refinement loop around REBK: the residuals of the augmented least-squares
// system  z + A x = b,  A^T z = 0  on the caller's FP64 matrix, and the update x += A^T dy.
//
// All sums run in a fixed order (per-row workgroup reductions, row chunks added in chunk order),
// so a run is reproducible bit for bit.  These kernels stream A once per call: they are HBM-bound
// (8 m n bytes per product) and run once per outer step, next to thousands of inner iterations.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rebk_device.h"
#include "rebk_internal.h"

namespace rebk {
namespace {

using namespace dev;

constexpr int kRows = 256;  // rows per chunk of the transposed product

// f[r] = (b[r] - z[r]) - sum_c A[r, c] x[c]; one workgroup per row.
__global__ void __launch_bounds__(256) resid_f_kernel(const double* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                      const double* __restrict__ b, const double* __restrict__ z,
                                                      const double* __restrict__ x, double* __restrict__ f) {
  __shared__ double red[256];
  for (int64_t r = blockIdx.x; r < m; r += gridDim.x) {
    const double* row = A + r * lda;
    double acc = 0.0;
    for (int64_t c = threadIdx.x; c < n; c += blockDim.x) acc += row[c] * x[c];
    const double s = wg_sum(acc, red);
    if (threadIdx.x == 0) f[r] = (b[r] - z[r]) - s;
  }
}

// partial[q * n + c] = sum over rows r of chunk q (kRows rows) of A[r, c] v[r]; thread per column.
__global__ void __launch_bounds__(256) gemv_t_partial_kernel(const double* __restrict__ A, int64_t lda, int64_t m,
                                                             int64_t n, const double* __restrict__ v,
                                                             double* __restrict__ partial) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t q = blockIdx.y;
  if (c >= n) return;
  const int64_t r0 = q * kRows, r1 = r0 + kRows < m ? r0 + kRows : m;
  double acc = 0.0;
  for (int64_t r = r0; r < r1; ++r) acc += A[r * lda + c] * v[r];
  partial[q * n + c] = acc;
}

// out[c] = beta * out[c] + alpha * sum_q partial[q * n + c] (q ascending); sq[c] = out[c]^2 if sq.
__global__ void gemv_t_finish_kernel(const double* __restrict__ partial, int64_t nchunks, int64_t n, double alpha,
                                     double beta, double* __restrict__ out, double* __restrict__ sq) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double s = 0.0;
  for (int64_t q = 0; q < nchunks; ++q) s += partial[q * n + c];
  const double o = beta == 0.0 ? alpha * s : beta * out[c] + alpha * s;
  out[c] = o;
  if (sq) sq[c] = o * o;
}

__global__ void axpy_kernel(double* __restrict__ y, const double* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += x[i];
}

// partials[blk] = sum over a fixed slice of v[i]^2 (or of the entries of a matrix, row by row)
__global__ void sumsq_kernel(const double* __restrict__ v, int64_t n, double* __restrict__ partials) {
  __shared__ double red[256];
  double e = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    e += v[i] * v[i];
  const double tot = wg_sum(e, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ void sumsq_matrix_kernel(const double* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                    double* __restrict__ partials) {
  __shared__ double red[256];
  double e = 0.0;
  for (int64_t r = blockIdx.x; r < m; r += gridDim.x)
    for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
      const double a = A[r * lda + c];
      e += a * a;
    }
  const double tot = wg_sum(e, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

}  // namespace

int64_t refine_chunks(int64_t m) { return (m + kRows - 1) / kRows; }

hipError_t launch_resid_f(const double* A, int64_t lda, int64_t m, int64_t n, const double* b, const double* z,
                          const double* x, double* f, hipStream_t st) {
  const unsigned g = (unsigned)(m < 65535 ? m : 65535);
  hipLaunchKernelGGL(resid_f_kernel, dim3(g), dim3(256), 0, st, A, lda, m, n, b, z, x, f);
  return hipGetLastError();
}

hipError_t launch_gemv_t(const double* A, int64_t lda, int64_t m, int64_t n, const double* v, double alpha,
                         double beta, double* out, double* sq, double* partial, hipStream_t st) {
  const int64_t nq = refine_chunks(m);
  if (nq > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gemv_t_partial_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nq), dim3(256), 0, st, A, lda,
                     m, n, v, partial);
  hipLaunchKernelGGL(gemv_t_finish_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, partial, nq, n, alpha,
                     beta, out, sq);
  return hipGetLastError();
}

hipError_t launch_axpy(double* y, const double* x, int64_t n, hipStream_t st) {
  const int64_t g = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)(g > 0 ? g : 1)), dim3(256), 0, st, y, x, n);
  return hipGetLastError();
}

hipError_t launch_sumsq(const double* v, int64_t n, double* partials, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(nparts), dim3(256), 0, st, v, n, partials);
  return hipGetLastError();
}

hipError_t launch_sumsq_matrix(const double* A, int64_t lda, int64_t m, int64_t n, double* partials, int nparts,
                               hipStream_t st) {
  hipLaunchKernelGGL(sumsq_matrix_kernel, dim3(nparts), dim3(256), 0, st, A, lda, m, n, partials);
  return hipGetLastError();
}

}  // namespace rebk
