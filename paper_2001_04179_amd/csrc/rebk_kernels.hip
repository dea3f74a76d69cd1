// HIP kernels for gfx950 (MI355X): panel packing, FP64 block weights, the counter-based block
// sampler, the single-workgroup REBK iteration kernel and the residual / error kernels (Du, Si,
// Sun, arXiv:2001.04179, Algorithm 1).  The whole-chip iteration kernel is in rebk_grid.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rebk_device.h"
#include "rebk_internal.h"

namespace rebk {
namespace {

using namespace dev;

__global__ void philox_kernel(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                              int64_t count, uint64_t* __restrict__ out) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
    uint64_t w0 = c0 + (uint64_t)q, w1 = c1, w2 = c2, w3 = c3;
    philox4x64_10(w0, w1, w2, w3, k0, k1);
    out[4 * q + 0] = w0;
    out[4 * q + 1] = w1;
    out[4 * q + 2] = w2;
    out[4 * q + 3] = w3;
  }
}

__global__ void sample_kernel(const uint64_t* __restrict__ T_row, int s, const uint64_t* __restrict__ T_col, int t,
                              uint64_t seed, uint64_t sys, int64_t k0, int64_t count, int32_t* __restrict__ j_out,
                              int32_t* __restrict__ i_out) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
    uint64_t c0 = (uint64_t)(k0 + q), c1 = sys, c2 = 0, c3 = 0;
    philox4x64_10(c0, c1, c2, c3, seed, 0);
    j_out[q] = draw_block(T_col, t, c0);
    i_out[q] = draw_block(T_row, s, c1);
  }
}

// ------------------------------------------------------------------ packing

// Column panels: A^T, row-major (n x ldc, ldc >= m, pad entries zero): entry (r, c) at c * ldc + r,
// so column block j is the contiguous m x nJ_j column-major panel (column stride ldc) at offset
// ldc * col_off[j].  32 x 32 tiles through LDS.
template <typename TIn, typename TP>
__global__ void pack_col_kernel(const TIn* __restrict__ A, int64_t lda, int64_t m, int64_t n, int64_t ldc,
                                TP* __restrict__ Acol) {
  __shared__ double tile[32][33];
  for (int64_t R = (int64_t)blockIdx.y * 32; R < m; R += (int64_t)gridDim.y * 32) {
    for (int64_t C = (int64_t)blockIdx.x * 32; C < n; C += (int64_t)gridDim.x * 32) {
      for (int q = threadIdx.y; q < 32; q += blockDim.y) {
        const int64_t r = R + q, c = C + threadIdx.x;
        tile[q][threadIdx.x] = (r < m && c < n) ? (double)A[r * lda + c] : 0.0;
      }
      __syncthreads();
      for (int q = threadIdx.y; q < 32; q += blockDim.y) {
        const int64_t r = R + threadIdx.x, c = C + q;
        if (r < m && c < n) Acol[c * ldc + r] = narrow<TP>(tile[threadIdx.x][q]);
      }
      __syncthreads();
    }
  }
}

// Row panels: block i is stored column-major (n x nI_i) at offset n * row_off[i], so entry
// (l, c) of the block sits at c * nI_i + (l - row_off[i]).  32 x 32 tiles through LDS.
template <typename TIn, typename TP>
__global__ void pack_row_kernel(const TIn* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                const int64_t* __restrict__ row_off, const int32_t* __restrict__ rowblk,
                                TP* __restrict__ Arow) {
  __shared__ double tile[32][33];
  for (int64_t R = (int64_t)blockIdx.y * 32; R < m; R += (int64_t)gridDim.y * 32) {
    for (int64_t C = (int64_t)blockIdx.x * 32; C < n; C += (int64_t)gridDim.x * 32) {
      for (int q = threadIdx.y; q < 32; q += blockDim.y) {
        const int64_t r = R + q, c = C + threadIdx.x;
        tile[q][threadIdx.x] = (r < m && c < n) ? (double)A[r * lda + c] : 0.0;
      }
      __syncthreads();
      for (int q = threadIdx.y; q < 32; q += blockDim.y) {
        const int64_t l = R + threadIdx.x, c = C + q;
        if (l < m && c < n) {
          const int i = rowblk[l];
          const int64_t r0 = row_off[i], nI = row_off[i + 1] - r0;
          Arow[n * r0 + c * nI + (l - r0)] = narrow<TP>(tile[threadIdx.x][q]);
        }
      }
      __syncthreads();
    }
  }
}

template <typename TIn>
__global__ void finite_kernel(const TIn* __restrict__ A, int64_t lda, int64_t m, int64_t n, int* bad) {
  int any = 0;
  for (int64_t r = blockIdx.y; r < m; r += gridDim.y)
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
      if (!isfinite((double)A[r * lda + c])) any = 1;
  if (any) atomicOr(bad, 1);
}

// ------------------------------------------------------------------ block weights (FP64, fixed order)
// ||A_{I_i,:}||_F^2 and ||A_{:,J_j}||_F^2 summed as: per matrix row, squares in ascending column
// order; then those row sums in ascending row order.  Every product is rounded before the add.

template <typename TP>
__global__ void row_sq_kernel(const TP* __restrict__ Arow, int64_t m, int64_t n, const int64_t* __restrict__ row_off,
                              const int32_t* __restrict__ rowblk, double* __restrict__ row_sq) {
#pragma clang fp contract(off)
  for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < m; l += (int64_t)gridDim.x * blockDim.x) {
    const int i = rowblk[l];
    const int64_t r0 = row_off[i], nI = row_off[i + 1] - r0;
    const TP* p = Arow + n * r0 + (l - r0);
    double acc = 0.0;
    for (int64_t c = 0; c < n; ++c) {
      const double v = widen(p[c * nI]);
      const double sq = v * v;
      acc = acc + sq;
    }
    row_sq[l] = acc;
  }
}

template <typename TP>
__global__ void colrow_sq_kernel(const TP* __restrict__ Acol, int64_t m, int64_t ldc, const int64_t* __restrict__ col_off,
                                 int t, double* __restrict__ colrow_sq) {
#pragma clang fp contract(off)
  const int64_t total = m * (int64_t)t;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / m, r = e - j * m;
    const int64_t c0 = col_off[j], nJ = col_off[j + 1] - c0;
    const TP* p = Acol + ldc * c0 + r;
    double acc = 0.0;
    for (int64_t c = 0; c < nJ; ++c) {
      const double v = widen(p[c * ldc]);
      const double sq = v * v;
      acc = acc + sq;
    }
    colrow_sq[e] = acc;
  }
}

__global__ void sum_rows_kernel(const double* __restrict__ row_sq, const int64_t* __restrict__ row_off, int s,
                                double* __restrict__ w_row) {
#pragma clang fp contract(off)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < s; i += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int64_t l = row_off[i]; l < row_off[i + 1]; ++l) acc = acc + row_sq[l];
    w_row[i] = acc;
  }
}

__global__ void sum_cols_kernel(const double* __restrict__ colrow_sq, int64_t m, int t, double* __restrict__ w_col) {
#pragma clang fp contract(off)
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < t; j += gridDim.x * blockDim.x) {
    const double* p = colrow_sq + (int64_t)j * m;
    double acc = 0.0;
    for (int64_t r = 0; r < m; ++r) acc = acc + p[r];
    w_col[j] = acc;
  }
}

// ------------------------------------------------------------------ one-workgroup solver
// The whole solve runs inside one workgroup: z (m), x (n) and the block vectors live in LDS, the
// panels stream from L2/HBM.  Meant for systems whose iterate fits in LDS (the latency of a grid
// barrier would dominate their tiny blocks).

size_t wg_lds_doubles(const SolveArgs& a) {
  return (size_t)a.m + (size_t)a.n + (size_t)a.max_nJ + (size_t)a.max_nI + kWgThreads + 8;
}

template <typename TP>
__global__ void __launch_bounds__(kWgThreads) wg_solve_kernel(SolveArgs a) {
  extern __shared__ double lds[];
  __shared__ int s_j[64], s_i[64];
  __shared__ int s_flag;
  const int T = blockDim.x, tid = threadIdx.x;
  const int64_t m = a.m, n = a.n;
  double* z = lds;
  double* x = z + m;
  double* v = x + n;
  double* u = v + a.max_nJ;
  double* red = u + a.max_nI;
  const TP* __restrict__ Arow = (const TP*)a.Arow;
  const TP* __restrict__ Acol = (const TP*)a.Acol;

  for (int64_t r = tid; r < m; r += T) z[r] = a.z_in ? a.z_in[r] : a.b[r];
  for (int64_t c = tid; c < n; c += T) x[c] = a.x_in ? a.x_in[c] : 0.0;
  if (a.y_out)
    for (int64_t r = tid; r < m; r += T) a.y_out[r] = 0.0;
  __syncthreads();

  const int64_t ce = a.check_every > 0 ? a.check_every : 1;
  const bool checking = a.x_ref != nullptr && a.tol > 0.0;
  int status = 0, stopped = 0;
  int64_t q_done = 0;
  double last_err2 = -1.0;
  int64_t last_check = -1;

  for (int64_t q = 0; q < a.max_iter; ++q) {
    const int64_t k = a.k0 + q + 1;
    if ((q & 63) == 0) {
      if (tid < 64 && q + tid < a.max_iter) {
        int jj, ii;
        draw_pair(a, k + tid, jj, ii);
        s_j[tid] = jj;
        s_i[tid] = ii;
      }
      __syncthreads();
    }
    const int j = s_j[q & 63], i = s_i[q & 63];
    if (tid == 0 && a.trace_j) {
      a.trace_j[q] = j;
      a.trace_i[q] = i;
    }

    // z^k = z^{k-1} - alpha/||A_{:,J}||_F^2 * A_{:,J} (A_{:,J}^T z^{k-1})
    const int64_t c0 = a.col_off[j];
    const int nJ = (int)(a.col_off[j + 1] - c0);
    const TP* __restrict__ P = Acol + a.ldc * c0;  // (r, c) at c * ldc + r
    colsum_colmajor(P, m, a.ldc, nJ, z, v, red);
    if (a.g) {  // refinement: project onto {A^T z = g}
      for (int c = tid; c < nJ; c += T) v[c] -= a.g[c0 + c];
      __syncthreads();
    }
    const double cc = a.coef_col[j];
    for (int64_t r = tid; r < m; r += T) {
      double acc = 0.0;
      for (int c = 0; c < nJ; ++c) acc += widen(P[c * a.ldc + r]) * v[c];
      z[r] -= cc * acc;
    }
    __syncthreads();

    // x^k = x^{k-1} - alpha/||A_{I,:}||_F^2 * A_{I,:}^T (A_{I,:} x^{k-1} - b_I + z^k_I)
    const int64_t r0 = a.row_off[i];
    const int nI = (int)(a.row_off[i + 1] - r0);
    const TP* __restrict__ Q = Arow + n * r0;  // (c, l) at c * nI + l
    for (int lb = 0; lb < nI; lb += T) {
      const int lw = min(T, nI - lb);
      const int ng = T / lw;
      const int g = tid / lw, l = lb + tid % lw;
      double acc = 0.0;
      if (g < ng)
        for (int64_t c = g; c < n; c += ng) acc += widen(Q[c * nI + l]) * x[c];
      red[tid] = acc;
      __syncthreads();
      if (tid < lw) {
        double s = 0.0;
        for (int gg = 0; gg < ng; ++gg) s += red[gg * lw + tid];
        u[lb + tid] = (s - a.b[r0 + lb + tid]) + z[r0 + lb + tid];
      }
      __syncthreads();
    }
    const double cr = a.coef_row[i];
    for (int64_t c = tid; c < n; c += T) {
      double acc = 0.0;
      const TP* col = Q + c * nI;
      for (int l = 0; l < nI; ++l) acc += widen(col[l]) * u[l];
      x[c] -= cr * acc;
    }
    if (a.y_out)  // refinement: x - x_in = A^T y
      for (int l = tid; l < nI; l += T) a.y_out[r0 + l] -= cr * u[l];
    __syncthreads();
    q_done = q + 1;

    if (checking && ((q + 1) % ce == 0 || q + 1 == a.max_iter)) {
      double e = 0.0;
      for (int64_t c = tid; c < n; c += T) {
        const double d = x[c] - a.x_ref[c];
        e += d * d;
      }
      const double e2 = wg_sum(e, red);
      last_err2 = e2;
      last_check = k;
      const double rel = sqrt(e2) / sqrt(a.xref_sq);
      if (rel < a.tol) { stopped = 1; status = 0; break; }
      if (!isfinite(e2) || rel > 1e6) { stopped = 1; status = 2; break; }
    }
  }

  for (int64_t r = tid; r < m; r += T)
    if (a.z_out) a.z_out[r] = z[r];
  for (int64_t c = tid; c < n; c += T) a.x_out[c] = x[c];
  if (tid == 0) {
    if (!stopped && checking) status = 1;
    a.status->status = status;
    a.status->stopped = stopped;
    a.status->last_k = a.k0 + q_done;
    a.status->err2 = last_err2;
    a.status->check_k = last_check;
  }
  (void)s_flag;
}

// ------------------------------------------------------------------ residual / error norms

// partials[blk] = sum over a slice of rows of (b - z - A x)_r^2 and, in partials[nparts + blk],
// a slice of columns of (A^T z)_c^2.  Fixed slices, fixed order: deterministic.
template <typename TP>
__global__ void residual_kernel(SolveArgs a, const double* __restrict__ x, const double* __restrict__ z,
                                double* __restrict__ partials) {
  __shared__ double red[kWgThreads];
  const TP* __restrict__ Arow = (const TP*)a.Arow;
  const TP* __restrict__ Acol = (const TP*)a.Acol;
  const int64_t m = a.m, n = a.n;
  const int nb = gridDim.x, blk = blockIdx.x, tid = threadIdx.x;
  double f2 = 0.0, g2 = 0.0;
  // rows of A x through the row panels: entry (l, c) at n*r0 + c*nI + (l - r0)
  for (int64_t l = (int64_t)blk * blockDim.x + tid; l < m; l += (int64_t)nb * blockDim.x) {
    int lo = 0, hi = a.s - 1;
    while (lo < hi) { const int mid = (lo + hi + 1) >> 1; if (a.row_off[mid] <= l) lo = mid; else hi = mid - 1; }
    const int64_t r0 = a.row_off[lo], nI = a.row_off[lo + 1] - r0;
    const TP* p = Arow + n * r0 + (l - r0);
    double acc = 0.0;
    for (int64_t c = 0; c < n; ++c) acc += widen(p[c * nI]) * x[c];
    const double f = a.b[l] - z[l] - acc;
    f2 += f * f;
  }
  // columns of A^T z through the column panels (A^T, row-major): entry (r, c) at c * ldc + r
  for (int64_t c = (int64_t)blk * blockDim.x + tid; c < n; c += (int64_t)nb * blockDim.x) {
    const TP* p = Acol + c * a.ldc;
    double acc = 0.0;
    for (int64_t r = 0; r < m; ++r) acc += widen(p[r]) * z[r];
    g2 += acc * acc;
  }
  const double F = wg_sum(f2, red);
  const double Gs = wg_sum(g2, red);
  if (tid == 0) {
    partials[blk] = F;
    partials[nb + blk] = Gs;
  }
}

__global__ void err2_kernel(const double* __restrict__ x, const double* __restrict__ xr, int64_t n,
                            double* __restrict__ partials) {
  __shared__ double red[kWgThreads];
  double e = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const double d = x[c] - xr[c];
    e += d * d;
  }
  const double tot = wg_sum(e, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_pack(const void* A, int a_dtype, int64_t lda, int panel_dtype, int64_t m, int64_t n, int64_t ldc,
                       const int64_t* row_off_d, const int64_t* col_off_d, const int32_t* rowblk_d,
                       const int32_t* colblk_d, void* Arow, void* Acol, hipStream_t st) {
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const unsigned gy = (unsigned)(m < 65535 ? m : 65535);
    const unsigned gx = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    const unsigned ty = (unsigned)((m + 31) / 32 < 65535 ? (m + 31) / 32 : 65535);
    const unsigned tx = (unsigned)((n + 31) / 32 < 65535 ? (n + 31) / 32 : 65535);
    if (a_dtype == 0) {
      hipLaunchKernelGGL((pack_col_kernel<double, TP>), dim3(tx, ty), dim3(32, 8), 0, st, (const double*)A, lda, m, n,
                         ldc, (TP*)Acol);
      hipLaunchKernelGGL((pack_row_kernel<double, TP>), dim3(tx, ty), dim3(32, 8), 0, st, (const double*)A, lda, m, n,
                         row_off_d, rowblk_d, (TP*)Arow);
    } else {
      hipLaunchKernelGGL((pack_col_kernel<float, TP>), dim3(tx, ty), dim3(32, 8), 0, st, (const float*)A, lda, m, n,
                         ldc, (TP*)Acol);
      hipLaunchKernelGGL((pack_row_kernel<float, TP>), dim3(tx, ty), dim3(32, 8), 0, st, (const float*)A, lda, m, n,
                         row_off_d, rowblk_d, (TP*)Arow);
    }
    return hipGetLastError();
  });
}

hipError_t launch_finite_check(const void* A, int a_dtype, int64_t lda, int64_t m, int64_t n, int* bad,
                               hipStream_t st) {
  const unsigned gy = (unsigned)(m < 65535 ? m : 65535);
  const unsigned gx = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  if (a_dtype == 0)
    hipLaunchKernelGGL((finite_kernel<double>), dim3(gx, gy), dim3(256), 0, st, (const double*)A, lda, m, n, bad);
  else
    hipLaunchKernelGGL((finite_kernel<float>), dim3(gx, gy), dim3(256), 0, st, (const float*)A, lda, m, n, bad);
  return hipGetLastError();
}

hipError_t launch_block_weights(const void* Arow, const void* Acol, int panel_dtype, int64_t m, int64_t n, int64_t ldc,
                                const int64_t* row_off_d, int32_t s, const int64_t* col_off_d, int32_t t,
                                const int32_t* rowblk_d, double* row_sq, double* colrow_sq, double* w_row,
                                double* w_col, hipStream_t st) {
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const unsigned g1 = (unsigned)((m + 255) / 256 < 4096 ? (m + 255) / 256 : 4096);
    hipLaunchKernelGGL((row_sq_kernel<TP>), dim3(g1), dim3(256), 0, st, (const TP*)Arow, m, n, row_off_d, rowblk_d,
                       row_sq);
    const int64_t tot = m * (int64_t)t;
    const unsigned g2 = (unsigned)((tot + 255) / 256 < 8192 ? (tot + 255) / 256 : 8192);
    hipLaunchKernelGGL((colrow_sq_kernel<TP>), dim3(g2), dim3(256), 0, st, (const TP*)Acol, m, ldc, col_off_d, t, colrow_sq);
    hipLaunchKernelGGL(sum_rows_kernel, dim3((s + 63) / 64), dim3(64), 0, st, row_sq, row_off_d, s, w_row);
    hipLaunchKernelGGL(sum_cols_kernel, dim3((t + 63) / 64), dim3(64), 0, st, colrow_sq, m, t, w_col);
    return hipGetLastError();
  });
}

hipError_t launch_sample(const uint64_t* T_row, int32_t s, const uint64_t* T_col, int32_t t, uint64_t seed,
                         uint64_t sys, int64_t k0, int64_t count, int32_t* j_out, int32_t* i_out, hipStream_t st) {
  const unsigned g = (unsigned)((count + 255) / 256 < 4096 ? (count + 255) / 256 : 4096);
  hipLaunchKernelGGL(sample_kernel, dim3(g > 0 ? g : 1), dim3(256), 0, st, T_row, s, T_col, t, seed, sys, k0, count,
                     j_out, i_out);
  return hipGetLastError();
}

hipError_t launch_philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1, int64_t count,
                         uint64_t* out, hipStream_t st) {
  const unsigned g = (unsigned)((count + 255) / 256 < 4096 ? (count + 255) / 256 : 4096);
  hipLaunchKernelGGL(philox_kernel, dim3(g > 0 ? g : 1), dim3(256), 0, st, c0, c1, c2, c3, k0, k1, count, out);
  return hipGetLastError();
}

size_t wg_solve_lds_bytes(const SolveArgs& a) { return wg_lds_doubles(a) * sizeof(double); }

hipError_t launch_wg_solve(const SolveArgs& a, int panel_dtype, int threads, size_t lds_bytes, hipStream_t st) {
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    hipError_t e = hipFuncSetAttribute((const void*)wg_solve_kernel<TP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((wg_solve_kernel<TP>), dim3(1), dim3(threads), lds_bytes, st, a);
    return hipGetLastError();
  });
}

hipError_t launch_residual(const void* Arow, const void* Acol, int panel_dtype, const SolveArgs& a, const double* x,
                           const double* z, double* partials, int nparts, hipStream_t st) {
  (void)Arow;
  (void)Acol;
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    hipLaunchKernelGGL((residual_kernel<TP>), dim3(nparts), dim3(kWgThreads), 0, st, a, x, z, partials);
    return hipGetLastError();
  });
}

hipError_t launch_err2(const double* x, const double* x_ref, int64_t n, double* partials, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(err2_kernel, dim3(nparts), dim3(kWgThreads), 0, st, x, x_ref, n, partials);
  return hipGetLastError();
}

}  // namespace rebk
