// Kernels of the learned warm start for REBK: a network b -> y (8192 -> 512 -> 512 -> 8192 in the
// benchmark) whose output gives the starting point x0 = A^T y, inside range(A^T) as Theorem 7 of
// Du, Si, Sun (arXiv:2001.04179) asks, and z0 = b - A x0, inside b + range(A).
//
// Training minimises (1 / 2 batch) sum ||A^T y - x_target||^2.  Every product is a GEMM on the
// matrix cores: half-precision operands, FP32 accumulation (v_mfma_f32_16x16x16_f16).  Weights
// have FP32 masters (Adam updates them) and half-precision copies for the products; the residual
// is scaled by a power of two before it is rounded to half precision, and the gradients are
// unscaled in FP32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rebk_device.h"
#include "rebk_internal.h"

namespace rebk {
namespace {

using namespace dev;

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;

// C (M x N, FP32, leading dimension ldc) = alpha * op(A) op(B) + beta * C, op(A) M x K and op(B)
// K x N from half-precision row-major storage:
//   TA = false: op(A)[i][k] = A[i * lda + k]    TA = true: op(A)[i][k] = A[k * lda + i]
//   TB = false: op(B)[k][j] = B[k * ldb + j]    TB = true: op(B)[k][j] = B[j * ldb + k]
// A workgroup (4 waves) computes a 64 x 64 tile of C; each wave a 32 x 32 sub-tile as 2 x 2
// MFMA 16 x 16 x 16 blocks.  The K loop stages 64 x 32 slices of op(A) and op(B)^T through LDS,
// loading along whichever index is contiguous in memory.  M, N multiples of 64, K of 32.
//
// MFMA 16x16x16 operand layout (lane l, 64 lanes): A block row l % 16, k = 4 (l / 16) .. +3;
// B block column l % 16, same k; the four results of lane l are rows 4 (l / 16) .. +3 of
// column l % 16.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_f16_kernel(int M, int N, int K, float alpha, const _Float16* __restrict__ A,
                                                       int lda, const _Float16* __restrict__ B, int ldb, float beta,
                                                       float* __restrict__ C, int ldc) {
  __shared__ _Float16 As[kBM][kBK + kPad];  // As[i][k] = op(A)[i0 + i][k0 + k]
  __shared__ _Float16 Bs[kBN][kBK + kPad];  // Bs[j][k] = op(B)[k0 + k][j0 + j]
  const int i0 = blockIdx.y * kBM, j0 = blockIdx.x * kBN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  const int lr = lane & 15, lk = 4 * (lane >> 4);
  for (int k0 = 0; k0 < K; k0 += kBK) {
#pragma unroll
    for (int e = tid; e < kBM * kBK; e += 256) {
      if (!TA) {
        const int i = e / kBK, k = e % kBK;
        As[i][k] = A[(size_t)(i0 + i) * lda + k0 + k];
      } else {
        const int k = e / kBM, i = e % kBM;
        As[i][k] = A[(size_t)(k0 + k) * lda + i0 + i];
      }
      if (TB) {
        const int j = e / kBK, k = e % kBK;
        Bs[j][k] = B[(size_t)(j0 + j) * ldb + k0 + k];
      } else {
        const int k = e / kBN, j = e % kBN;
        Bs[j][k] = B[(size_t)(k0 + k) * ldb + j0 + j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 16) {
      h4 av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const _Float16* p = &As[wi + a * 16 + lr][kk + lk];
        av[a] = h4{p[0], p[1], p[2], p[3]};
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const _Float16* p = &Bs[wj + b * 16 + lr][kk + lk];
        bv[b] = h4{p[0], p[1], p[2], p[3]};
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16f16(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wi + a * 16 + lk + r, col = j0 + wj + b * 16 + lr;
        float* c = C + (size_t)row * ldc + col;
        *c = beta == 0.f ? alpha * acc[a][b][r] : alpha * acc[a][b][r] + beta * *c;
      }
}

// out16[e] = half(scale * in[e]) from FP64 (the network's input, A) or FP32 (weights)
template <typename T>
__global__ void to_half_kernel(const T* __restrict__ in, int64_t count, double scale, _Float16* __restrict__ out16) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    out16[e] = (_Float16)(float)(scale * (double)in[e]);
}

// out = act(C + bias[col]) for a rows x cols FP32 matrix; act = relu or identity; writes the half
// copy (always) and an FP32 copy (if out32)
__global__ void bias_act_kernel(const float* __restrict__ C, const float* __restrict__ bias, int64_t rows, int cols,
                                int relu, _Float16* __restrict__ out16, float* __restrict__ out32) {
  const int64_t count = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    float v = C[e] + bias[e % cols];
    if (relu) v = v > 0.f ? v : 0.f;
    out16[e] = (_Float16)v;
    if (out32) out32[e] = v;
  }
}

// R = X0 - Xt (FP32); per-block partial sums of R^2 (FP64) and of max |R|
__global__ void residual_kernel(const float* __restrict__ X0, const double* __restrict__ Xt, int64_t count,
                                float* __restrict__ R, double* __restrict__ part_sq, float* __restrict__ part_max) {
  __shared__ double red[256];
  __shared__ float redm[256];
  double s = 0.0;
  float mx = 0.f;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)X0[e] - Xt[e];
    const float df = (float)d;
    R[e] = df;
    s += d * d;
    mx = fabsf(df) > mx ? fabsf(df) : mx;
  }
  const double tot = wg_sum(s, red);
  redm[threadIdx.x] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = 0.f;
    for (int q = 0; q < (int)blockDim.x; ++q) m = redm[q] > m ? redm[q] : m;
    part_sq[blockIdx.x] = tot;
    part_max[blockIdx.x] = m;
  }
}

// out16 = half(s * in) (the scaled residual)
__global__ void scale_half_kernel(const float* __restrict__ in, int64_t count, float s, _Float16* __restrict__ out16) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    out16[e] = (_Float16)(s * in[e]);
}

// out16 = half(D) where the activation H is positive, else 0 (back-propagation through relu)
__global__ void relu_back_kernel(const float* __restrict__ D, const _Float16* __restrict__ H, int64_t count,
                                 _Float16* __restrict__ out16) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    out16[e] = (float)H[e] > 0.f ? (_Float16)D[e] : (_Float16)0.f;
}

// out[c] = scale * sum over rows of D[r][c] (half input, rows in order): bias gradients
__global__ void colsum_half_kernel(const _Float16* __restrict__ D, int rows, int cols, float scale,
                                   float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += (float)D[(size_t)r * cols + c];
  out[c] = scale * s;
}

// Adam (Kingma and Ba, ICLR 2015) on one parameter array; writes the half copy (if p16).  omb1 and
// omb2 are 1 - beta1 and 1 - beta2 rounded from FP64 (1 - (float)beta2 would be off by about 1e-5
// relative for beta2 = 0.999, and the bias corrections c1, c2 are formed in FP64 too).
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t count, float lr, float b1, float omb1, float b2, float omb2,
                            float eps, float c1, float c2, _Float16* __restrict__ p16) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    const float ge = g[e];
    const float me = b1 * m[e] + omb1 * ge;
    const float ve = b2 * v[e] + omb2 * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float pe = p[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
    p[e] = pe;
    if (p16) p16[e] = (_Float16)pe;
  }
}

// Deterministic initial weights: uniform in (-bound, bound) from Philox4x64-10 (counter (e, tag),
// key (seed, 0), the top 53 bits of word 0)
__global__ void init_uniform_kernel(float* __restrict__ p, int64_t count, float bound, uint64_t seed, uint64_t tag) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t c0 = (uint64_t)e, c1 = tag, c2 = 0, c3 = 0;
    philox4x64_10(c0, c1, c2, c3, seed, 0);
    const double u = (double)(c0 >> 11) * (1.0 / 9007199254740992.0);
    p[e] = (float)((2.0 * u - 1.0) * bound);
  }
}

__global__ void widen_kernel(const float* __restrict__ in, int64_t count, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (double)in[e];
}

// C (M x N, FP64) = alpha * A (M x K) B (K x N), all FP64 row-major; 16 x 16 tiles, K in steps of
// 16 through LDS.  Forms x0 = out_scale A^T y exactly (to FP64 rounding) in range(A^T).
__global__ void __launch_bounds__(256) gemm_f64_kernel(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                       int lda, const double* __restrict__ B, int ldb,
                                                       double* __restrict__ C, int ldc) {
  __shared__ double As[16][17], Bs[16][17];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < K; k0 += 16) {
    As[ty][tx] = (row < M && k0 + tx < K) ? A[(size_t)row * lda + k0 + tx] : 0.0;
    Bs[ty][tx] = (k0 + ty < K && col < N) ? B[(size_t)(k0 + ty) * ldb + col] : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += As[ty][k] * Bs[k][tx];
    __syncthreads();
  }
  if (row < M && col < N) C[(size_t)row * ldc + col] = alpha * acc;
}

unsigned blocks_for(int64_t count) {
  const int64_t g = (count + 255) / 256;
  return (unsigned)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

}  // namespace

hipError_t launch_gemm_f16(bool ta, bool tb, int M, int N, int K, float alpha, const _Float16* A, int lda,
                           const _Float16* B, int ldb, float beta, float* C, int ldc, hipStream_t st) {
  if (M % kBM || N % kBN || K % kBK) return hipErrorInvalidValue;
  const dim3 grid(N / kBN, M / kBM);
  if (!ta && !tb) hipLaunchKernelGGL((gemm_f16_kernel<false, false>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  if (!ta && tb) hipLaunchKernelGGL((gemm_f16_kernel<false, true>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  if (ta && !tb) hipLaunchKernelGGL((gemm_f16_kernel<true, false>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  if (ta && tb) hipLaunchKernelGGL((gemm_f16_kernel<true, true>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  return hipGetLastError();
}

hipError_t launch_to_half_f64(const double* in, int64_t count, double scale, _Float16* out, hipStream_t st) {
  hipLaunchKernelGGL((to_half_kernel<double>), dim3(blocks_for(count)), dim3(256), 0, st, in, count, scale, out);
  return hipGetLastError();
}
hipError_t launch_to_half_f32(const float* in, int64_t count, _Float16* out, hipStream_t st) {
  hipLaunchKernelGGL((to_half_kernel<float>), dim3(blocks_for(count)), dim3(256), 0, st, in, count, 1.0, out);
  return hipGetLastError();
}
hipError_t launch_bias_act(const float* C, const float* bias, int64_t rows, int cols, int relu, _Float16* out16,
                           float* out32, hipStream_t st) {
  hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for(rows * cols)), dim3(256), 0, st, C, bias, rows, cols, relu,
                     out16, out32);
  return hipGetLastError();
}
hipError_t launch_mlp_residual(const float* X0, const double* Xt, int64_t count, float* R, double* part_sq,
                               float* part_max, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(residual_kernel, dim3(nparts), dim3(256), 0, st, X0, Xt, count, R, part_sq, part_max);
  return hipGetLastError();
}
hipError_t launch_scale_half(const float* in, int64_t count, float s, _Float16* out, hipStream_t st) {
  hipLaunchKernelGGL(scale_half_kernel, dim3(blocks_for(count)), dim3(256), 0, st, in, count, s, out);
  return hipGetLastError();
}
hipError_t launch_relu_back(const float* D, const _Float16* H, int64_t count, _Float16* out, hipStream_t st) {
  hipLaunchKernelGGL(relu_back_kernel, dim3(blocks_for(count)), dim3(256), 0, st, D, H, count, out);
  return hipGetLastError();
}
hipError_t launch_colsum_half(const _Float16* D, int rows, int cols, float scale, float* out, hipStream_t st) {
  hipLaunchKernelGGL(colsum_half_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, D, rows, cols, scale, out);
  return hipGetLastError();
}
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1, float omb1,
                       float b2, float omb2, float eps, float c1, float c2, _Float16* p16, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(count)), dim3(256), 0, st, p, g, m, v, count, lr, b1, omb1, b2, omb2,
                     eps, c1, c2, p16);
  return hipGetLastError();
}
hipError_t launch_init_uniform(float* p, int64_t count, float bound, uint64_t seed, uint64_t tag, hipStream_t st) {
  hipLaunchKernelGGL(init_uniform_kernel, dim3(blocks_for(count)), dim3(256), 0, st, p, count, bound, seed, tag);
  return hipGetLastError();
}
hipError_t launch_gemm_f64(int M, int N, int K, double alpha, const double* A, int lda, const double* B, int ldb,
                           double* C, int ldc, hipStream_t st) {
  hipLaunchKernelGGL(gemm_f64_kernel, dim3((N + 15) / 16, (M + 15) / 16), dim3(256), 0, st, M, N, K, alpha, A, lda, B,
                     ldb, C, ldc);
  return hipGetLastError();
}

hipError_t launch_widen(const float* in, int64_t count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(widen_kernel, dim3(blocks_for(count)), dim3(256), 0, st, in, count, out);
  return hipGetLastError();
}

}  // namespace rebk
