// Block constants beta = ||B||_2^2 / ||B||_F^2 of every row block A_{I_i,:} and column block
// A_{:,J_j} (Section 2.2, Remark 9: the stepsize alpha = 1 / beta_max, beta_max the largest of
// them, and 0 < alpha < 2 / beta_max guarantee convergence).
//
// ||B||_2^2 is the largest eigenvalue of the Gram matrix of B's shorter side (B B^T or B^T B, of
// order d = min(rows, cols)), ||B||_F^2 its trace.  Step 1 forms every Gram matrix in FP64 from
// the stored panel values (16 x 16 output tiles, the two strips staged in LDS).  Step 2 runs a
// power iteration per block, one workgroup each, with the Rayleigh quotient as the estimate: it
// approaches the largest eigenvalue from below, at a rate set by the ratio of the two largest.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rebk_device.h"
#include "rebk_internal.h"

namespace rebk {
namespace {

using namespace dev;

constexpr int kTile = 16;

// Gram of block g: G[a1][a2] = sum_{t < L} X(a1, t) X(a2, t), X(a, t) = P[base + a * sa + t * st].
template <typename TP>
__global__ void __launch_bounds__(256) gram_kernel(const TP* __restrict__ P, const GramDesc* __restrict__ desc,
                                                   const int32_t* __restrict__ tile_block,
                                                   const int32_t* __restrict__ tile_a1, const int32_t* __restrict__ tile_a2,
                                                   double* __restrict__ gram) {
  __shared__ double s1[kTile][kTile + 1], s2[kTile][kTile + 1];
  const int tileid = blockIdx.x;
  const GramDesc d = desc[tile_block[tileid]];
  const int a1_0 = tile_a1[tileid], a2_0 = tile_a2[tileid];
  const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
  double acc = 0.0;
  for (int64_t t0 = 0; t0 < d.L; t0 += kTile) {
    // s1[a][t] = X(a1_0 + a, t0 + t), s2[a][t] = X(a2_0 + a, t0 + t)
    {
      const int a = ty, t = tx;
      const int64_t tt = t0 + t;
      s1[a][t] = (a1_0 + a < d.d && tt < d.L) ? widen(P[d.base + (int64_t)(a1_0 + a) * d.sa + tt * d.st]) : 0.0;
      s2[a][t] = (a2_0 + a < d.d && tt < d.L) ? widen(P[d.base + (int64_t)(a2_0 + a) * d.sa + tt * d.st]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kTile; ++t) acc += s1[ty][t] * s2[tx][t];
    __syncthreads();
  }
  const int a1 = a1_0 + ty, a2 = a2_0 + tx;
  if (a1 < d.d && a2 < d.d) gram[d.gram + (int64_t)a1 * d.d + a2] = acc;
}

// Power iteration on Gram g (d x d, symmetric positive semidefinite), one workgroup per block.
// out[g] = the Rayleigh quotient after the last step, tr[g] = trace.  Stops when the quotient
// changes by at most rtol relative, or after max_steps.
__global__ void __launch_bounds__(256) power_kernel(const GramDesc* __restrict__ desc, const double* __restrict__ gram,
                                                    int max_steps, double rtol, double* __restrict__ out,
                                                    double* __restrict__ tr, int32_t* __restrict__ steps_out) {
  extern __shared__ double lds[];
  __shared__ double red[256];
  const GramDesc d = desc[blockIdx.x];
  const int D = d.d, tid = threadIdx.x, T = blockDim.x;
  const double* G = gram + d.gram;
  double* q = lds;      // current vector (unit norm)
  double* w = lds + D;  // G q
  // trace; starting vector: positive, deterministic, not symmetric in the index
  double t = 0.0;
  for (int a = tid; a < D; a += T) t += G[(int64_t)a * D + a];
  const double trace = wg_sum(t, red);
  double nq = 0.0;
  for (int a = tid; a < D; a += T) {
    q[a] = 1.0 + 0.5 * (double)((a * 2654435761u) >> 16 & 1023) / 1023.0;
    nq += q[a] * q[a];
  }
  nq = wg_sum(nq, red);
  for (int a = tid; a < D; a += T) q[a] /= sqrt(nq);
  __syncthreads();
  double lam = 0.0;
  int step = 0;
  for (; step < max_steps; ++step) {
    double qw = 0.0, ww = 0.0;
    for (int a = tid; a < D; a += T) {
      // (G q)_a = sum_b G[b][a] q_b (G is symmetric): consecutive threads read consecutive words
      double acc = 0.0;
#pragma unroll 8
      for (int b = 0; b < D; ++b) acc += G[(int64_t)b * D + a] * q[b];
      w[a] = acc;
      qw += q[a] * acc;
      ww += acc * acc;
    }
    qw = wg_sum(qw, red);
    ww = wg_sum(ww, red);
    const double prev = lam;
    lam = qw;  // q has unit norm
    if (!(ww > 0.0)) break;  // G q = 0: the block is zero
    const double inv = 1.0 / sqrt(ww);
    for (int a = tid; a < D; a += T) q[a] = w[a] * inv;
    __syncthreads();
    if (step > 0 && fabs(lam - prev) <= rtol * lam) {
      ++step;
      break;
    }
  }
  if (tid == 0) {
    out[blockIdx.x] = lam;
    tr[blockIdx.x] = trace;
    steps_out[blockIdx.x] = step;
  }
}

}  // namespace

hipError_t launch_gram(const void* P, int panel_dtype, const GramDesc* desc, int ntiles, const int32_t* tile_block,
                       const int32_t* tile_a1, const int32_t* tile_a2, double* gram, hipStream_t st) {
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    hipLaunchKernelGGL((gram_kernel<TP>), dim3(ntiles), dim3(kTile * kTile), 0, st, (const TP*)P, desc, tile_block,
                       tile_a1, tile_a2, gram);
    return hipGetLastError();
  });
}

hipError_t launch_power(const GramDesc* desc, int nblocks, int max_d, const double* gram, int max_steps, double rtol,
                        double* lam, double* trace, int32_t* steps, hipStream_t st) {
  const size_t lds = 2 * (size_t)max_d * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)power_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(power_kernel, dim3(nblocks), dim3(256), lds, st, desc, gram, max_steps, rtol, lam, trace, steps);
  return hipGetLastError();
}

}  // namespace rebk
