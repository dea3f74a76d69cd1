// Device-side building blocks shared by the kernel translation units: panel element types,
// Philox4x64-10 and the block draw, workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rebk_internal.h"

namespace rebk {
namespace dev {

// ------------------------------------------------------------------ element types

template <int DT> struct PanelType;
template <> struct PanelType<0> { using T = double; };
template <> struct PanelType<1> { using T = float; };
template <> struct PanelType<2> { using T = __bf16; };
template <> struct PanelType<3> { using T = _Float16; };

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ double widen(float v) { return (double)v; }
__device__ __forceinline__ double widen(__bf16 v) { return (double)(float)v; }
__device__ __forceinline__ double widen(_Float16 v) { return (double)(float)v; }

template <typename T> __device__ __forceinline__ T narrow(double v) { return (T)v; }

// ------------------------------------------------------------------ Philox4x64-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): round
// function on four 64-bit words with two multipliers, Weyl-sequence key schedule, 10 rounds.

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3,
                                              uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = kPhiloxM0 * c0, hi0 = __umul64hi(kPhiloxM0, c0);
    const uint64_t lo1 = kPhiloxM1 * c2, hi1 = __umul64hi(kPhiloxM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
}

// First block whose cumulative threshold exceeds the top 53 bits of the word (thresholds are
// nondecreasing and the last one is 2^53, so the search always ends inside the table).
__device__ __forceinline__ int draw_block(const uint64_t* __restrict__ T, int nb, uint64_t word) {
  const uint64_t d = word >> 11;
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (d < T[mid]) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Blocks (j, i) of iteration k (1-based): counter (k-1, sys, 0, 0), key (seed, 0); word 0 draws
// the column block, word 1 the row block.
template <typename Args>
__device__ __forceinline__ void draw_pair(const Args& a, int64_t k, int& j, int& i) {
  uint64_t c0 = (uint64_t)(k - 1), c1 = a.sys, c2 = 0, c3 = 0;
  philox4x64_10(c0, c1, c2, c3, a.seed, 0);
  j = draw_block(a.T_col, a.t, c0);
  i = draw_block(a.T_row, a.s, c1);
}

// ------------------------------------------------------------------ workgroup-level helpers

// Sum of `val` over the workgroup; every thread receives the result.  red has blockDim.x slots.
__device__ __forceinline__ double wg_sum(double val, double* red) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) val += __shfl_down(val, o, 64);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = val;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int q = 0; q < nw; ++q) s += red[q];
  __syncthreads();
  return s;
}

// out[c] = sum_{r < rows} P[c * ld + r] * y[r] for c < w, P column-major (rows x w, column stride
// ld) in any memory, y in LDS.  Each column gets T / w consecutive threads (coalesced along r); partial sums
// meet in red (blockDim slots).  Columns beyond blockDim.x are processed in chunks.  Ends with a
// barrier.
template <typename TP>
__device__ __forceinline__ void colsum_colmajor(const TP* __restrict__ P, int64_t rows, int64_t ld, int w,
                                                const double* y, double* out, double* red) {
  const int T = blockDim.x, tid = threadIdx.x;
  for (int cb = 0; cb < w; cb += T) {
    const int cw = min(T, w - cb);
    const int gpc = T / cw;  // threads per column
    const int c = cb + tid / gpc, g = tid % gpc;
    double acc = 0.0;
    if (tid / gpc < cw) {
      const TP* col = P + (int64_t)c * ld;
      for (int64_t r = g; r < rows; r += gpc) acc += widen(col[r]) * y[r];
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < cw) {
      double s = 0.0;
      for (int q = 0; q < gpc; ++q) s += red[tid * gpc + q];
      out[cb + tid] = s;
    }
    __syncthreads();
  }
}

template <typename F>
hipError_t dispatch_panel(int dt, F&& f) {
  switch (dt) {
    case 0: return f(PanelType<0>{});
    case 1: return f(PanelType<1>{});
    case 2: return f(PanelType<2>{});
    case 3: return f(PanelType<3>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dev
}  // namespace rebk
