// HIP kernels for gfx950 (MI355X): panel packing, FP64 block weights, the counter-based block
// sampler, and the two REBK iteration kernels (Du, Si, Sun, arXiv:2001.04179, Algorithm 1).
//
// Cross-workgroup communication in the persistent grid kernel goes exclusively through
// device-scope atomic operations (relaxed loads, stores and FP64 adds), which are coherent
// across the eight XCDs without cache-maintenance fences; ordering between a workgroup's data
// atomics and its barrier arrival is enforced by waiting for their completion
// (s_waitcnt vmcnt(0)) before arriving.  On gfx950 an agent-scope release fence writes back the
// whole L2 of the XCD and costs several microseconds per workgroup, which is why it is avoided.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rebk_internal.h"

namespace rebk {
namespace {

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
__device__ __forceinline__ void draw_pair(const SolveArgs& a, int64_t k, int& j, int& i) {
  uint64_t c0 = (uint64_t)(k - 1), c1 = a.sys, c2 = 0, c3 = 0;
  philox4x64_10(c0, c1, c2, c3, a.seed, 0);
  j = draw_block(a.T_col, a.t, c0);
  i = draw_block(a.T_row, a.s, c1);
}

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

// Column panels: block j is m x nJ_j, row-major, at offset m * col_off[j].
template <typename TIn, typename TP>
__global__ void pack_col_kernel(const TIn* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                const int64_t* __restrict__ col_off, const int32_t* __restrict__ colblk,
                                TP* __restrict__ Acol) {
  for (int64_t r = blockIdx.y; r < m; r += gridDim.y) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
      const int j = colblk[c];
      const int64_t c0 = col_off[j], nJ = col_off[j + 1] - c0;
      Acol[m * c0 + r * nJ + (c - c0)] = narrow<TP>((double)A[r * lda + c]);
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
__global__ void colrow_sq_kernel(const TP* __restrict__ Acol, int64_t m, const int64_t* __restrict__ col_off, int t,
                                 double* __restrict__ colrow_sq) {
#pragma clang fp contract(off)
  const int64_t total = m * (int64_t)t;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / m, r = e - j * m;
    const int64_t c0 = col_off[j], nJ = col_off[j + 1] - c0;
    const TP* p = Acol + m * c0 + r * nJ;
    double acc = 0.0;
    for (int64_t c = 0; c < nJ; ++c) {
      const double v = widen(p[c]);
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

// out[c] = sum_{r < rows} P[r * w + c] * y[r] for c < w, P row-major (rows x w) in any memory,
// y in LDS.  Threads form T / w row groups per column; partial sums meet in red (blockDim slots).
// Columns beyond blockDim.x are processed in chunks.  Ends with a barrier.
template <typename TP>
__device__ __forceinline__ void colsum_rowmajor(const TP* __restrict__ P, int64_t rows, int w, const double* y,
                                                double* out, double* red) {
  const int T = blockDim.x, tid = threadIdx.x;
  for (int cb = 0; cb < w; cb += T) {
    const int cw = min(T, w - cb);
    const int ng = T / cw;
    const int g = tid / cw, c = cb + tid % cw;
    double acc = 0.0;
    if (g < ng)
      for (int64_t r = g; r < rows; r += ng) acc += widen(P[r * w + c]) * y[r];
    red[tid] = acc;
    __syncthreads();
    if (tid < cw) {
      double s = 0.0;
      for (int q = 0; q < ng; ++q) s += red[q * cw + tid];
      out[cb + tid] = s;
    }
    __syncthreads();
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
    const TP* __restrict__ P = Acol + m * c0;
    colsum_rowmajor(P, m, nJ, z, v, red);
    const double cc = a.coef_col[j];
    for (int64_t r = tid; r < m; r += T) {
      double acc = 0.0;
      for (int c = 0; c < nJ; ++c) acc += widen(P[r * nJ + c]) * v[c];
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

// ------------------------------------------------------------------ persistent grid solver
//
// Ownership: workgroup w owns rows [w*m/G, (w+1)*m/G) of z and columns [w*n/G, (w+1)*n/G) of x,
// both resident in LDS for the whole launch.  Per round one grid barrier separates:
//   round k:  x-update of iteration k-1 (needs u^{k-1}), z-update of iteration k (needs v^k),
//             partial sums of v^{k+1} = A_{:,J_{k+1}}^T z^k over owned rows, partial sums of
//             A_{I_k,:} x^{k-1} over owned columns plus (z^k - b) on owned rows of I_k, and the
//             partial error of x^{k-1}; all added into a striped accumulator with FP64 atomics.
// The z-chain never reads x, so running the x-chain one iteration behind is exact.  The slab of
// a column block is read from HBM once (for the partial sums) and kept in LDS for the next
// round's update; likewise for the row blocks.

constexpr unsigned kSpinLimit = 1u << 22;
constexpr int kLine = 32;  // unsigned words per 128-byte line

__device__ __forceinline__ unsigned ld_u32(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_u32(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_f64(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_f64(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_f64(double* p, double v) { unsafeAtomicAdd(p, v); }

// Wait until every memory operation this wave issued has completed (atomics performed at the
// device coherence point); the memory clobber keeps the compiler from moving accesses across.
__device__ __forceinline__ void wait_mem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Two-level counting barrier: workgroups arrive on one of `groups` counters; the last arrival of
// a group arrives on the root counter; the last root arrival writes the release flag of every
// group.  Counters grow monotonically within a launch (epoch = 1, 2, ...).  Returns false on a
// spin-limit timeout (then every workgroup leaves its loop).
__device__ bool grid_barrier(const GridSync& gs, unsigned epoch, int* s_ok) {
  wait_mem();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned G = gridDim.x, NG = (unsigned)gs.groups, g = blockIdx.x % NG;
    const unsigned gsize = (G - g + NG - 1) / NG;
    unsigned* root = gs.bar;
    unsigned* gcnt = gs.bar + kLine * (1 + g);
    unsigned* rel = gs.bar + kLine * (1 + NG + g);
    const unsigned old = __hip_atomic_fetch_add(gcnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == epoch * gsize - 1) {
      const unsigned o2 = __hip_atomic_fetch_add(root, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (o2 == epoch * NG - 1)
        for (unsigned q = 0; q < NG; ++q) st_u32(gs.bar + kLine * (1 + NG + q), epoch);
    }
    int ok = 1;
    unsigned spins = 0;
    while ((int)(ld_u32(rel) - epoch) < 0) {
      if ((++spins & 255u) == 0) {
        if (__hip_atomic_load(gs.timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
        if (spins > kSpinLimit) {
          __hip_atomic_store(gs.timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

struct GridLayout {
  int NR, NC;      // max rows / columns owned by one workgroup
  size_t dbl;      // doubles before the panel slabs
  size_t slabC;    // panel elements of one column slab buffer
  size_t slabR;    // panel elements of one row slab buffer
};

__host__ __device__ inline GridLayout grid_layout(int64_t m, int64_t n, int max_nI, int max_nJ, int G, int threads) {
  GridLayout L;
  L.NR = (int)((m + G - 1) / G);
  L.NC = (int)((n + G - 1) / G);
  L.dbl = 2 * (size_t)L.NR + (size_t)L.NC + (size_t)max_nJ + (size_t)max_nI + (size_t)threads + 8;
  L.slabC = (size_t)L.NR * max_nJ;
  L.slabR = (size_t)L.NC * max_nI;
  return L;
}

template <typename TP>
__global__ void __launch_bounds__(kGridThreads) grid_solve_kernel(SolveArgs a, GridSync gs) {
  extern __shared__ double lds[];
  __shared__ int s_j[128], s_i[128];
  __shared__ int s_ok;
  __shared__ double s_err2;
  const int G = gridDim.x, w = blockIdx.x, tid = threadIdx.x, T = blockDim.x;
  const int64_t m = a.m, n = a.n;
  const int MJ = a.max_nJ, MI = a.max_nI;
  const GridLayout L = grid_layout(m, n, MI, MJ, G, T);
  const int64_t r0 = (int64_t)w * m / G, r1 = (int64_t)(w + 1) * m / G;
  const int64_t cA = (int64_t)w * n / G, cB = (int64_t)(w + 1) * n / G;
  const int nr = (int)(r1 - r0), nc = (int)(cB - cA);

  double* z = lds;
  double* zp = z + L.NR;
  double* x = zp + L.NR;
  double* v = x + L.NC;
  double* u = v + MJ;
  double* red = u + MI;
  TP* slabC = (TP*)(lds + L.dbl);
  TP* slabR = slabC + 2 * L.slabC;

  const TP* __restrict__ Arow = (const TP*)a.Arow;
  const TP* __restrict__ Acol = (const TP*)a.Acol;
  const int S = gs.stripes, E = gs.stride;
  const int my_stripe = w % S;
  const size_t bufsz = (size_t)S * E;
  const int64_t K = a.max_iter;
  const int64_t ce = a.check_every > 0 ? a.check_every : 1;
  const bool checking = a.x_ref != nullptr && a.tol > 0.0;
  const int err_slot = MJ + MI;

  // resident state
  for (int rr = tid; rr < nr; rr += T) z[rr] = a.z_in ? a.z_in[r0 + rr] : a.b[r0 + rr];
  for (int cc = tid; cc < nc; cc += T) x[cc] = a.x_in ? a.x_in[cA + cc] : 0.0;

  // block draws: relative iteration q (1-based) lives in ring slot (q - 1) & 127; refilled 64 at a time
  auto refill = [&](int64_t qfirst) {  // draws for relative iterations qfirst .. qfirst+63
    if (tid < 64) {
      const int64_t q = qfirst + tid;
      if (q <= K) {
        int jj, ii;
        draw_pair(a, a.k0 + q, jj, ii);
        s_j[(q - 1) & 127] = jj;
        s_i[(q - 1) & 127] = ii;
      }
    }
  };
  refill(1);
  refill(65);
  __syncthreads();
  int64_t filled_to = 128;  // draws available for q <= filled_to

  auto stage_col = [&](int j, int buf) -> int {  // slab of column block j over owned rows
    const int64_t c0 = a.col_off[j];
    const int nJ = (int)(a.col_off[j + 1] - c0);
    const TP* src = Acol + m * c0 + r0 * nJ;
    TP* dst = slabC + (size_t)buf * L.slabC;
    const int len = nr * nJ;
    for (int e = tid; e < len; e += T) dst[e] = src[e];
    return nJ;
  };
  auto stage_row = [&](int i, int buf) -> int {  // slab of row block i over owned columns
    const int64_t rI = a.row_off[i];
    const int nI = (int)(a.row_off[i + 1] - rI);
    const TP* src = Arow + n * rI + cA * nI;
    TP* dst = slabR + (size_t)buf * L.slabR;
    const int len = nc * nI;
    for (int e = tid; e < len; e += T) dst[e] = src[e];
    return nI;
  };
  auto accbuf = [&](int64_t rr) -> double* { return gs.acc + (size_t)(rr % 3) * bufsz; };

  // partial of A_{:,J}^T z over owned rows (slab in buffer `buf`) -> accumulator
  auto push_q = [&](int nJ, int buf, double* dst) {
    const TP* Sl = slabC + (size_t)buf * L.slabC;
    colsum_rowmajor(Sl, nr, nJ, z, v, red);  // v used as scratch here; it is re-read after the barrier
    for (int c = tid; c < nJ; c += T) add_f64(dst + c, v[c]);
  };

  unsigned epoch = 0;
  int status = 0, stopped = 0;
  int64_t last_k = a.k0;
  double last_err2 = -1.0;
  int64_t last_check = -1;
  bool alive = true;

  // ---------------- prologue: partial sums of v^1 = A_{:,J_1}^T z^0
  {
    __syncthreads();
    const int j1 = s_j[0];
    const int nJ = stage_col(j1, 0);
    __syncthreads();
    push_q(nJ, 0, accbuf(0) + (size_t)my_stripe * E);
    alive = grid_barrier(gs, ++epoch, &s_ok);
  }

  int64_t rr = 1;
  for (; alive && rr <= K; ++rr) {
    const int64_t k = a.k0 + rr;
    if (rr + 32 > filled_to && filled_to < K) {  // keep >= 32 draws ahead
      __syncthreads();
      refill(filled_to + 1);
      filled_to += 64;
      __syncthreads();
    }
    const int jk = s_j[(rr - 1) & 127], ik = s_i[(rr - 1) & 127];
    const int jn = rr < K ? s_j[rr & 127] : 0;
    const int ip = rr >= 2 ? s_i[(rr - 2) & 127] : 0;
    const int nJk = (int)(a.col_off[jk + 1] - a.col_off[jk]);
    const int nIp = (int)(a.row_off[ip + 1] - a.row_off[ip]);
    if (w == 0 && tid == 0 && a.trace_j) {
      a.trace_j[rr - 1] = jk;
      a.trace_i[rr - 1] = ik;
    }

    // A. reduced values of the previous round
    {
      const double* src = accbuf(rr - 1);
      for (int e = tid; e < E; e += T) {
        const bool want = (e < nJk) || (rr >= 2 && e >= MJ && e < MJ + nIp) || (e == err_slot);
        if (!want) continue;
        double sum = 0.0;
        for (int q = 0; q < S; ++q) sum += ld_f64(src + (size_t)q * E + e);
        if (e < MJ) v[e] = sum;
        else if (e < MJ + MI) u[e - MJ] = sum;
        else s_err2 = sum;
      }
      __syncthreads();
    }

    // B. stop rule on x^{k-2} (its error was summed in the previous round)
    if (checking && rr >= 3 && ((rr - 2) % ce == 0)) {
      const double e2 = s_err2;
      last_err2 = e2;
      last_check = k - 2;
      const double rel = sqrt(e2) / sqrt(a.xref_sq);
      if (rel < a.tol || !isfinite(e2) || rel > 1e6) {
        stopped = 1;
        status = (rel < a.tol) ? 0 : 2;
        last_k = k - 2;
        for (int q = tid; q < nr; q += T) z[q] = zp[q];  // z^{k-2}
        __syncthreads();
        break;
      }
    }

    // C. x^{k-1} = x^{k-2} - coef_{i_{k-1}} A_{I,C}^T u^{k-1} on owned columns
    if (rr >= 2 && nc > 0) {
      const TP* Sl = slabR + (size_t)((rr - 1) & 1) * L.slabR;  // (c, l) at c * nIp + l
      const double cr = a.coef_row[ip];
      // columns x row-groups mapping
      const int ng = T / nc;
      const int g = tid / nc, cc = tid % nc;
      double acc = 0.0;
      if (g < ng)
        for (int l = g; l < nIp; l += ng) acc += widen(Sl[cc * nIp + l]) * u[l];
      red[tid] = acc;
      __syncthreads();
      if (tid < nc) {
        double s2 = 0.0;
        for (int q = 0; q < ng; ++q) s2 += red[q * nc + tid];
        x[tid] -= cr * s2;
      }
      __syncthreads();
    }

    // D. z^k = z^{k-1} - coef_{j_k} A_{R,J_k} v^k on owned rows (slab staged last round)
    {
      const TP* Sl = slabC + (size_t)((rr - 1) & 1) * L.slabC;
      const double cc = a.coef_col[jk];
      for (int q = tid; q < nr; q += T) {
        double acc = 0.0;
        for (int c = 0; c < nJk; ++c) acc += widen(Sl[q * nJk + c]) * v[c];
        zp[q] = z[q];
        z[q] -= cc * acc;
      }
      __syncthreads();
    }

    double* dst = accbuf(rr) + (size_t)my_stripe * E;
    // E. partial sums of v^{k+1} = A_{:,J_{k+1}}^T z^k
    if (rr < K) {
      const int nJn = stage_col(jn, rr & 1);
      __syncthreads();
      push_q(nJn, rr & 1, dst);
    }

    // F. partial sums of u^k = A_{I_k,:} x^{k-1} - b_{I_k} + z^k_{I_k}
    {
      const int nI = stage_row(ik, rr & 1);
      __syncthreads();
      if (nc > 0) {
        const TP* Sl = slabR + (size_t)(rr & 1) * L.slabR;
        for (int l = tid; l < nI; l += T) {
          double acc = 0.0;
          for (int cc = 0; cc < nc; ++cc) acc += widen(Sl[cc * nI + l]) * x[cc];
          add_f64(dst + MJ + l, acc);
        }
      }
      const int64_t rI = a.row_off[ik];
      const int64_t lo = rI > r0 ? rI : r0, hi = (rI + nI) < r1 ? (rI + nI) : r1;
      for (int64_t l = lo + tid; l < hi; l += T) add_f64(dst + MJ + (l - rI), z[l - r0] - a.b[l]);
    }

    // G. partial error of x^{k-1}
    if (checking && rr >= 2 && ((rr - 1) % ce == 0)) {
      double e = 0.0;
      for (int cc = tid; cc < nc; cc += T) {
        const double d = x[cc] - a.x_ref[cA + cc];
        e += d * d;
      }
      const double tot = wg_sum(e, red);
      if (tid == 0 && nc > 0) add_f64(dst + err_slot, tot);
    }

    // H. clear the accumulator of the next round, then the grid barrier
    {
      double* nb = accbuf(rr + 1);
      const size_t lo = (size_t)w * bufsz / G, hi = (size_t)(w + 1) * bufsz / G;
      for (size_t e = lo + tid; e < hi; e += T) st_f64(nb + e, 0.0);
    }
    alive = grid_barrier(gs, ++epoch, &s_ok);
  }

  if (alive && !stopped) {
    // epilogue: u^K from the last round, x^K, and the error of x^K
    const int ip = s_i[(K - 1) & 127];
    const int nIp = (int)(a.row_off[ip + 1] - a.row_off[ip]);
    {
      const double* src = accbuf(K);
      for (int e = tid; e < E; e += T) {
        const bool want = (e >= MJ && e < MJ + nIp) || (e == err_slot);
        if (!want) continue;
        double sum = 0.0;
        for (int q = 0; q < S; ++q) sum += ld_f64(src + (size_t)q * E + e);
        if (e < MJ + MI) u[e - MJ] = sum;
        else s_err2 = sum;
      }
      __syncthreads();
    }
    bool done = false;
    if (checking && K >= 2 && ((K - 1) % ce == 0)) {
      const double e2 = s_err2;
      last_err2 = e2;
      last_check = a.k0 + K - 1;
      const double rel = sqrt(e2) / sqrt(a.xref_sq);
      if (rel < a.tol || !isfinite(e2) || rel > 1e6) {
        stopped = 1;
        status = (rel < a.tol) ? 0 : 2;
        last_k = a.k0 + K - 1;
        for (int q = tid; q < nr; q += T) z[q] = zp[q];
        __syncthreads();
        done = true;
      }
    }
    if (!done) {
      if (nc > 0) {
        const TP* Sl = slabR + (size_t)(K & 1) * L.slabR;
        const double cr = a.coef_row[ip];
        const int ng = T / nc;
        const int g = tid / nc, cc = tid % nc;
        double acc = 0.0;
        if (g < ng)
          for (int l = g; l < nIp; l += ng) acc += widen(Sl[cc * nIp + l]) * u[l];
        red[tid] = acc;
        __syncthreads();
        if (tid < nc) {
          double s2 = 0.0;
          for (int q = 0; q < ng; ++q) s2 += red[q * nc + tid];
          x[tid] -= cr * s2;
        }
        __syncthreads();
      }
      last_k = a.k0 + K;
      if (a.x_ref != nullptr) {
        double e = 0.0;
        for (int cc = tid; cc < nc; cc += T) {
          const double d = x[cc] - a.x_ref[cA + cc];
          e += d * d;
        }
        const double tot = wg_sum(e, red);
        double* dst = accbuf(K + 1) + (size_t)my_stripe * E;
        if (tid == 0 && nc > 0) add_f64(dst + err_slot, tot);
        alive = grid_barrier(gs, ++epoch, &s_ok);
        if (alive) {
          if (tid == 0) {
            double sum = 0.0;
            for (int q = 0; q < S; ++q) sum += ld_f64(accbuf(K + 1) + (size_t)q * E + err_slot);
            s_err2 = sum;
          }
          __syncthreads();
          last_err2 = s_err2;
          last_check = a.k0 + K;
          if (checking) {
            const double rel = sqrt(last_err2) / sqrt(a.xref_sq);
            if (rel < a.tol) { stopped = 1; status = 0; }
            else if (!isfinite(last_err2) || rel > 1e6) { stopped = 1; status = 2; }
            else status = 1;
          }
        }
      }
    }
  }

  for (int q = tid; q < nr; q += T)
    if (a.z_out) a.z_out[r0 + q] = z[q];
  for (int q = tid; q < nc; q += T) a.x_out[cA + q] = x[q];
  if (w == 0 && tid == 0) {
    a.status->status = alive ? status : -4;
    a.status->stopped = stopped;
    a.status->last_k = last_k;
    a.status->err2 = last_err2;
    a.status->check_k = last_check;
  }
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
  // columns of A^T z through the column panels: entry (r, c) at m*c0 + r*nJ + (c - c0)
  for (int64_t c = (int64_t)blk * blockDim.x + tid; c < n; c += (int64_t)nb * blockDim.x) {
    int lo = 0, hi = a.t - 1;
    while (lo < hi) { const int mid = (lo + hi + 1) >> 1; if (a.col_off[mid] <= c) lo = mid; else hi = mid - 1; }
    const int64_t c0 = a.col_off[lo], nJ = a.col_off[lo + 1] - c0;
    const TP* p = Acol + m * c0 + (c - c0);
    double acc = 0.0;
    for (int64_t r = 0; r < m; ++r) acc += widen(p[r * nJ]) * z[r];
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

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_pack(const void* A, int a_dtype, int64_t lda, int panel_dtype, int64_t m, int64_t n,
                       const int64_t* row_off_d, const int64_t* col_off_d, const int32_t* rowblk_d,
                       const int32_t* colblk_d, void* Arow, void* Acol, hipStream_t st) {
  return dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const unsigned gy = (unsigned)(m < 65535 ? m : 65535);
    const unsigned gx = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    const unsigned ty = (unsigned)((m + 31) / 32 < 65535 ? (m + 31) / 32 : 65535);
    const unsigned tx = (unsigned)((n + 31) / 32 < 65535 ? (n + 31) / 32 : 65535);
    if (a_dtype == 0) {
      hipLaunchKernelGGL((pack_col_kernel<double, TP>), dim3(gx, gy), dim3(256), 0, st, (const double*)A, lda, m, n,
                         col_off_d, colblk_d, (TP*)Acol);
      hipLaunchKernelGGL((pack_row_kernel<double, TP>), dim3(tx, ty), dim3(32, 8), 0, st, (const double*)A, lda, m, n,
                         row_off_d, rowblk_d, (TP*)Arow);
    } else {
      hipLaunchKernelGGL((pack_col_kernel<float, TP>), dim3(gx, gy), dim3(256), 0, st, (const float*)A, lda, m, n,
                         col_off_d, colblk_d, (TP*)Acol);
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

hipError_t launch_block_weights(const void* Arow, const void* Acol, int panel_dtype, int64_t m, int64_t n,
                                const int64_t* row_off_d, int32_t s, const int64_t* col_off_d, int32_t t,
                                const int32_t* rowblk_d, double* row_sq, double* colrow_sq, double* w_row,
                                double* w_col, hipStream_t st) {
  return dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const unsigned g1 = (unsigned)((m + 255) / 256 < 4096 ? (m + 255) / 256 : 4096);
    hipLaunchKernelGGL((row_sq_kernel<TP>), dim3(g1), dim3(256), 0, st, (const TP*)Arow, m, n, row_off_d, rowblk_d,
                       row_sq);
    const int64_t tot = m * (int64_t)t;
    const unsigned g2 = (unsigned)((tot + 255) / 256 < 8192 ? (tot + 255) / 256 : 8192);
    hipLaunchKernelGGL((colrow_sq_kernel<TP>), dim3(g2), dim3(256), 0, st, (const TP*)Acol, m, col_off_d, t, colrow_sq);
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
  return dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    hipError_t e = hipFuncSetAttribute((const void*)wg_solve_kernel<TP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((wg_solve_kernel<TP>), dim3(1), dim3(threads), lds_bytes, st, a);
    return hipGetLastError();
  });
}

size_t grid_solve_lds_bytes(const SolveArgs& a, int grid, int panel_dtype) {
  const GridLayout L = grid_layout(a.m, a.n, a.max_nI, a.max_nJ, grid, kGridThreads);
  const size_t esz = panel_dtype == 0 ? 8 : (panel_dtype == 1 ? 4 : 2);
  return L.dbl * sizeof(double) + 2 * (L.slabC + L.slabR) * esz + 64;
}

hipError_t grid_solve_max_blocks(int panel_dtype, size_t lds_bytes, int* blocks_per_cu) {
  return dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    hipError_t e = hipFuncSetAttribute((const void*)grid_solve_kernel<TP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds_bytes);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)grid_solve_kernel<TP>, kGridThreads,
                                                        lds_bytes);
  });
}

hipError_t launch_grid_solve(const SolveArgs& a, const GridSync& gs, int panel_dtype, int grid, hipStream_t st) {
  return dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const size_t lds = grid_solve_lds_bytes(a, grid, panel_dtype);
    hipError_t e = hipFuncSetAttribute((const void*)grid_solve_kernel<TP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    SolveArgs aa = a;
    GridSync gg = gs;
    void* args[] = {&aa, &gg};
    return hipLaunchCooperativeKernel((const void*)grid_solve_kernel<TP>, dim3(grid), dim3(kGridThreads), args,
                                      (unsigned)lds, st);
  });
}

hipError_t launch_residual(const void* Arow, const void* Acol, int panel_dtype, const SolveArgs& a, const double* x,
                           const double* z, double* partials, int nparts, hipStream_t st) {
  (void)Arow;
  (void)Acol;
  return dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
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
