// Batched REBK for gfx950: many independent systems, many right-hand sides, one launch
// (Du, Si, Sun, arXiv:2001.04179, Algorithm 1 applied to each system and right-hand side).
//
// Every workgroup runs one task: R right-hand sides of one system, from start to stop.  All
// right-hand sides of a system share its block sequence (the Philox counter carries the system
// id, not the right-hand side), so one read of a panel element feeds R accumulators: the block
// products become small GEMMs, A_{:,J}^T Z and A_{I,:} X with R columns.  The iterates Z (m x R)
// and X (n x R) stay in LDS for the whole task, stored right-hand side after right-hand side so
// that consecutive lanes touch consecutive words.  The host orders the tasks so that the tasks of
// one system are dispatched to the same XCD (workgroup b goes to XCD b mod 8); they walk the same
// panels at about the same pace and share them through that XCD's L2.
//
// The iterates are FP64 and the panels any of FP64/FP32/BF16/FP16, widened exactly.  The
// contractions run as FP64 FMAs on the vector units: on this chip FP64 matrix cores have the same
// peak as the vector units, and a narrower type for the iterates would not reach the tolerances
// the method is run to.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rebk_device.h"
#include "rebk_internal.h"

namespace rebk {
namespace {

using namespace dev;

template <int CTRL>
__device__ __forceinline__ double bdpp(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false));
}
// Sum over aligned groups of `width` lanes (power of two <= 64); every lane of a group gets the
// group's sum.  All 64 lanes must execute it.
__device__ __forceinline__ double lane_group_sum(double v, int width) {
  if (width >= 2) v += bdpp<0xB1>(v);    // quad_perm [1,0,3,2]
  if (width >= 4) v += bdpp<0x4E>(v);    // quad_perm [2,3,0,1]
  if (width >= 8) v += bdpp<0x141>(v);   // row_half_mirror
  if (width >= 16) v += bdpp<0x140>(v);  // row_mirror
  if (width >= 32) v += __shfl_xor(v, 16, 64);
  if (width >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Pointers read from the task table are generic; the compiler would access them with flat
// instructions, which also count on the LDS wait counter, so every LDS read of the iterates would
// wait for all panel loads in flight.  These casts state that they point to global memory.
#define GLOBAL_AS __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const GLOBAL_AS T* gptr(const T* p) {
  return (const GLOBAL_AS T*)p;
}
template <typename T>
__device__ __forceinline__ GLOBAL_AS T* gptr(T* p) {
  return (GLOBAL_AS T*)p;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Four consecutive panel entries (a chunk aligned to 4 entries) held in their stored type until
// they are used, so a thread can keep many chunks in flight: one 16-byte load for FP32, two for
// FP64, one 8-byte load for the 2-byte types.  get(i) widens entry i exactly to FP64.
template <typename TP>
struct Chunk4;
template <>
struct Chunk4<float> {
  f32x4 v;
  __device__ __forceinline__ void load(const GLOBAL_AS float* p) { v = *(const GLOBAL_AS f32x4*)p; }
  __device__ __forceinline__ double get(int i) const { return (double)v[i]; }
};
template <>
struct Chunk4<double> {
  f64x2 a, b;
  __device__ __forceinline__ void load(const GLOBAL_AS double* p) {
    a = *(const GLOBAL_AS f64x2*)p;
    b = *(const GLOBAL_AS f64x2*)(p + 2);
  }
  __device__ __forceinline__ double get(int i) const { return i < 2 ? a[i] : b[i - 2]; }
};
template <>
struct Chunk4<__bf16> {
  u32x2 v;  // entry 0 in the low half of the first word
  __device__ __forceinline__ void load(const GLOBAL_AS __bf16* p) { v = *(const GLOBAL_AS u32x2*)p; }
  __device__ __forceinline__ double get(int i) const {
    const unsigned w = v[i >> 1];
    return (double)__uint_as_float((i & 1) ? (w & 0xffff0000u) : (w << 16));
  }
};
template <>
struct Chunk4<_Float16> {
  u32x2 v;
  __device__ __forceinline__ void load(const GLOBAL_AS _Float16* p) { v = *(const GLOBAL_AS u32x2*)p; }
  __device__ __forceinline__ double get(int i) const {
    const unsigned w = v[i >> 1];
    return (double)(float)__builtin_bit_cast(_Float16, (unsigned short)((i & 1) ? (w >> 16) : (w & 0xffffu)));
  }
};

__device__ __forceinline__ int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

constexpr int kDrawBatch = 64;  // block draws computed at a time
// panel loads a thread issues before it consumes them (one entry each): a task's passes over a
// panel are chains of such groups, so the number in flight sets the streaming rate of the CU.
// With 1024 threads a wave has half the registers (and the CU twice the threads): half as many.
template <int R, int kThreads>
constexpr int unroll_for() { return (R >= 4 ? 16 : 8) / (kThreads >= 1024 ? 2 : 1); }
// 4-entry vector loads in flight: phases whose accumulators are R values per lane, and phases
// that keep 4 R accumulators (four rows at once)
template <int R, int kThreads>
constexpr int vec_unroll_light() { return (R >= 2 ? 8 : 16) / (kThreads >= 1024 ? 2 : 1); }
template <int R, int kThreads>
constexpr int vec_unroll_heavy() { return (R >= 2 ? 4 : 8) / (kThreads >= 1024 ? 2 : 1); }

struct BatchLayout {
  size_t z, x, v, u, ew, total;  // offsets in doubles
};

__host__ __device__ inline BatchLayout batch_layout(int64_t m, int64_t n, int R, int max_nJ, int max_nI,
                                                    int threads) {
  BatchLayout L;
  L.z = 0;
  L.x = L.z + (size_t)R * m;
  L.v = L.x + (size_t)R * n;
  L.u = L.v + (size_t)R * max_nJ;
  L.ew = L.u + (size_t)R * max_nI;
  L.total = L.ew + 2 * (size_t)R * ((threads + 63) / 64) + 2 * (size_t)R;
  return L;
}

template <typename TP, int R, int kThreads>
__device__ void run_task(const BatchSys& S, const BatchTask& tk, const BatchArgs& a, double* lds, int* s_j,
                         int* s_i) {
  const int T = blockDim.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = (T + 63) >> 6;
  const int64_t m = S.m, n = S.n;
  const BatchLayout L = batch_layout(m, n, R, a.max_nJ, a.max_nI, T);
  double* z = lds + L.z;    // z[k * m + r]
  double* x = lds + L.x;    // x[k * n + c]
  double* v = lds + L.v;    // v[k * max_nJ + c]
  double* u = lds + L.u;    // u[k * max_nI + l]
  double* ew = lds + L.ew;  // per-wave partial errors, then R totals and R reference norms
  double* etot = ew + 2 * (size_t)R * nw;
  double* xr2 = etot + R;
  const int MJ = a.max_nJ, MI = a.max_nI;
  const GLOBAL_AS TP* __restrict__ Arow = gptr((const TP*)S.Arow);
  const GLOBAL_AS TP* __restrict__ Acol = gptr((const TP*)S.Acol);
  const GLOBAL_AS int64_t* __restrict__ col_off = gptr(S.col_off);
  const GLOBAL_AS int64_t* __restrict__ row_off = gptr(S.row_off);
  const GLOBAL_AS double* __restrict__ coef_col = gptr(S.coef_col);
  const GLOBAL_AS double* __restrict__ coef_row = gptr(S.coef_row);
  const GLOBAL_AS double* __restrict__ bvec = gptr(tk.b);
  const GLOBAL_AS double* __restrict__ xref = gptr(tk.x_ref);
  constexpr int kUnroll = unroll_for<R, kThreads>();

  for (int64_t e = tid; e < (int64_t)R * m; e += T) z[e] = bvec[e];
  if (tk.x_in) {
    const GLOBAL_AS double* x0 = gptr(tk.x_in);
    for (int64_t e = tid; e < (int64_t)R * n; e += T) x[e] = x0[e];
  } else {
    for (int64_t e = tid; e < (int64_t)R * n; e += T) x[e] = 0.0;
  }

  if (a.z0_from_x0 && tk.x_in) {
    // z0 = b - A x0 (a start in b + range(A), as Theorem 7 asks), one thread per row, from the
    // row panels: row l of block i at n * r0_i + c * nI_i + (l - r0_i)
    __syncthreads();
    for (int64_t l = tid; l < m; l += T) {
      int lo = 0, hi = S.s - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_off[mid] <= l) lo = mid; else hi = mid - 1;
      }
      const int64_t rb = row_off[lo], nb = row_off[lo + 1] - rb;
      const GLOBAL_AS TP* p = Arow + n * rb + (l - rb);
      double acc[R];
#pragma unroll
      for (int k = 0; k < R; ++k) acc[k] = 0.0;
      for (int64_t c = 0; c < n; ++c) {
        const double av = widen(p[c * nb]);
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] += av * x[k * n + c];
      }
#pragma unroll
      for (int k = 0; k < R; ++k) z[k * m + l] = bvec[k * m + l] - acc[k];
    }
    __syncthreads();
    // fallback: a start with ||b - A x0|| >= ||b|| is no better than x0 = 0; use x0 = 0, z0 = b
    double zz[R], bb[R];
#pragma unroll
    for (int k = 0; k < R; ++k) zz[k] = bb[k] = 0.0;
    for (int64_t l = tid; l < m; l += T) {
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const double zv = z[k * m + l], bv = bvec[k * m + l];
        zz[k] += zv * zv;
        bb[k] += bv * bv;
      }
    }
    double* scratch = lds + L.ew;  // 2 R per wave (the error scratch is not in use yet)
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const double s1 = lane_group_sum(zz[k], 64), s2 = lane_group_sum(bb[k], 64);
      if (lane == 0) {
        scratch[(wid * R + k) * 2] = s1;
        scratch[(wid * R + k) * 2 + 1] = s2;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < R; ++k) {
      double tz = 0.0, tb = 0.0;
      for (int q = 0; q < nw; ++q) {
        tz += scratch[(q * R + k) * 2];
        tb += scratch[(q * R + k) * 2 + 1];
      }
      if (!(tz < tb)) {  // uniform across the workgroup
        for (int64_t c = tid; c < n; c += T) x[k * n + c] = 0.0;
        for (int64_t l = tid; l < m; l += T) z[k * m + l] = bvec[k * m + l];
      }
    }
    __syncthreads();
  }
  const bool checking = tk.x_ref != nullptr;
  const bool stopping = checking && a.tol > 0.0;
  const int64_t ce = a.check_every > 0 ? a.check_every : 1;

  // Per right-hand side sum over c < n of f(k, c), reduced in a fixed order; results in out[k].
  auto colwise_sum = [&](auto f, double* out) {
    double acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = 0.0;
    for (int64_t c = tid; c < n; c += T) {
#pragma unroll
      for (int k = 0; k < R; ++k) acc[k] += f(k, c);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const double s = lane_group_sum(acc[k], 64);
      if (lane == 0) ew[wid * R + k] = s;
    }
    __syncthreads();
    if (tid < R) {
      double s = 0.0;
      for (int q = 0; q < nw; ++q) s += ew[q * R + tid];
      out[tid] = s;
    }
    __syncthreads();
  };
  if (checking) {
    colwise_sum([&](int k, int64_t c) { const double r = xref[k * n + c]; return r * r; }, xr2);
    if (tid < R) tk.xref2_out[tid] = xr2[tid];
  }

  int status = 1;
  int64_t done = 0;
  for (int64_t q = 0; q < a.max_iter; ++q) {
    const int64_t k1 = q + 1;  // 1-based iteration number
    if ((q % kDrawBatch) == 0) {
      __syncthreads();
      if (tid < kDrawBatch && q + tid < a.max_iter) {
        int jj, ii;
        draw_pair(S, k1 + tid, jj, ii);
        s_j[tid] = jj;
        s_i[tid] = ii;
      }
      __syncthreads();
    }
    const int j = s_j[q % kDrawBatch], i = s_i[q % kDrawBatch];

    // ---- z-phase: V = A_{:,J}^T Z (nJ x R).  Column runs start at multiples of 16 entries and
    // are zero-padded to ldc, so every lane reads whole aligned 4-row chunks: G lanes per column,
    // chunks g, g + G, ...; rows past m hold 0 in the panel and read a valid z row.
    const int64_t c0 = col_off[j];
    const int nJ = (int)(col_off[j + 1] - c0);
    const int64_t ldc = S.ldc;
    const GLOBAL_AS TP* __restrict__ P = Acol + ldc * c0;  // (r, c) at c * ldc + r
    if constexpr (R >= 4) {
      // wide tiles: one panel entry per load (the 4-row form would not fit in registers)
      int G = T / pow2_at_least(nJ);
      if (G > 64) G = 64;
      if (G < 1) G = 1;
      const int per = T / G;
      for (int cb = 0; cb < nJ; cb += per) {
        const int c = cb + tid / G, g = tid % G;
        double acc[R];
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = 0.0;
        if (c < nJ) {
          const GLOBAL_AS TP* col = P + (int64_t)c * ldc;
          for (int64_t r = g; r < m; r += (int64_t)G * kUnroll) {
            double av[kUnroll];
#pragma unroll
            for (int e = 0; e < kUnroll; ++e) {
              const int64_t rr = r + (int64_t)e * G;
              const double w = widen(col[rr < m ? rr : m - 1]);
              av[e] = rr < m ? w : 0.0;
            }
#pragma unroll
            for (int e = 0; e < kUnroll; ++e) {
              const int64_t rr = r + (int64_t)e * G;
              const int64_t rc = rr < m ? rr : m - 1;
#pragma unroll
              for (int k = 0; k < R; ++k) acc[k] += av[e] * z[k * m + rc];
            }
          }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = lane_group_sum(acc[k], G);
        if (c < nJ && g == 0) {
#pragma unroll
          for (int k = 0; k < R; ++k) v[k * MJ + c] = acc[k];
        }
      }
      __syncthreads();
      const double cc = coef_col[j];
      for (int64_t r = tid; r < m; r += T) {
        double acc[R];
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = 0.0;
        for (int cb2 = 0; cb2 < nJ; cb2 += kUnroll) {
          double av[kUnroll];
#pragma unroll
          for (int e = 0; e < kUnroll; ++e) {
            const int ce_ = cb2 + e < nJ ? cb2 + e : nJ - 1;
            const double w = widen(P[(int64_t)ce_ * ldc + r]);
            av[e] = cb2 + e < nJ ? w : 0.0;
          }
#pragma unroll
          for (int e = 0; e < kUnroll; ++e) {
            const int ce_ = cb2 + e < nJ ? cb2 + e : nJ - 1;
#pragma unroll
            for (int k = 0; k < R; ++k) acc[k] += av[e] * v[k * MJ + ce_];
          }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) z[k * m + r] -= cc * acc[k];
      }
      __syncthreads();
    } else {
    const int64_t nq = (m + 3) >> 2;
      {
        constexpr int U = vec_unroll_light<R, kThreads>();
        int G = T / pow2_at_least(nJ);
        if (G > 64) G = 64;
        if (G < 1) G = 1;
        const int per = T / G;
        for (int cb = 0; cb < nJ; cb += per) {
          const int c = cb + tid / G, g = tid % G;
          double acc[R];
  #pragma unroll
          for (int k = 0; k < R; ++k) acc[k] = 0.0;
          if (c < nJ) {
            const GLOBAL_AS TP* col = P + (int64_t)c * ldc;
            for (int64_t q0 = g; q0 < nq; q0 += (int64_t)G * U) {
              Chunk4<TP> ch[U];
  #pragma unroll
              for (int e = 0; e < U; ++e) {  // clamped chunk: no branch around the load
                const int64_t qe = q0 + (int64_t)e * G;
                ch[e].load(col + 4 * (qe < nq ? qe : nq - 1));
              }
  #pragma unroll
              for (int e = 0; e < U; ++e) {
                const int64_t qe = q0 + (int64_t)e * G;
                const int64_t qc = qe < nq ? qe : nq - 1;
                const double on = qe < nq ? 1.0 : 0.0;
  #pragma unroll
                for (int i4 = 0; i4 < 4; ++i4) {
                  const int64_t row = 4 * qc + i4 < m ? 4 * qc + i4 : m - 1;
                  const double av = on * ch[e].get(i4);
  #pragma unroll
                  for (int k = 0; k < R; ++k) acc[k] += av * z[k * m + row];
                }
              }
            }
          }
  #pragma unroll
          for (int k = 0; k < R; ++k) acc[k] = lane_group_sum(acc[k], G);
          if (c < nJ && g == 0) {
  #pragma unroll
            for (int k = 0; k < R; ++k) v[k * MJ + c] = acc[k];
          }
        }
      }
      __syncthreads();
      // ---- z update: Z -= coef_J * A_{:,J} V, one thread per 4-row chunk
      {
        constexpr int U = vec_unroll_heavy<R, kThreads>();
        const double cc = coef_col[j];
        for (int64_t qq = tid; qq < nq; qq += T) {
          double acc[4][R];
  #pragma unroll
          for (int i4 = 0; i4 < 4; ++i4)
  #pragma unroll
            for (int k = 0; k < R; ++k) acc[i4][k] = 0.0;
          for (int cb2 = 0; cb2 < nJ; cb2 += U) {
            Chunk4<TP> ch[U];
  #pragma unroll
            for (int e = 0; e < U; ++e) {
              const int ce_ = cb2 + e < nJ ? cb2 + e : nJ - 1;
              ch[e].load(P + (int64_t)ce_ * ldc + 4 * qq);
            }
  #pragma unroll
            for (int e = 0; e < U; ++e) {
              const int ce_ = cb2 + e < nJ ? cb2 + e : nJ - 1;
              const double on = cb2 + e < nJ ? 1.0 : 0.0;
  #pragma unroll
              for (int i4 = 0; i4 < 4; ++i4) {
                const double av = on * ch[e].get(i4);
  #pragma unroll
                for (int k = 0; k < R; ++k) acc[i4][k] += av * v[k * MJ + ce_];
              }
            }
          }
  #pragma unroll
          for (int i4 = 0; i4 < 4; ++i4) {
            const int64_t row = 4 * qq + i4;
            if (row < m) {
  #pragma unroll
              for (int k = 0; k < R; ++k) z[k * m + row] -= cc * acc[i4][k];
            }
          }
        }
      }
      __syncthreads();
    }
    // ---- x-phase: U = A_{I,:} X - B_I + Z_I (nI x R), G lanes per row sum strided columns
    const int64_t r0 = row_off[i];
    const int nI = (int)(row_off[i + 1] - r0);
    const GLOBAL_AS TP* __restrict__ Q = Arow + n * r0;  // (l, c) at c * nI + l
    // whole aligned 4-row chunks in every column of the block (all blocks but a ragged last one)
    const bool vrow = R <= 2 && (nI & 3) == 0 && ((n * r0) & 3) == 0;
    const int nqI = nI >> 2;
    if (vrow) {
      constexpr int U = vec_unroll_heavy<R, kThreads>();
      int G = T / pow2_at_least(nqI);
      if (G > 64) G = 64;
      if (G < 1) G = 1;
      const int per = T / G;
      for (int lb = 0; lb < nqI; lb += per) {
        const int lq = lb + tid / G, g = tid % G;
        double acc[4][R];
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4)
#pragma unroll
          for (int k = 0; k < R; ++k) acc[i4][k] = 0.0;
        if (lq < nqI) {
          for (int64_t c = g; c < n; c += (int64_t)G * U) {
            Chunk4<TP> ch[U];
#pragma unroll
            for (int e = 0; e < U; ++e) {
              const int64_t ce_ = c + (int64_t)e * G;
              ch[e].load(Q + (ce_ < n ? ce_ : n - 1) * nI + 4 * lq);
            }
#pragma unroll
            for (int e = 0; e < U; ++e) {
              const int64_t ce_ = c + (int64_t)e * G;
              const int64_t cl = ce_ < n ? ce_ : n - 1;
              const double on = ce_ < n ? 1.0 : 0.0;
#pragma unroll
              for (int k = 0; k < R; ++k) {
                const double xv = on * x[k * n + cl];
#pragma unroll
                for (int i4 = 0; i4 < 4; ++i4) acc[i4][k] += ch[e].get(i4) * xv;
              }
            }
          }
        }
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4)
#pragma unroll
          for (int k = 0; k < R; ++k) acc[i4][k] = lane_group_sum(acc[i4][k], G);
        if (lq < nqI && g == 0) {
#pragma unroll
          for (int i4 = 0; i4 < 4; ++i4) {
            const int l = 4 * lq + i4;
#pragma unroll
            for (int k = 0; k < R; ++k)
              u[k * MI + l] = (acc[i4][k] - bvec[k * m + r0 + l]) + z[k * m + r0 + l];
          }
        }
      }
    } else {
      int G = T / pow2_at_least(nI);
      if (G > 64) G = 64;
      if (G < 1) G = 1;
      const int per = T / G;
      for (int lb = 0; lb < nI; lb += per) {
        const int l = lb + tid / G, g = tid % G;
        double acc[R];
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = 0.0;
        if (l < nI) {
          for (int64_t c = g; c < n; c += (int64_t)G * kUnroll) {
            double av[kUnroll];
#pragma unroll
            for (int e = 0; e < kUnroll; ++e) {
              const int64_t cc = c + (int64_t)e * G;
              const double w = widen(Q[(cc < n ? cc : n - 1) * nI + l]);
              av[e] = cc < n ? w : 0.0;
            }
#pragma unroll
            for (int e = 0; e < kUnroll; ++e) {
              const int64_t cc = c + (int64_t)e * G;
              const int64_t ccl = cc < n ? cc : n - 1;
#pragma unroll
              for (int k = 0; k < R; ++k) acc[k] += av[e] * x[k * n + ccl];
            }
          }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = lane_group_sum(acc[k], G);
        if (l < nI && g == 0) {
#pragma unroll
          for (int k = 0; k < R; ++k) u[k * MI + l] = (acc[k] - bvec[k * m + r0 + l]) + z[k * m + r0 + l];
        }
      }
    }
    __syncthreads();
    // ---- x update: X -= coef_I * A_{I,:}^T U
    if (vrow) {
      // W lanes per column, one 4-row chunk each; every thread handles U columns at once
      constexpr int U = vec_unroll_light<R, kThreads>();
      const double cr = coef_row[i];
      int W = pow2_at_least(nqI);
      if (W > 64) W = 64;
      const int per = T / W;
      const int sub = tid % W;
      for (int64_t cb = 0; cb < n; cb += (int64_t)per * U) {
        double acc[U][R];
#pragma unroll
        for (int e = 0; e < U; ++e)
#pragma unroll
          for (int k = 0; k < R; ++k) acc[e][k] = 0.0;
        for (int lq = sub; lq < nqI; lq += W) {
          Chunk4<TP> ch[U];
#pragma unroll
          for (int e = 0; e < U; ++e) {
            const int64_t c = cb + tid / W + (int64_t)e * per;
            ch[e].load(Q + (c < n ? c : n - 1) * nI + 4 * lq);
          }
#pragma unroll
          for (int e = 0; e < U; ++e)
#pragma unroll
            for (int k = 0; k < R; ++k)
#pragma unroll
              for (int i4 = 0; i4 < 4; ++i4) acc[e][k] += ch[e].get(i4) * u[k * MI + 4 * lq + i4];
        }
#pragma unroll
        for (int e = 0; e < U; ++e)
#pragma unroll
          for (int k = 0; k < R; ++k) acc[e][k] = lane_group_sum(acc[e][k], W);
        if (sub == 0) {
#pragma unroll
          for (int e = 0; e < U; ++e) {
            const int64_t c = cb + tid / W + (int64_t)e * per;
            if (c < n) {
#pragma unroll
              for (int k = 0; k < R; ++k) x[k * n + c] -= cr * acc[e][k];
            }
          }
        }
      }
    } else {
      const double cr = coef_row[i];
      constexpr int W = 8;
      const int per = T / W;
      for (int64_t cb = 0; cb < n; cb += per) {
        const int64_t c = cb + tid / W;
        const int sub = tid % W;
        double acc[R];
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = 0.0;
        if (c < n) {
          const GLOBAL_AS TP* col = Q + c * nI;
          for (int l0 = sub; l0 < nI; l0 += W * kUnroll) {
            double av[kUnroll];
#pragma unroll
            for (int e = 0; e < kUnroll; ++e) {
              const int le = l0 + e * W < nI ? l0 + e * W : nI - 1;
              const double w = widen(col[le]);
              av[e] = l0 + e * W < nI ? w : 0.0;
            }
#pragma unroll
            for (int e = 0; e < kUnroll; ++e) {
              const int le = l0 + e * W < nI ? l0 + e * W : nI - 1;
#pragma unroll
              for (int k = 0; k < R; ++k) acc[k] += av[e] * u[k * MI + le];
            }
          }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = lane_group_sum(acc[k], W);
        if (c < n && sub == 0) {
#pragma unroll
          for (int k = 0; k < R; ++k) x[k * n + c] -= cr * acc[k];
        }
      }
    }
    __syncthreads();
    done = k1;

    // ---- stop rule: every right-hand side below tol relative to its reference
    if (checking && (k1 % ce == 0 || k1 == a.max_iter)) {
      colwise_sum([&](int k, int64_t c) { const double d = x[k * n + c] - xref[k * n + c]; return d * d; }, etot);
      bool all_ok = true, bad = false;
      for (int k = 0; k < R; ++k) {
        const double rel = sqrt(etot[k]) / (xr2[k] > 0.0 ? sqrt(xr2[k]) : 1.0);  // absolute if x_ref = 0
        all_ok = all_ok && rel < a.tol;
        bad = bad || !isfinite(etot[k]) || rel > 1e6;
      }
      if (stopping && all_ok) { status = 0; break; }
      if (bad) { status = 2; break; }
    }
  }

  {
    GLOBAL_AS double* xo = gptr(tk.x_out);
    for (int64_t e = tid; e < (int64_t)R * n; e += T) xo[e] = x[e];
  }
  if (tk.z_out) {
    GLOBAL_AS double* zo = gptr(tk.z_out);
    for (int64_t e = tid; e < (int64_t)R * m; e += T) zo[e] = z[e];
  }
  if (tid < R) tk.err2_out[tid] = checking ? etot[tid] : -1.0;
  if (tid == 0) {
    if (!stopping && status == 1) status = checking ? 1 : 0;
    *tk.iters_out = done;
    *tk.status_out = status;
  }
}

// One kernel per tile width R (every task of a launch has width R) and per workgroup size (256,
// 512 or 1024 threads): a single kernel holding all three widths needs more registers than a
// wave has and spills.
template <typename TP, int R, int kThreads>
__global__ void __launch_bounds__(kThreads) batch_solve_kernel(BatchArgs a) {
  extern __shared__ double lds[];
  __shared__ int s_j[kDrawBatch], s_i[kDrawBatch];
  if ((int)blockIdx.x >= a.ntasks) return;
  const BatchTask tk = a.tasks[blockIdx.x];
  if (tk.sys < 0 || tk.R != R) return;
  const BatchSys S = a.sys[tk.sys];
  run_task<TP, R, kThreads>(S, tk, a, lds, s_j, s_i);
}

}  // namespace

size_t batch_lds_bytes(int64_t m, int64_t n, int R, int max_nJ, int max_nI, int threads) {
  return batch_layout(m, n, R, max_nJ, max_nI, threads).total * sizeof(double);
}

namespace {
template <typename TP>
const void* batch_kernel_ptr(int R, int threads) {
  if (threads > 512) {
    return R == 1 ? (const void*)batch_solve_kernel<TP, 1, 1024>
                  : (R == 2 ? (const void*)batch_solve_kernel<TP, 2, 1024> : (const void*)batch_solve_kernel<TP, 4, 1024>);
  }
  if (threads <= 256) {
    return R == 1 ? (const void*)batch_solve_kernel<TP, 1, 256>
                  : (R == 2 ? (const void*)batch_solve_kernel<TP, 2, 256> : (const void*)batch_solve_kernel<TP, 4, 256>);
  }
  return R == 1 ? (const void*)batch_solve_kernel<TP, 1, 512>
                : (R == 2 ? (const void*)batch_solve_kernel<TP, 2, 512> : (const void*)batch_solve_kernel<TP, 4, 512>);
}
}  // namespace

hipError_t batch_max_blocks(int panel_dtype, int threads, int R, size_t lds_bytes, int* blocks_per_cu) {
  if (R != 1 && R != 2 && R != 4) return hipErrorInvalidValue;
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const void* k = batch_kernel_ptr<TP>(R, threads);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, threads, lds_bytes);
  });
}

hipError_t launch_batch_solve(const BatchArgs& a, int panel_dtype, int threads, int R, size_t lds_bytes,
                              hipStream_t st) {
  if ((threads != 256 && threads != 512 && threads != 1024) || (R != 1 && R != 2 && R != 4)) return hipErrorInvalidValue;
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const void* k = batch_kernel_ptr<TP>(R, threads);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    BatchArgs aa = a;
    void* args[] = {&aa};
    return hipLaunchKernel(k, dim3(a.ntasks), dim3(threads), args, lds_bytes, st);
  });
}

}  // namespace rebk
