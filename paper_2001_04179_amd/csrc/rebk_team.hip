// Team REBK for gfx950: one tile of up to kTeamR right-hand sides of one system solved by P
// workgroups together (Du, Si, Sun, arXiv:2001.04179, Algorithm 1 on each right-hand side).
//
// A batch task runs on one compute unit, whose memory parallelism caps its panel stream at tens of
// GB/s, so a system that needs far more iterations than the others (an ill-conditioned one) sets
// the time of the whole batch.  A team spreads such a system over P compute units.  Workgroup p
// owns rows [p m / P, (p + 1) m / P) of Z and B and columns [p n / P, (p + 1) n / P) of X, for all
// right-hand sides of the tile, in LDS.  The z-chain never reads x, so the x-chain runs one
// iteration behind and a single team-wide reduction per iteration carries, for every right-hand
// side,
//   - partials of v^{k+1} = A_{:,J_{k+1}}^T z^k over owned rows,
//   - partials of u^k = A_{I_k,:} x^{k-1} - b_{I_k} + z^k_{I_k} (owned columns; z - b on owned
//     rows), and
//   - on iterations the stop rule checks, partials of ||x^{k-1} - x_ref||^2 over owned columns.
// Each workgroup reads its two panel slabs (A_{R_p, J} and A_{I, C_p}) once per iteration into
// LDS; each serves the partial sums of one round and the update of the next.
//
// Reduction: the round's entries are numbered compactly (v, then u, then the errors).  Entry e is
// summed by workgroup e mod P, which polls it in all P partial vectors, adds the P values in a
// fixed order and publishes the sum; every workgroup then reads all sums.  Every value crossing
// workgroups is a pair of 64-bit device-scope atomic words that both carry the round's epoch, so
// a reader tells a current value from a stale or torn one without fences or counters.  Every
// workgroup sees the same sums, so a run is reproducible bit for bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rebk_device.h"
#include "rebk_internal.h"
#include "rebk_team.h"

namespace rebk {
namespace {

using namespace dev;

constexpr int R = kTeamR;
constexpr int T = kTeamThreads;
constexpr unsigned kSpinLimit = 1u << 22;  // polls before a wait gives up (seconds)
constexpr int kRing = 128;                 // block draws kept: iteration q in slot (q - 1) mod 128
constexpr int kPre = 16;                   // slab entries per thread loaded ahead into registers
static_assert(kTeamR == 16, "the block products are 16-column matrix-core tiles");
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Pointers taken from the task tables are generic; the compiler would access them with flat
// instructions, which also count on the LDS wait counter, so every LDS access would wait for the
// panel loads and reduction stores in flight.  These casts state that they point to global memory.
#define GAS __attribute__((address_space(1)))
template <typename X>
__device__ __forceinline__ const GAS X* gp(const X* p) {
  return (const GAS X*)p;
}
template <typename X>
__device__ __forceinline__ GAS X* gp(X* p) {
  return (GAS X*)p;
}
typedef unsigned long long u64;

__device__ __forceinline__ u64 ld_dev(const GAS u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(GAS u64* p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// value v for epoch ep as the pair p[0] = (ep, high half of the bits), p[1] = (low half, ep)
__device__ __forceinline__ void put_tagged(GAS u64* p, double v, unsigned ep) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  st_dev(p, ((unsigned long long)ep << 32) | (bits >> 32));
  st_dev(p + 1, (bits << 32) | (unsigned long long)ep);
}
__device__ __forceinline__ bool tagged_ok(unsigned long long w0, unsigned long long w1, unsigned ep) {
  return (unsigned)(w0 >> 32) == ep && (unsigned)w1 == ep;
}
__device__ __forceinline__ double tagged_value(unsigned long long w0, unsigned long long w1) {
  return __longlong_as_double((long long)((w0 << 32) | (w1 >> 32)));
}

template <int CTRL>
__device__ __forceinline__ double tdpp(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false));
}
// Sum over aligned groups of `width` lanes (a power of two <= 64); every lane of a group gets the
// group's sum.  All 64 lanes must execute it.
__device__ __forceinline__ double team_group_sum(double v, int width) {
  if (width >= 2) v += tdpp<0xB1>(v);    // quad_perm [1,0,3,2]
  if (width >= 4) v += tdpp<0x4E>(v);    // quad_perm [2,3,0,1]
  if (width >= 8) v += tdpp<0x141>(v);   // row_half_mirror
  if (width >= 16) v += tdpp<0x140>(v);  // row_mirror
  if (width >= 32) v += __shfl_xor(v, 16, 64);
  if (width >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}
// floor(e / d) and e mod d for 0 <= e < 2^24 and d >= 1, from a float reciprocal and one correction
__device__ __forceinline__ int div_by(int e, int d, float inv, int& rem) {
  int q = (int)((float)e * inv);
  if (q * d > e) --q;
  else if ((q + 1) * d <= e) ++q;
  rem = e - q * d;
  return q;
}
struct TeamLayout {
  int NR, NC;      // rows / columns a workgroup owns, at most
  int VJ, UI;      // strides of the right-hand sides in v and u
  int SC, SR;      // slab strides: column slab entry (q, c) at c * SC + q, row slab (l, c) at c * SR + l
  size_t z, zp, bl, x, v, u, dbl;  // offsets in doubles; dbl: doubles before the slabs
  size_t sC, sR;   // panel entries per slab buffer (two buffers of each)
};

__host__ __device__ inline TeamLayout team_layout(int64_t m, int64_t n, int P, int MJ, int MI) {
  TeamLayout L;
  L.NR = (int)((m + P - 1) / P) + 1;
  L.NC = (int)((n + P - 1) / P) + 1;
  // odd strides put the right-hand sides (and slab columns) on different LDS banks
  L.VJ = MJ | 1;
  L.UI = MI | 1;
  L.SC = L.NR | 1;
  L.SR = MI | 1;
  L.z = 0;
  L.zp = L.z + (size_t)R * L.NR;
  L.bl = L.zp + (size_t)R * L.NR;
  L.x = L.bl + (size_t)R * L.NR;
  L.v = L.x + (size_t)R * L.NC;
  L.u = L.v + (size_t)R * L.VJ;
  L.dbl = (L.u + (size_t)R * L.UI + 1) & ~(size_t)1;
  L.sC = ((size_t)L.SC * MJ + 7) / 8 * 8;
  L.sR = ((size_t)L.SR * L.NC + 7) / 8 * 8;
  return L;
}

template <typename TP>
__global__ void __launch_bounds__(T) team_solve_kernel(BatchArgs a, TeamArgs ta) {
  extern __shared__ double lds[];
  __shared__ int s_nJ[kRing], s_nI[kRing];
  __shared__ int64_t s_c0[kRing], s_r0[kRing];
  __shared__ double s_cc[kRing], s_cr[kRing];
  __shared__ double s_err[R], s_xr2[R];
  __shared__ int s_bad;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const TeamTask tt = ta.teams[ta.team_of_wg[blockIdx.x]];
  const BatchTask tk = a.tasks[tt.task];
  const BatchSys S = a.sys[tk.sys];
  const int P = tt.P, p = (int)blockIdx.x - tt.wg0, nk = tk.R, E = tt.E;
  const int64_t m = S.m, n = S.n;
  const int MJ = a.max_nJ, MI = a.max_nI;
  const TeamLayout L = team_layout(m, n, P, MJ, MI);
  const int64_t r0 = (int64_t)p * m / P, r1 = (int64_t)(p + 1) * m / P;
  const int64_t cA = (int64_t)p * n / P, cB = (int64_t)(p + 1) * n / P;
  const int nr = (int)(r1 - r0), nc = (int)(cB - cA);
  double* z = lds + L.z;    // z[k * NR + q], q < nr
  double* zp = lds + L.zp;  // previous z (returned when the stop rule fires one iteration late)
  double* bl = lds + L.bl;  // b on owned rows
  double* x = lds + L.x;    // x[k * NC + c], c < nc
  double* v = lds + L.v;    // reduced v[k * VJ + c]
  double* u = lds + L.u;    // reduced u[k * UI + l]
  TP* slabC = (TP*)(lds + L.dbl);
  TP* slabR = slabC + 2 * L.sC;
  const GAS TP* __restrict__ Arow = gp((const TP*)S.Arow);
  const GAS TP* __restrict__ Acol = gp((const TP*)S.Acol);
  const GAS double* __restrict__ bvec = gp(tk.b);
  const GAS double* __restrict__ xref = gp(tk.x_ref);
  const GAS int64_t* __restrict__ col_off = gp(S.col_off);
  const GAS int64_t* __restrict__ row_off = gp(S.row_off);
  const GAS double* __restrict__ coef_col = gp(S.coef_col);
  const GAS double* __restrict__ coef_row = gp(S.coef_row);
  GAS u64* const part = gp(tt.part);
  GAS u64* const sum = gp(tt.sum);
  GAS int* const timeout = gp(ta.timeout);
  const int64_t K = a.max_iter;
  const int64_t ce = a.check_every > 0 ? a.check_every : 1;
  const bool checking = tk.x_ref != nullptr;
  const bool stopping = checking && a.tol > 0.0;

  if (tid == 0) s_bad = 0;
  for (int e = tid; e < R * nr; e += T) {
    const int k = e / nr, q = e - k * nr;
    const double bv = k < nk ? bvec[(int64_t)k * m + r0 + q] : 0.0;
    z[k * L.NR + q] = bv;
    zp[k * L.NR + q] = bv;
    bl[k * L.NR + q] = bv;
  }
  for (int e = tid; e < R * nc; e += T) {
    const int k = e / nc, c = e - k * nc;
    x[k * L.NC + c] = (k < nk && tk.x_in) ? gp(tk.x_in)[(int64_t)k * n + cA + c] : 0.0;
  }

  auto slot = [&](int64_t q) -> int { return (int)((q - 1) & (kRing - 1)); };
  auto refill = [&](int64_t first) {  // draws of iterations first .. first + 63
    if (tid < 64) {
      const int64_t q = first + tid;
      if (q <= K) {
        int jj, ii;
        draw_pair(S, q, jj, ii);
        const int sl = slot(q);
        s_c0[sl] = col_off[jj];
        s_nJ[sl] = (int)(col_off[jj + 1] - col_off[jj]);
        s_r0[sl] = row_off[ii];
        s_nI[sl] = (int)(row_off[ii + 1] - row_off[ii]);
        s_cc[sl] = coef_col[jj];
        s_cr[sl] = coef_row[ii];
      }
    }
  };
  refill(1);
  refill(65);
  int64_t filled = 128;
  __syncthreads();

  // This round's two slabs: the column slab of iteration qc (owned rows of the nJ columns of J;
  // column panels hold A^T, so each column is a run of the owned rows; entry (q, c) goes to
  // c * SC + q) and the row slab of iteration qr (owned columns of I: one run of nc x nI entries
  // of the column-major row panel; entry (l, c) goes to c * SR + l).  fetch(), called before the
  // previous round's reduction, issues the first kPre entries of each thread into registers;
  // place(), after this round's updates, stores them and copies the rest.
  struct SlabCopy {
    const GAS TP* c;  // column slab source (NULL: none)
    const GAS TP* r;  // row slab source
    TP* dc;
    TP* dr;
    int nJ, nI, CT, total;
    float inv_nr, inv_nI;
  };
  // Entry e of the copy: source and LDS destination (column slab for e < CT, then row slab).
  auto src_of = [&](const SlabCopy& sc, int e) -> const GAS TP* {
    int rem;
    const int c = div_by(e < sc.CT ? e : 0, nr > 0 ? nr : 1, sc.inv_nr, rem);
    return e < sc.CT ? sc.c + (int64_t)c * S.ldc + rem : sc.r + (e - sc.CT);
  };
  auto dst_of = [&](const SlabCopy& sc, int e) -> TP* {
    int rc, rr;
    const int c = div_by(e < sc.CT ? e : 0, nr > 0 ? nr : 1, sc.inv_nr, rc);
    const int f = e < sc.CT ? 0 : e - sc.CT;
    const int l = div_by(f, sc.nI > 0 ? sc.nI : 1, sc.inv_nI, rr);
    return e < sc.CT ? sc.dc + c * L.SC + rc : sc.dr + l * L.SR + rr;
  };
  // Every thread issues its kPre loads without branches (entries past the end read the first
  // entry of the row slab, or the start of the row panel), so they are all in flight at once.
  auto fetch = [&](const SlabCopy& sc, TP (&pre)[kPre]) {
    if (sc.total == 0) return;
    // column-slab entry e = c nr + q: (c, q) of e = tid + j T follow from those of j - 1 by adding
    // (T / nr, T mod nr) with a carry
    const int nrr = nr > 0 ? nr : 1;
    int qT;
    const int cT = div_by(T, nrr, sc.inv_nr, qT);
    int q0;
    int c0 = div_by(tid, nrr, sc.inv_nr, q0);
#pragma unroll
    for (int j = 0; j < kPre; ++j) {
      const int e = tid + j * T;
      const GAS TP* src = e < sc.CT ? sc.c + (int64_t)c0 * S.ldc + q0 : sc.r + ((e < sc.total ? e : sc.CT) - sc.CT);
      pre[j] = *src;
      q0 += qT;
      c0 += cT;
      if (q0 >= nrr) {
        q0 -= nrr;
        ++c0;
      }
    }
  };
  auto place = [&](const SlabCopy& sc, TP (&pre)[kPre]) {
    if (sc.total == 0) return;
#pragma unroll
    for (int j = 0; j < kPre; ++j) {
      const int e = tid + j * T;
      if (e < sc.total) *dst_of(sc, e) = pre[j];
    }
    constexpr int kMore = 4;
    for (int e0 = kPre * T; e0 < sc.total; e0 += kMore * T) {  // larger slabs: kMore more per pass
      TP more[kMore];
#pragma unroll
      for (int j = 0; j < kMore; ++j) {
        const int e = e0 + tid + j * T;
        more[j] = *src_of(sc, e < sc.total ? e : sc.CT);
      }
#pragma unroll
      for (int j = 0; j < kMore; ++j) {
        const int e = e0 + tid + j * T;
        if (e < sc.total) *dst_of(sc, e) = more[j];
      }
    }
  };

  // Partial vectors: the entries of a round are [0, nk nJ) of v (k nJ + c), then nk nI of u
  // (k nI + l), then nk errors (k).
  // ||x - x_ref||^2 (or ||x_ref||^2 with ref_only) over owned columns, wave w taking the
  // right-hand sides w, w + 4, ...
  auto part_err = [&](GAS u64* Pw, int base, unsigned ep, bool ref_only) {
    for (int k0 = 0; k0 < R; k0 += T / 64) {
      const int k = k0 + wave;
      double e = 0.0;
      if (k < nk) {
        const GAS double* xr = xref + (int64_t)k * n + cA;
        for (int c = lane; c < nc; c += 64) {
          const double d = ref_only ? xr[c] : x[k * L.NC + c] - xr[c];
          e += d * d;
        }
      }
      e = team_group_sum(e, 64);
      if (k < nk && lane == 0) put_tagged(Pw + 2 * (size_t)(base + k), e, ep);
    }
  };

  // Team-wide sum of the round's partial vectors (published with epoch ep): v gets nk x nJ
  // entries, u nk x nI, s_err nk with has_err.  Returns false after a spin-limit timeout.
  auto reduce = [&](unsigned ep, int nJ, int nI, bool has_err) -> bool {
    const int nv = nk * nJ, nu = nk * nI, N = nv + nu + (has_err ? nk : 0);
    const int par = (int)(ep & 1u);
    const GAS u64* Pb = part + (size_t)par * P * E * 2;
    GAS u64* Sv = sum + (size_t)par * E * 2;
    bool ok = true;
    unsigned spins = 0;
    auto give_up = [&]() -> bool {  // bounded waiting
      if ((++spins & 63u) == 0) {
        if (__hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
        if (spins > kSpinLimit) {
          __hip_atomic_store(timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          return true;
        }
      }
      return false;
    };
    // 1. entries p, p + P, ...: LE lanes per entry, lane `sub` polls workgroups sub, sub + LE, ...
    //    (up to 4 each); a lane group takes up to kEM entries at once, so that all the loads of a
    //    pass are in flight together
    {
      constexpr int kEM = 4;
      int LE = 1;
      while (LE < P && LE < 64) LE *= 2;
      const int EPW = 64 / LE, grp = lane / LE, sub = lane % LE;
      const int nown = N > p ? (N - p + P - 1) / P : 0;
      const int groups = (T / 64) * EPW;  // lane groups of the workgroup
      for (int j0 = 0; j0 < nown; j0 += groups * kEM) {  // uniform over the workgroup
        const int g = wave * EPW + grp;
        unsigned pending = 0;
#pragma unroll
        for (int m = 0; m < kEM; ++m)
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
            if (j0 + g + m * groups < nown && sub + s4 * LE < P) pending |= 1u << (4 * m + s4);
        const unsigned mine = pending;
        double vals[kEM * 4];
#pragma unroll
        for (int q = 0; q < kEM * 4; ++q) vals[q] = 0.0;
        while (ok) {
          u64 w0[kEM * 4], w1[kEM * 4];
#pragma unroll
          for (int q = 0; q < kEM * 4; ++q)
            if ((pending >> q) & 1u) {  // (each slot has its own registers: the loads overlap)
              const GAS u64* a = Pb + ((size_t)(sub + (q % 4) * LE) * E + p + (j0 + g + (q / 4) * groups) * P) * 2;
              w0[q] = ld_dev(a);
              w1[q] = ld_dev(a + 1);
            }
#pragma unroll
          for (int q = 0; q < kEM * 4; ++q)
            if (((pending >> q) & 1u) && tagged_ok(w0[q], w1[q], ep)) {
              vals[q] = tagged_value(w0[q], w1[q]);
              pending &= ~(1u << q);
            }
          if (!__any(pending != 0)) break;
          if (give_up()) ok = false;
        }
#pragma unroll
        for (int m = 0; m < kEM; ++m) {
          double acc = 0.0;
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
            if ((mine >> (4 * m + s4)) & 1u) acc += vals[4 * m + s4];
          acc = team_group_sum(acc, LE);
          const int jm = j0 + g + m * groups;
          if (ok && jm < nown && sub == 0) put_tagged(Sv + 2 * (size_t)(p + jm * P), acc, ep);
        }
      }
    }
    // 2. every entry of the reduced vector, up to 8 per thread per pass
    for (int i0 = 0; i0 < N; i0 += 8 * T) {
      unsigned pending = 0;
#pragma unroll
      for (int t8 = 0; t8 < 8; ++t8)
        if (i0 + t8 * T + tid < N) pending |= 1u << t8;
      const unsigned mine = pending;
      double vals[8];
      while (ok) {
        u64 w0[8], w1[8];
#pragma unroll
        for (int t8 = 0; t8 < 8; ++t8)
          if ((pending >> t8) & 1u) {
            const GAS u64* q = Sv + 2 * (size_t)(i0 + t8 * T + tid);
            w0[t8] = ld_dev(q);
            w1[t8] = ld_dev(q + 1);
          }
#pragma unroll
        for (int t8 = 0; t8 < 8; ++t8)
          if (((pending >> t8) & 1u) && tagged_ok(w0[t8], w1[t8], ep)) {
            vals[t8] = tagged_value(w0[t8], w1[t8]);
            pending &= ~(1u << t8);
          }
        if (!__any(pending != 0)) break;
        if (give_up()) ok = false;
      }
      if (ok) {
#pragma unroll
        for (int t8 = 0; t8 < 8; ++t8)
          if ((mine >> t8) & 1u) {
            const int i = i0 + t8 * T + tid;
            if (i < nv) {
              const int k = i / nJ, c = i - k * nJ;
              v[k * L.VJ + c] = vals[t8];
            } else if (i < nv + nu) {
              const int t = i - nv, k = t / nI, l = t - k * nI;
              u[k * L.UI + l] = vals[t8];
            } else {
              s_err[i - nv - nu] = vals[t8];
            }
          }
      }
    }
    if (!ok) s_bad = 1;  // never cleared: a timeout ends the launch
    __syncthreads();
    return s_bad == 0;
  };

  auto part_ptr = [&](unsigned ep) -> GAS u64* { return part + ((size_t)(ep & 1u) * P + p) * E * 2; };
  // stop rule on s_err (the same values in every workgroup): 0 stop on tol, 2 diverged, 1 go on
  auto check = [&]() -> int {
    bool all_ok = true, bad = false;
    for (int k = 0; k < nk; ++k) {
      const double rel = sqrt(s_err[k]) / (s_xr2[k] > 0.0 ? sqrt(s_xr2[k]) : 1.0);  // absolute if x_ref = 0
      all_ok = all_ok && rel < a.tol;
      bad = bad || !isfinite(s_err[k]) || rel > 1e6;
    }
    if (stopping && all_ok) return 0;
    if (bad) return 2;
    return 1;
  };

  unsigned epoch = 0;
  bool alive = true;
  int status = 1;
  int64_t done = K;

  // Round r = 0 .. K + 1 (one reduction each; every piece of code below appears once, which keeps
  // the loop within the instruction cache):
  //   z-step z^r = z^{r-1} - coef_J A_{R_p,J_r} v^r (1 <= r <= K, keeping z^{r-1}),
  //   x-step x^{r-1} = x^{r-2} - coef_I A_{I_{r-1},C_p}^T u^{r-1} (r >= 2),
  //   partials of v^{r+1} (r < K), of u^r (1 <= r <= K) and of the error of x^{r-1} where the stop
  //   rule checks it (round 0: ||x_ref||^2 instead).
  // The column slab of iteration q and the row slab of iteration q live in buffer q & 1.
  // The slabs of round rr: the column slab of v^{rr+1} and the row slab of u^{rr}.
  auto make_copy = [&](int64_t rr) -> SlabCopy {
    SlabCopy c;
    const int64_t qc = rr + 1 <= K ? rr + 1 : 0, qr = (rr >= 1 && rr <= K) ? rr : 0;
    c.nJ = qc ? s_nJ[slot(qc)] : 0;
    c.nI = qr ? s_nI[slot(qr)] : 0;
    c.c = Acol + S.ldc * (qc ? s_c0[slot(qc)] : 0) + r0;
    c.r = Arow + n * (qr ? s_r0[slot(qr)] : 0) + cA * c.nI;
    c.dc = slabC + (size_t)(qc & 1) * L.sC;
    c.dr = slabR + (size_t)(qr & 1) * L.sR;
    c.CT = c.nJ * nr;
    c.total = c.CT + c.nI * nc;
    c.inv_nr = nr > 0 ? 1.0f / (float)nr : 0.0f;
    c.inv_nI = c.nI > 0 ? 1.0f / (float)c.nI : 0.0f;
    return c;
  };
  // each round's slab loads are issued before the previous reduction (into registers), so they
  // land while it waits; the round stores them after its updates
  TP pre[kPre];
  SlabCopy sc_next = make_copy(0);
  fetch(sc_next, pre);
  for (int64_t r = 0; r <= K + 1; ++r) {
    if (r + 2 > filled && filled < K) {
      refill(filled + 1);
      filled += 64;
      __syncthreads();
    }
    const bool zs = r >= 1 && r <= K, xs = r >= 2;
    const int64_t qc = r + 1 <= K ? r + 1 : 0, qr = zs ? r : 0;
    const int nJr = zs ? s_nJ[slot(r)] : 0;
    const double ccr = zs ? s_cc[slot(r)] : 0.0;
    const int nIp = xs ? s_nI[slot(r - 1)] : 0;
    const double crp = xs ? s_cr[slot(r - 1)] : 0.0;
    const int nJn = qc ? s_nJ[slot(qc)] : 0;
    const int nIr = qr ? s_nI[slot(qr)] : 0;
    const int64_t rIr = qr ? s_r0[slot(qr)] : 0;
    TP* const Cbuf0 = slabC;
    TP* const Rbuf0 = slabR;
    const bool has_err = checking && (r == 0 || (r >= 2 && ((r - 1) % ce == 0 || r - 1 == K)));
    GAS u64* const Pw = part_ptr(epoch + 1);
    const unsigned ep = epoch + 1;

    const SlabCopy sc = sc_next;  // this round's slabs, in flight since the previous round

    // The four block products of the round share one loop (mode 0: z-step, 1: x-step, 2: partial
    // v, 3: partial u), each a product of a slab block with the kTeamR right-hand sides:
    //   out(i, k) = sum_{t < len} M[i si + t st] w[k ws + t],  i < nitems, k < 16,
    // on the FP64 matrix cores: wave w takes the 16-item tiles w, w + 4, ...; one
    // v_mfma_f64_16x16x4f64 per 4 values of t, in increasing t (a fixed order).  Lane l supplies
    // A(i0 + l mod 16, t0 + l / 16) and B(t0 + l / 16, k = l mod 16) and receives
    // out(i0 + l / 16 + 4 j, l mod 16) in register j < 4; entries past nitems or len are zeros.
#pragma unroll 1
    for (int mode = 0; mode < 4; ++mode) {
      if (mode == 2) {  // the updates are done: store the slabs, then the partial products
        place(sc, pre);
        __syncthreads();
      }
      const TP* M;
      const double* w;
      int si, st, nitems, len, ws;
      if (mode == 0) {
        if (!zs) continue;
        M = Cbuf0 + (size_t)(r & 1) * L.sC;  // A_{R_p, J_r}: entry (q, c) at c SC + q
        si = 1; st = L.SC; nitems = nr; len = nJr; w = v; ws = L.VJ;
      } else if (mode == 1) {
        if (!xs) continue;
        M = Rbuf0 + (size_t)((r - 1) & 1) * L.sR;  // A_{I_{r-1}, C_p}: entry (l, c) at c SR + l
        si = L.SR; st = 1; nitems = nc; len = nIp; w = u; ws = L.UI;
      } else if (mode == 2) {
        if (nJn == 0) continue;
        M = Cbuf0 + (size_t)(qc & 1) * L.sC;
        si = L.SC; st = 1; nitems = nJn; len = nr; w = z; ws = L.NR;
      } else {
        if (nIr == 0) continue;
        M = Rbuf0 + (size_t)(qr & 1) * L.sR;
        si = 1; st = L.SR; nitems = nIr; len = nc; w = x; ws = L.NC;
      }
      const int li = lane & 15, lt = lane >> 4;
      for (int i0 = wave * 16; i0 < nitems; i0 += T / 4) {  // uniform over the wave
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        const int ia = i0 + li < nitems ? i0 + li : nitems - 1;
        const bool a_on = i0 + li < nitems;
        for (int t0 = 0; t0 < len; t0 += 16) {  // operands of 4 steps loaded first, so they overlap
          double av[4], bv[4];
#pragma unroll
          for (int u4 = 0; u4 < 4; ++u4) {
            const int t = t0 + 4 * u4 + lt;
            const bool on = t < len;
            const int tc = on ? t : len - 1;
            // unconditional loads from clamped (valid) addresses, masked afterwards: a load under
            // a branch would wait for itself before the next one
            const double a = widen(M[ia * si + tc * st]);
            const double b = w[li * ws + tc];
            av[u4] = (a_on && on) ? a : 0.0;
            bv[u4] = on ? b : 0.0;
          }
#pragma unroll
          for (int u4 = 0; u4 < 4; ++u4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u4], bv[u4], acc, 0, 0, 0);
        }
        const int k = li;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int it = i0 + lt + 4 * j;
          if (it >= nitems) continue;
          const double val = acc[j];
          if (mode == 0) {
            const double zo = z[k * L.NR + it];
            zp[k * L.NR + it] = zo;
            z[k * L.NR + it] = zo - ccr * val;
          } else if (mode == 1) {
            x[k * L.NC + it] -= crp * val;
          } else if (mode == 2) {
            if (k < nk) put_tagged(Pw + 2 * (size_t)(k * nJn + it), val, ep);
          } else if (k < nk) {
            const int64_t gl = rIr + it;
            const bool own = gl >= r0 && gl < r1;
            const double t = own ? val + (z[k * L.NR + (gl - r0)] - bl[k * L.NR + (gl - r0)]) : val;
            put_tagged(Pw + 2 * (size_t)(nk * nJn + k * nIr + it), t, ep);
          }
        }
      }
    }
    if (has_err) part_err(Pw, nk * (nJn + nIr), ep, r == 0);
    if (r <= K) {  // the next round's slab loads
      sc_next = make_copy(r + 1);
      fetch(sc_next, pre);
    }
    if (nJn == 0 && nIr == 0 && !has_err) break;  // the last round of a run without checks
    alive = reduce(++epoch, nJn, nIr, has_err);
    if (!alive) break;
    if (r == 0) {
      if (checking && tid < nk) s_xr2[tid] = s_err[tid];
      __syncthreads();
      continue;
    }
    if (has_err) {  // the stop rule at iteration r - 1: x is x^{r-1}
      const int st = check();
      if (st != 1 || r - 1 == K) {
        status = st;
        done = r - 1;
        if (zs) {  // z has moved on to z^r: return z^{r-1}
          for (int e = tid; e < R * nr; e += T) {
            const int k = e / nr, q = e - k * nr;
            z[k * L.NR + q] = zp[k * L.NR + q];
          }
          __syncthreads();
        }
        break;
      }
    }
  }
  if (!stopping && status == 1) status = checking ? 1 : 0;

  for (int e = tid; e < R * nc; e += T) {
    const int k = e / nc, c = e - k * nc;
    if (k < nk) gp(tk.x_out)[(int64_t)k * n + cA + c] = x[k * L.NC + c];
  }
  if (tk.z_out)
    for (int e = tid; e < R * nr; e += T) {
      const int k = e / nr, q = e - k * nr;
      if (k < nk) gp(tk.z_out)[(int64_t)k * m + r0 + q] = z[k * L.NR + q];
    }
  if (p == 0) {
    if (tid < nk) {
      gp(tk.err2_out)[tid] = checking ? s_err[tid] : -1.0;
      if (checking) gp(tk.xref2_out)[tid] = s_xr2[tid];
    }
    if (tid == 0) {
      *gp(tk.iters_out) = done;
      *gp(tk.status_out) = alive ? status : -4;
    }
  }
}

template <typename TP>
const void* team_kernel_ptr() {
  return (const void*)team_solve_kernel<TP>;
}

}  // namespace

size_t team_lds_bytes(int64_t m, int64_t n, int P, int max_nJ, int max_nI, int panel_dtype) {
  const size_t esz = panel_dtype == 0 ? 8 : (panel_dtype == 1 ? 4 : 2);
  const TeamLayout L = team_layout(m, n, P, max_nJ, max_nI);
  return L.dbl * sizeof(double) + 2 * (L.sC + L.sR) * esz + 64;
}

hipError_t team_max_blocks(int panel_dtype, size_t lds_bytes, int* blocks_per_cu) {
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const void* k = team_kernel_ptr<TP>();
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, kTeamThreads, lds_bytes);
  });
}

hipError_t launch_team_solve(const BatchArgs& a, const TeamArgs& ta, int wgs, int panel_dtype, size_t lds_bytes,
                             hipStream_t st) {
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const void* k = team_kernel_ptr<TP>();
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    BatchArgs aa = a;
    TeamArgs tt = ta;
    void* args[] = {&aa, &tt};
    return hipLaunchCooperativeKernel(k, dim3(wgs), dim3(kTeamThreads), args, (unsigned)lds_bytes, st);
  });
}

}  // namespace rebk
