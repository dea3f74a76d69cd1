// Persistent cooperative REBK kernel for gfx950 (Du, Si, Sun, arXiv:2001.04179, Algorithm 1).
//
// Ownership: workgroup w owns rows [w*m/G, (w+1)*m/G) of z and columns [w*n/G, (w+1)*n/G) of x;
// both stay in LDS for the whole launch.  One grid-wide reduction per iteration carries
//   - the partial sums of v^{k+1} = A_{:,J_{k+1}}^T z^k over owned rows,
//   - the partial sums of u^k = A_{I_k,:} x^{k-1} - b_{I_k} + z^k_{I_k} (owned columns, plus
//     z - b on owned rows), and
//   - the partial error ||x^{k-1} - x_ref||^2 over owned columns.
// The z-chain never reads x, so running the x-chain one iteration behind the z-chain is exact and
// needs a single synchronisation per iteration.
//
// Reduction: a deterministic reduce-scatter and all-gather without counters or fences.  Every
// value crossing workgroups is published as two 64-bit atomic words that both carry the
// iteration's epoch, so a reader can tell a current value from a stale or half-written one.  The
// partial vector is cut into chunks of kChunk entries; workgroup c owns chunk c (c, c + G, ... for
// long vectors): it polls that chunk of every workgroup's partial vector, sums the G partials in
// a fixed order and publishes the tagged sums.  Every workgroup then reads the reduced vector
// once.  Each sum is formed by one workgroup, so all workgroups see bit-identical reduced vectors
// and a run is reproducible bit for bit.  All cross-workgroup traffic uses device-scope atomic
// loads and stores, coherent across the eight XCDs without cache maintenance (an agent-scope
// release fence writes back the XCD's L2 and costs microseconds on gfx950).
//
// Panel slabs: the column slab A_{R_w, J} (owned rows; column panels hold A^T, so the slab is |J|
// runs of the owned rows) and the row slab A_{I, C_w} (owned columns, contiguous in the
// column-major row panel) are read from HBM once each: for the partial sums of one round and,
// from LDS, for the update of the next.  Because the block sequence depends only on the
// counter-based generator, waves 1..3 copy the next round's slabs straight into LDS with
// global_load_lds while the reduction is in flight.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rebk_device.h"
#include "rebk_internal.h"

namespace rebk {
namespace {

using namespace dev;

constexpr unsigned kSpinLimit = 1u << 22;  // polls before a barrier gives up (seconds)
// Entries per reduction chunk (1, 2, 4 or 8).  Smaller chunks mean more owners, each polling fewer
// bytes per round; on the 20000 x 2000 workload 1 is fastest (2: +4%, 4: +3%, 8: +13% per
// iteration).
constexpr int kChunk = 1;
static_assert(kChunk == 1 || kChunk == 2 || kChunk == 4 || kChunk == 8, "chunk of 1, 2, 4 or 8 entries");
constexpr int kCopies = kGridSumCopies;     // copies of the reduced vector

template <int N>
struct Count {
  static constexpr int value = N;
};

__device__ __forceinline__ unsigned long long ld_u64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Workgroup-scope load: served by the caches, so it may return an out-of-date value; used only
// for epoch-tagged data, whose tag exposes an out-of-date value.
__device__ __forceinline__ unsigned long long ld_u64_cached(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st_u64(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A value published for one epoch: two 64-bit atomic words, each carrying the 32-bit epoch next
// to one half of the FP64 bit pattern.  A reader accepts the pair only when both words carry the
// epoch it waits for, so it never takes a stale value or a pair torn between two epochs; no fence
// or counter is needed to order the data with its arrival.  A vector of tagged values is stored
// in chunks of kChunk entries, each a run of 2 kChunk words: the first words of the entries in
// entry order, then their second words in reverse order, so that the word pairs of a run sit
// mirror-symmetrically and lane p of a run finds its partner in lane 2 kChunk - 1 - p.
__device__ __forceinline__ int tag_word(int e, int plane) {
  const int j = e % kChunk, run = (e / kChunk) * 2 * kChunk;
  return plane == 0 ? run + j : run + 2 * kChunk - 1 - j;
}
__device__ __forceinline__ void st_tagged(unsigned long long* p, int e, double v, unsigned epoch) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  st_u64(p + tag_word(e, 0), ((unsigned long long)epoch << 32) | (bits >> 32));
  st_u64(p + tag_word(e, 1), (bits << 32) | (unsigned long long)epoch);
}
__device__ __forceinline__ bool tag_ok(unsigned long long w0, unsigned long long w1, unsigned epoch) {
  return (unsigned)(w0 >> 32) == epoch && (unsigned)w1 == epoch;
}
__device__ __forceinline__ double tag_value(unsigned long long w0, unsigned long long w1) {
  return __longlong_as_double((long long)((w0 << 32) | (w1 >> 32)));
}

// Wait until every memory operation this wave issued has completed (including copies into LDS);
// the memory clobber keeps the compiler from moving accesses across.
__device__ __forceinline__ void wait_mem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

struct GridLayout {
  int NR, NC;     // max rows / columns owned by one workgroup
  size_t dbl;     // doubles before the panel slabs
  size_t slabC;   // panel elements of one column-slab buffer
  size_t slabR;   // panel elements of one row-slab buffer
};

// Workgroup w of G owns entries [own_lo(w), own_lo(w + 1)) of a dimension of size `total`: the
// boundaries w * total / G rounded down to a multiple of `al`, so that the panel runs a workgroup
// copies start on 16-byte boundaries (rows: al = 16 / panel bytes, as column panels have a row
// stride of a multiple of 16 entries; columns: al = 8, so that the offset c * |I| of a row slab is a
// multiple of 16 bytes for any block size).  A part holds at most ceil(total / G) + al entries.
constexpr int kColOwnAlign = 8;
__host__ __device__ inline int64_t own_lo(int64_t w, int64_t total, int G, int al) {
  return w >= G ? total : (w * total / G) / al * al;
}

// row_lds: the row slabs are staged in LDS (else the x-steps read them from the row panels in HBM,
// for systems whose slabs do not fit).  esz: bytes per panel entry.
__host__ __device__ inline GridLayout grid_layout(int64_t m, int64_t n, int max_nI, int max_nJ, int G, int threads,
                                                  bool row_lds, int esz) {
  GridLayout L;
  L.NR = (int)((m + G - 1) / G) + 16 / esz;
  L.NC = (int)((n + G - 1) / G) + kColOwnAlign;
  // an even count of doubles keeps the slab buffers after them 16-byte aligned
  L.dbl = (4 * (size_t)L.NR + 2 * (size_t)L.NC + (size_t)max_nJ + (size_t)max_nI + (size_t)threads + 8 + 1) & ~(size_t)1;
  // slab buffers padded to 8 entries, so every buffer starts 16-byte aligned in LDS
  L.slabC = ((size_t)L.NR * max_nJ + 7) / 8 * 8;
  L.slabR = row_lds ? ((size_t)L.NC * max_nI + 7) / 8 * 8 : 0;
  return L;
}

// Largest power of two <= x, clamped to [1, 64] (lanes that cooperate on one dot product).
__device__ __forceinline__ int lanes_per_item(int threads, int items) {
  int q = items > 0 ? threads / items : threads;
  int p = 1;
  while (p * 2 <= q && p < 64) p *= 2;
  return p;
}

// Data-parallel-primitive lane exchange of an FP64 value (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false));
}
// The word held by the mirror lane of this lane's run of 2 kChunk lanes (lane p <-> 2 kChunk - 1 - p):
// a data-parallel-primitive move (row mirror for runs of 16, half-row mirror for 8, reversed quad
// for 4, swapped pairs for 2).
__device__ __forceinline__ unsigned long long mirror_word(unsigned long long x) {
  constexpr int ctrl = kChunk == 8 ? 0x140 : (kChunk == 4 ? 0x141 : (kChunk == 2 ? 0x1B : 0xB1));
  const int lo = (int)(unsigned)x, hi = (int)(unsigned)(x >> 32);
  const unsigned nlo = (unsigned)__builtin_amdgcn_update_dpp(0, lo, ctrl, 0xF, 0xF, false);
  const unsigned nhi = (unsigned)__builtin_amdgcn_update_dpp(0, hi, ctrl, 0xF, 0xF, false);
  return ((unsigned long long)nhi << 32) | nlo;
}
// Sum over aligned groups of `width` lanes (a power of two <= 64); every lane of a group gets the
// group's sum.  Quad permutations, half-row and row mirrors stay inside a row of 16 lanes.
__device__ __forceinline__ double group_sum(double v, int width) {
  if (width >= 2) v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  if (width >= 4) v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  if (width >= 8) v += dpp_f64<0x141>(v);   // row_half_mirror
  if (width >= 16) v += dpp_f64<0x140>(v);  // row_mirror
  if (width >= 32) v += __shfl_xor(v, 16, 64);
  if (width >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

constexpr int kRing = 128;  // block draws kept ahead (relative iteration q in slot (q - 1) & 127)

// Whether `runs` runs of `len` panel elements (run r at src + r * stride, landing at dst + r * len)
// are whole 4-byte-aligned dwords at both ends, as the LDS copy below needs (always true for 4- and
// 8-byte panels; for 2-byte panels it depends on the offsets).  The same for every thread.
template <typename TP>
__device__ __forceinline__ bool dma_ok(const TP* src, int64_t stride, int runs, int len, const TP* dst) {
  if (sizeof(TP) >= 4 || runs <= 0) return true;
  return (((uintptr_t)src | (uintptr_t)dst) & 3) == 0 && (len & 1) == 0 && (runs == 1 || (stride & 1) == 0);
}

// Copy those runs into LDS.  Waves 1..3 issue global_load_lds copies, the pieces of all runs spread
// over the three waves: 1-KB pieces (16 bytes per lane) when every run starts and ends on 16-byte
// boundaries at both ends, else 256-byte pieces (one dword per lane).  Lane l of a copy lands at
// the copy's LDS address + l x (bytes per lane).  The copies are asynchronous and complete for
// the issuing wave after s_waitcnt vmcnt(0).
template <typename TP>
__device__ __forceinline__ void dma_runs(const TP* src, int64_t stride, int runs, int len, TP* dst) {
  const int wave = (int)(threadIdx.x >> 6) - 1, lane = (int)(threadIdx.x & 63);
  const int bytes = len * (int)sizeof(TP);
  const bool wide = ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0) && (bytes & 15) == 0 &&
                    (runs <= 1 || ((stride * (int64_t)sizeof(TP)) & 15) == 0);
  const int per_lane = wide ? 16 : 4, piece = 64 * per_lane;
  const int pieces = (bytes + piece - 1) / piece;
  const int total = runs * pieces;
  for (int p = wave; p < total; p += 3) {
    const int r = p / pieces, off = (p - r * pieces) * piece;
    const char* s = (const char*)(src + (int64_t)r * stride);
    char* d = (char*)(dst + (size_t)r * len);
    if (off + lane * per_lane < bytes) {
      if (wide)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(s + off + lane * 16),
                                         (__attribute__((address_space(3))) void*)(d + off), 16, 0, 0);
      else
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(s + off + lane * 4),
                                         (__attribute__((address_space(3))) void*)(d + off), 4, 0, 0);
    }
  }
}

template <typename TP, bool RowLds>
__global__ void __launch_bounds__(kGridThreads) grid_solve_kernel(SolveArgs a, GridSync gs) {
  extern __shared__ double lds[];
  // per-draw metadata: blocks, their sizes, panel offsets and step coefficients
  __shared__ int s_j[kRing], s_i[kRing], s_nJ[kRing], s_nI[kRing];
  __shared__ int64_t s_c0[kRing], s_r0[kRing];
  __shared__ double s_cc[kRing], s_cr[kRing];
  __shared__ int s_ok;
  __shared__ double s_red[(kGridThreads / 64) * kChunk];
  __shared__ double s_err2;
  const int G = gridDim.x, w = blockIdx.x, tid = threadIdx.x, T = blockDim.x;
  const int64_t m = a.m, n = a.n;
  const int MJ = a.max_nJ, MI = a.max_nI;
  const GridLayout L = grid_layout(m, n, MI, MJ, G, T, RowLds, (int)sizeof(TP));
  const int ra = 16 / (int)sizeof(TP);
  const int64_t r0 = own_lo(w, m, G, ra), r1 = own_lo(w + 1, m, G, ra);
  const int64_t cA = own_lo(w, n, G, kColOwnAlign), cB = own_lo(w + 1, n, G, kColOwnAlign);
  const int nr = (int)(r1 - r0), nc = (int)(cB - cA);

  double* z = lds;          // z on owned rows
  double* zp = z + L.NR;    // previous z (returned when the stop rule fires one iteration late)
  double* bl = zp + L.NR;   // b on owned rows
  double* x = bl + L.NR;    // x on owned columns
  double* xr = x + L.NC;    // x_ref on owned columns
  double* v = xr + L.NC;    // reduced A_{:,J}^T z
  double* u = v + MJ;       // reduced A_{I,:} x - b_I + z_I
  double* yv = u + MI + T + 8;  // y on owned rows (refinement), after the reduction scratch
  TP* slabC = (TP*)(lds + L.dbl);
  TP* slabR = slabC + 2 * L.slabC;

  const TP* __restrict__ Arow = (const TP*)a.Arow;
  const TP* __restrict__ Acol = (const TP*)a.Acol;
  const int E = gs.stride;
  const int NCH = E / kChunk;  // reduction chunks; workgroup c owns chunks c, c + G, ...
  const int err_slot = MJ + MI;
  const int64_t K = a.max_iter;
  const int64_t ce = a.check_every > 0 ? a.check_every : 1;
  const bool checking = a.x_ref != nullptr && a.tol > 0.0;
  const int kHalf = T / 2;  // waves 0-1: z side, waves 2-3: x side

  for (int q = tid; q < nr; q += T) {
    z[q] = a.z_in ? a.z_in[r0 + q] : a.b[r0 + q];
    zp[q] = z[q];
    bl[q] = a.b[r0 + q];
  }
  for (int q = tid; q < nc; q += T) {
    x[q] = a.x_in ? a.x_in[cA + q] : 0.0;
    xr[q] = a.x_ref ? a.x_ref[cA + q] : 0.0;
  }
  for (int q = tid; q < nr; q += T) yv[q] = 0.0;

  auto refill = [&](int64_t first) {  // draws of relative iterations first .. first+63
    if (tid < 64) {
      const int64_t q = first + tid;
      if (q <= K) {
        int jj, ii;
        draw_pair(a, a.k0 + q, jj, ii);
        const int sl = (int)((q - 1) & (kRing - 1));
        s_j[sl] = jj;
        s_i[sl] = ii;
        s_c0[sl] = a.col_off[jj];
        s_nJ[sl] = (int)(a.col_off[jj + 1] - a.col_off[jj]);
        s_r0[sl] = a.row_off[ii];
        s_nI[sl] = (int)(a.row_off[ii + 1] - a.row_off[ii]);
        s_cc[sl] = a.coef_col[jj];
        s_cr[sl] = a.coef_row[ii];
      }
    }
  };
  auto slot = [&](int64_t q) -> int { return (int)((q - 1) & (kRing - 1)); };
  refill(1);
  refill(65);
  __syncthreads();
  int64_t filled_to = 128;

  // Column slab: nJ runs of nr elements (column panels hold A^T), stored run after run in LDS, so
  // entry (q, c) of the slab sits at c * nr + q.  Row slab: one run of nc * nI elements, entry
  // (l, c) at c * nI + l.
  struct Src {
    const TP* c;
    int runs;
    const TP* r;
    int lr;
  };
  auto slab_src = [&](int64_t qc, int64_t qr) -> Src {
    Src sr{nullptr, 0, nullptr, 0};
    if (qc >= 1 && nr > 0) {
      const int sl = slot(qc);
      sr.c = Acol + a.ldc * s_c0[sl] + r0;
      sr.runs = s_nJ[sl];
    }
    if (RowLds && qr >= 1 && nc > 0) {
      const int sl = slot(qr);
      sr.r = Arow + n * s_r0[sl] + cA * s_nI[sl];
      sr.lr = nc * s_nI[sl];
    }
    return sr;
  };
  // row slab of iteration q (owned columns of row block I_q, column-major nc x |I_q|): in LDS
  // buffer `buf`, or straight from the row panel
  auto row_src = [&](int64_t q, int buf) -> const TP* {
    if constexpr (RowLds) {
      (void)q;
      return slabR + (size_t)buf * L.slabR;
    } else {
      (void)buf;
      const int sl = slot(q);
      return Arow + n * s_r0[sl] + cA * s_nI[sl];
    }
  };
  // refinement: v^{q} -= g_J (the z-step then projects onto {A^T z = g}); all threads call it
  auto apply_g = [&](int64_t q) {
    if (a.g == nullptr || q < 1 || q > K) return;
    const int sl = slot(q);
    const int64_t c0 = s_c0[sl];
    for (int c = tid; c < s_nJ[sl]; c += T) v[c] -= a.g[c0 + c];
    __syncthreads();
  };
  // refinement: y_I -= coef_I u^q on the owned rows of I_q (the x-step is x -= A_I^T (coef_I u))
  auto yupdate = [&](int64_t q, int lt, int nt) {
    const int sl = slot(q);
    const int64_t rI = s_r0[sl], rE = rI + s_nI[sl];
    const int64_t lo = rI > r0 ? rI : r0, hi = rE < r1 ? rE : r1;
    const double cr = s_cr[sl];
    for (int64_t l = lo + lt; l < hi; l += nt) yv[l - r0] -= cr * u[l - rI];
  };
  auto copy_plain = [&](const Src& sr, TP* dC, TP* dR) {  // every thread, ordinary loads; NULL: skip
    if (dC)
      for (int e = tid; e < sr.runs * nr; e += T) {
        const int c = e / nr, q = e - c * nr;
        dC[e] = sr.c[(int64_t)c * a.ldc + q];
      }
    if (dR)
      for (int e = tid; e < sr.lr; e += T) dR[e] = sr.r[e];
  };

  // One grid-wide reduction of this round's partial vectors (entries [0, nq), [MJ, MJ + np) and,
  // with has_err, err_slot; every workgroup has published them tagged with `epoch`), in two
  // steps, while waves 1..3 copy the next round's slabs (column slab of iteration qc into column
  // buffer bufC, row slab of iteration qr into row buffer bufR) straight into LDS.
  //   1. Workgroup c owns chunk c (and c + G, ...) of the vectors: all its waves poll that chunk of
  //      every workgroup's partial vector (2 kChunk lanes read one workgroup's run), add the G
  //      partials in a fixed order (per lane over its workgroups, across the lane groups of the
  //      wave, then across the waves) and publish the tagged sums in kCopies copies.  Owners
  //      start their slab copies afterwards: a wave's loads complete in order, so polls issued
  //      behind the copies would wait for them.
  //   2. Wave 0 of every workgroup reads the reduced vector from copy w mod kCopies into v, u and
  //      s_err2; the copies spread the readers over more memory channels.
  // Returns false after a spin-limit timeout.
  auto need = [&](int e, int nq, int np, bool has_err) -> bool {
    return e < nq || (e >= MJ && e < MJ + np) || (has_err && e == err_slot);
  };
  constexpr int K2 = 2 * kChunk;  // lanes (words) per chunk run
  const int p2 = tid & (K2 - 1);  // this lane's word in a run
  const bool first = p2 < kChunk;  // lane holds a first word; its entry is p2 (else K2 - 1 - p2)
  const int je = first ? p2 : K2 - 1 - p2;
  auto sync_round = [&](unsigned epoch, int par, int nq, int np, bool has_err, int64_t qc, int bufC, int64_t qr,
                        int bufR) -> bool {
    int ok = 1;
    if (tid == 0) s_ok = 1;  // (the previous reader of s_ok passed a barrier since)
    unsigned spins = 0;
    auto give_up = [&]() -> bool {  // bounded waiting; true when this thread must stop waiting
      if ((++spins & 63u) == 0) {
        if (__hip_atomic_load(gs.timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
        if (spins > kSpinLimit) {
          __hip_atomic_store(gs.timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          return true;
        }
      }
      return false;
    };
    // Poll N runs per lane (run k at addr(k), this lane's word p2) until every value marked in
    // `pending` carries the epoch; vals[k] receives this lane's entry of run k.  The whole wave
    // runs the loop: the lanes of a run exchange words.
    auto poll_runs = [&](auto count, auto addr, unsigned pending, double* vals) {
      constexpr int N = decltype(count)::value;
      while (ok) {
        unsigned long long wd[N];
#pragma unroll
        for (int k = 0; k < N; ++k) wd[k] = ld_u64(addr(k) + p2);
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const unsigned long long o = mirror_word(wd[k]);
          const unsigned long long w0 = first ? wd[k] : o, w1 = first ? o : wd[k];
          if (((pending >> k) & 1u) && tag_ok(w0, w1, epoch)) {
            vals[k] = tag_value(w0, w1);
            pending &= ~(1u << k);
          }
        }
        if (!__any(pending != 0)) break;
        if (give_up()) ok = 0;
      }
    };
    const bool any = nq > 0 || np > 0 || has_err;
    const Src sr = slab_src(qc, qr);
    TP* dC = slabC + (size_t)bufC * L.slabC;
    TP* dR = RowLds ? slabR + (size_t)bufR * L.slabR : slabR;
    const bool okC = dma_ok(sr.c, a.ldc, sr.runs, nr, dC);
    const bool okR = dma_ok(sr.r, 0, sr.lr > 0 ? 1 : 0, sr.lr, dR);
    auto start_copies = [&]() {  // waves 1..3: the next slabs, straight into LDS
      if (tid >= 64) {
        if (okC) dma_runs(sr.c, a.ldc, sr.runs, nr, dC);
        if (okR) dma_runs(sr.r, 0, sr.lr > 0 ? 1 : 0, sr.lr, dR);
      }
    };
    const bool owner = any && w < NCH;
    if (!owner) start_copies();
    const int lane = tid & 63;
    const size_t V2 = (size_t)E * 2;
    unsigned long long* Sring = gs.gsum + (size_t)(epoch % kGridSumRing) * kCopies * V2;
    if (owner) {
      const unsigned long long* P = gs.part + (size_t)par * G * V2;
      constexpr int kRuns = K2;                // runs per lane per pass
      const int rows = T / K2, row = tid / K2;  // workgroups read per load step of the workgroup
      for (int c = w; c < NCH; c += G) {  // uniform over the workgroup
        const int e0 = c * kChunk;
        bool chunk_needed = false;
        for (int j = 0; j < kChunk; ++j) chunk_needed |= need(e0 + j, nq, np, has_err);
        if (!chunk_needed) continue;
        const bool mine = first && need(e0 + je, nq, np, has_err);
        double acc = 0.0;
        for (int mb0 = 0; mb0 < G; mb0 += kRuns * rows) {
          unsigned pending = 0;
#pragma unroll
          for (int k = 0; k < kRuns; ++k)
            if (mine && mb0 + k * rows + row < G) pending |= 1u << k;
          double vals[kRuns];
          poll_runs(Count<kRuns>{}, [&](int k) {
            int mb = mb0 + k * rows + row;
            mb = mb < G ? mb : G - 1;
            return P + (size_t)mb * V2 + (size_t)c * K2;
          }, pending, vals);
#pragma unroll
          for (int k = 0; k < kRuns; ++k)
            if (mine && mb0 + k * rows + row < G) acc += vals[k];
        }
        // lanes p2 < kChunk hold entry e0 + p2 summed over their workgroups: add the lane groups
        // of the wave (butterfly: every lane gets the same sum), then the waves in order
#pragma unroll
        for (int o = K2; o < 64; o *= 2) acc += __shfl_xor(acc, o, 64);
        if (lane < kChunk) s_red[(tid >> 6) * kChunk + lane] = acc;
        __syncthreads();
        if (tid < kChunk * kCopies) {
          const int j = tid % kChunk, cp = tid / kChunk;
          if (need(e0 + j, nq, np, has_err)) {
            double t = 0.0;
            for (int q = 0; q < (T >> 6); ++q) t += s_red[q * kChunk + j];
            st_tagged(Sring + (size_t)cp * V2, e0 + j, t, epoch);
          }
        }
        __syncthreads();
      }
      start_copies();
    }
    // step 2 (wave 0): the reduced vector, 64 / K2 chunks per load instruction
    if (tid < 64 && any) {
      const unsigned long long* Sg = Sring + (size_t)(w % kCopies) * V2;
      constexpr int kPer = 64 / K2;  // chunks per load instruction
      const int r = lane / K2;
      for (int cb = 0; cb < NCH; cb += 8 * kPer) {  // up to 8 load instructions per pass
        unsigned pending = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int c = cb + kPer * k + r;
          if (c < NCH && first && need(c * kChunk + je, nq, np, has_err)) pending |= 1u << k;
        }
        double vals[8];
        poll_runs(Count<8>{}, [&](int k) {
          int c = cb + kPer * k + r;
          c = c < NCH ? c : NCH - 1;
          return Sg + (size_t)c * K2;
        }, pending, vals);
        if (ok && first) {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int c = cb + kPer * k + r;
            const int e = c * kChunk + je;
            if (c < NCH && need(e, nq, np, has_err)) {
              if (e < MJ) v[e] = vals[k];
              else if (e < MJ + MI) u[e - MJ] = vals[k];
              else s_err2 = vals[k];
            }
          }
        }
      }
    }
    // slabs of 2-byte panels that are not whole aligned dwords are copied with ordinary loads;
    // then wait for the copies this wave started
    if (!okC || !okR) copy_plain(sr, okC ? nullptr : dC, okR ? nullptr : dR);
    wait_mem();
    if (!ok) s_ok = 0;
    __syncthreads();
    const bool all_ok = s_ok != 0;
    return all_ok;
  };

  // The steps below run on threads [t0, t0 + nt) of the workgroup (whole waves), given as the
  // local index lt = tid - t0 and nt: in the iteration loop the z-side steps run on waves 0-1 and
  // the x-side steps on waves 2-3, at the same time.
  // z <- z - coef * A_{R,J} v on owned rows (slab entry (q, c) at c * nr + q); keeps the previous z.
  auto zupdate = [&](const TP* Sl, int nJ, double coef, int lt, int nt) {
    for (int q = lt; q < nr; q += nt) {
      const TP* row = Sl + q;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0, a5 = 0.0, a6 = 0.0, a7 = 0.0;
      int c = 0;
      for (; c + 7 < nJ; c += 8) {  // eight independent chains
        a0 += widen(row[(c + 0) * nr]) * v[c + 0];
        a1 += widen(row[(c + 1) * nr]) * v[c + 1];
        a2 += widen(row[(c + 2) * nr]) * v[c + 2];
        a3 += widen(row[(c + 3) * nr]) * v[c + 3];
        a4 += widen(row[(c + 4) * nr]) * v[c + 4];
        a5 += widen(row[(c + 5) * nr]) * v[c + 5];
        a6 += widen(row[(c + 6) * nr]) * v[c + 6];
        a7 += widen(row[(c + 7) * nr]) * v[c + 7];
      }
      for (; c < nJ; ++c) a0 += widen(row[c * nr]) * v[c];
      a0 += a4;
      a1 += a5;
      a2 += a6;
      a3 += a7;
      zp[q] = z[q];
      z[q] -= coef * ((a0 + a1) + (a2 + a3));
    }
  };
  // x <- x - coef * A_{I,C}^T u on owned columns (column-major slab nc x nI)
  auto xupdate = [&](const TP* Sl, int nI, double coef, int lt, int nt) {
    const int tpc = lanes_per_item(nt, nc);  // lanes per owned column
    const int cp = nt / tpc, sub = lt % tpc;
    for (int c0 = 0; c0 < nc; c0 += cp) {
      const int cc = c0 + lt / tpc;
      double acc = 0.0;
      if (cc < nc) {
        const TP* col = Sl + (size_t)cc * nI;
        if constexpr (RowLds) {
#pragma unroll 4
          for (int l = sub; l < nI; l += tpc) acc += widen(col[l]) * u[l];
        } else {  // from HBM: more loads in flight
#pragma unroll 16
          for (int l = sub; l < nI; l += tpc) acc += widen(col[l]) * u[l];
        }
      }
      acc = group_sum(acc, tpc);
      if (cc < nc && sub == 0) x[cc] -= coef * acc;
    }
  };
  // publish A_{R,J}^T z over owned rows (slab entry (q, c) at c * nr + q) as entries [0, nJ):
  // tq lanes per column, partial sums meet with lane exchanges
  auto push_q = [&](const TP* Sl, int nJ, unsigned long long* P, unsigned ep, int lt, int nt) {
    const int tq = lanes_per_item(nt, nJ), per = nt / tq, sub = lt % tq;
    for (int c0 = 0; c0 < nJ; c0 += per) {
      const int c = c0 + lt / tq;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      if (c < nJ) {
        const TP* col = Sl + (size_t)c * nr;
        int q = sub;
        for (; q + 3 * tq < nr; q += 4 * tq) {  // four independent chains
          a0 += widen(col[q]) * z[q];
          a1 += widen(col[q + tq]) * z[q + tq];
          a2 += widen(col[q + 2 * tq]) * z[q + 2 * tq];
          a3 += widen(col[q + 3 * tq]) * z[q + 3 * tq];
        }
        for (; q < nr; q += tq) a0 += widen(col[q]) * z[q];
      }
      const double acc = group_sum((a0 + a1) + (a2 + a3), tq);
      if (c < nJ && sub == 0) st_tagged(P, c, acc, ep);
    }
  };
  // partial error ||x - x_ref||^2 over owned columns (one whole wave calls it)
  auto err_partial = [&](unsigned long long* P, unsigned ep) {
    const int lane = tid & 63;
    double e = 0.0;
    for (int cc = lane; cc < nc; cc += 64) {
      const double d = x[cc] - xr[cc];
      e += d * d;
    }
    int width = 1;
    while (width < nc && width < 64) width *= 2;
    e = group_sum(e, width);
    if (lane == 0) st_tagged(P, err_slot, e, ep);
  };

  unsigned epoch = 0;
  int status = 0, stopped = 0;
  int64_t last_k = a.k0;
  double last_err2 = -1.0;
  int64_t last_check = -1;
  bool alive = true;

  // ---------------- prologue: partial sums of v^1 = A_{:,J_1}^T z^0
  {
    TP* d1 = slabC + 1 * L.slabC;  // the column slab of iteration q lives in buffer q & 1
    copy_plain(slab_src(1, 0), d1, nullptr);
    __syncthreads();
    const int nJ1 = s_nJ[slot(1)];
    push_q(d1, nJ1, gs.part + (size_t)w * E * 2, epoch + 1, tid, T);
    alive = sync_round(++epoch, 0, nJ1, 0, false, K >= 2 ? 2 : 0, 0, 1, 1);
    if (alive) apply_g(1);
  }

  int64_t rr = 1;
  for (; alive && rr <= K; ++rr) {
    const int64_t k = a.k0 + rr;
    if (rr + 34 > filled_to && filled_to < K) {
      refill(filled_to + 1);
      filled_to += 64;
      __syncthreads();
    }
    const int sk = slot(rr);
    const int nJk = s_nJ[sk], nIk = s_nI[sk];
    const int nIp = rr >= 2 ? s_nI[slot(rr - 1)] : 0;
    const int nJn = rr < K ? s_nJ[slot(rr + 1)] : 0;
    if (w == 0 && tid == 0 && a.trace_j) {
      a.trace_j[rr - 1] = s_j[sk];
      a.trace_i[rr - 1] = s_i[sk];
    }

    // phase A: z^k on owned rows (column slab of J_k); x^{k-1} on owned columns (row slab of I_{k-1})
    if (tid < kHalf) {
      zupdate(slabC + (size_t)(rr & 1) * L.slabC, nJk, s_cc[sk], tid, kHalf);
    } else {
      const int lt = tid - kHalf, nt = T - kHalf;
      if (nIp > 0 && nc > 0) xupdate(row_src(rr - 1, (int)((rr - 1) & 1)), nIp, s_cr[slot(rr - 1)], lt, nt);
      if (nIp > 0 && a.y_out) yupdate(rr - 1, lt, nt);
    }
    __syncthreads();
    // phase B: this workgroup's partial vector: A_{:,J_{k+1}}^T z^k (row groups), A_{I_k,C} x^{k-1}
    // + (z^k - b) on owned rows of I_k, and ||x^{k-1} - x_ref||^2
    unsigned long long* P = gs.part + ((size_t)(rr & 1) * G + w) * E * 2;
    const unsigned ep = epoch + 1;
    const bool has_err = checking && rr >= 2 && ((rr - 1) % ce == 0);
    if (tid < kHalf) {
      if (nJn > 0) push_q(slabC + (size_t)((rr + 1) & 1) * L.slabC, nJn, P, ep, tid, kHalf);
    } else {
      const TP* Sr = row_src(rr, (int)(rr & 1));
      const int64_t rI = s_r0[sk];
      for (int l = tid - kHalf; l < nIk; l += T - kHalf) {
        double acc = 0.0;
        if constexpr (RowLds) {
#pragma unroll 4
          for (int cc = 0; cc < nc; ++cc) acc += widen(Sr[cc * nIk + l]) * x[cc];
        } else {  // from HBM: more loads in flight
#pragma unroll 16
          for (int cc = 0; cc < nc; ++cc) acc += widen(Sr[cc * nIk + l]) * x[cc];
        }
        const int64_t gl = rI + l;
        if (gl >= r0 && gl < r1) acc += z[gl - r0] - bl[gl - r0];
        st_tagged(P, MJ + l, acc, ep);
      }
      if (has_err && tid >= T - 64) err_partial(P, ep);  // wave 3
    }
    alive = sync_round(++epoch, (int)(rr & 1), nJn, nIk, has_err, rr + 2 <= K ? rr + 2 : 0, (int)(rr & 1),
                       rr + 1 <= K ? rr + 1 : 0, (int)((rr + 1) & 1));
    if (!alive) break;
    if (nJn > 0) apply_g(rr + 1);
    // v = v^{k+1}, u = u^k, s_err2 = ||x^{k-1} - x_ref||^2
    if (has_err) {
      const double e2 = s_err2;
      last_err2 = e2;
      last_check = k - 1;
      const double rel = sqrt(e2) / sqrt(a.xref_sq);
      if (rel < a.tol || !isfinite(e2) || rel > 1e6) {
        stopped = 1;
        status = rel < a.tol ? 0 : 2;
        last_k = k - 1;
        for (int q = tid; q < nr; q += T) z[q] = zp[q];  // z^{k-1}
        __syncthreads();
        break;
      }
    }
  }

  if (alive && !stopped) {
    // epilogue: x^K from u^K, then the error of x^K
    const int sK = slot(K);
    if (nc > 0) xupdate(row_src(K, (int)(K & 1)), s_nI[sK], s_cr[sK], tid, T);
    if (a.y_out) yupdate(K, tid, T);
    __syncthreads();
    last_k = a.k0 + K;
    if (a.x_ref != nullptr) {
      const int par = (int)((K + 1) & 1);
      if (tid < 64) err_partial(gs.part + ((size_t)par * G + w) * E * 2, epoch + 1);
      alive = sync_round(++epoch, par, 0, 0, true, 0, 0, 0, 0);
      if (alive) {
        last_err2 = s_err2;
        last_check = a.k0 + K;
        if (checking) {
          const double rel = sqrt(last_err2) / sqrt(a.xref_sq);
          if (rel < a.tol) {
            stopped = 1;
            status = 0;
          } else if (!isfinite(last_err2) || rel > 1e6) {
            stopped = 1;
            status = 2;
          } else {
            status = 1;
          }
        }
      }
    }
  }

  for (int q = tid; q < nr; q += T)
    if (a.z_out) a.z_out[r0 + q] = z[q];
  for (int q = tid; q < nc; q += T) a.x_out[cA + q] = x[q];
  if (a.y_out)
    for (int q = tid; q < nr; q += T) a.y_out[r0 + q] = yv[q];
  if (w == 0 && tid == 0) {
    a.status->status = alive ? status : -4;
    a.status->stopped = stopped;
    a.status->last_k = last_k;
    a.status->err2 = last_err2;
    a.status->check_k = last_check;
  }
}

}  // namespace

size_t grid_solve_lds_bytes(const SolveArgs& a, int grid, int panel_dtype, bool row_lds) {
  const size_t esz = panel_dtype == 0 ? 8 : (panel_dtype == 1 ? 4 : 2);
  const GridLayout L = grid_layout(a.m, a.n, a.max_nI, a.max_nJ, grid, kGridThreads, row_lds, (int)esz);
  return L.dbl * sizeof(double) + 2 * (L.slabC + L.slabR) * esz + 64;
}

template <typename TP>
const void* grid_kernel_ptr(bool row_lds) {
  return row_lds ? (const void*)grid_solve_kernel<TP, true> : (const void*)grid_solve_kernel<TP, false>;
}

hipError_t grid_solve_max_blocks(int panel_dtype, size_t lds_bytes, bool row_lds, int* blocks_per_cu) {
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const void* k = grid_kernel_ptr<TP>(row_lds);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, kGridThreads, lds_bytes);
  });
}

hipError_t launch_grid_solve(const SolveArgs& a, const GridSync& gs, int panel_dtype, int grid, bool row_lds,
                             hipStream_t st) {
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const void* k = grid_kernel_ptr<TP>(row_lds);
    const size_t lds = grid_solve_lds_bytes(a, grid, panel_dtype, row_lds);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    SolveArgs aa = a;
    GridSync gg = gs;
    void* args[] = {&aa, &gg};
    return hipLaunchCooperativeKernel(k, dim3(grid), dim3(kGridThreads), args, (unsigned)lds, st);
  });
}

}  // namespace rebk
