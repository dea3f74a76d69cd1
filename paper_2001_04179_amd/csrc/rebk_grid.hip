// Persistent cooperative REBK kernels for gfx950 (Du, Si, Sun, arXiv:2001.04179, Algorithm 1): the
// grid kernel below, and after it the pipelined kernel (one broadcast hop per iteration).
//
// Ownership: workgroup w owns rows [w*m/G, (w+1)*m/G) of z and columns [w*n/G, (w+1)*n/G) of x,
// each boundary rounded down to 16 bytes of panel entries (rows) or 8 columns (own_lo); both stay
// in LDS for the whole launch.  One grid-wide reduction per iteration carries
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
// Workgroup barrier that waits only for this wave's LDS operations: copies into LDS still in
// flight keep going (their waves wait for them with wait_mem before the data is read).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

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

// ---------------------------------------------------------------------------------------------
// Pipelined whole-chip kernel: one broadcast hop per iteration on the critical path.
//
// The x-step of iteration t needs A_{I_t} x^{t-1}, and x^{t-1} = x^{t-3} - c_{t-2} A_{I_{t-2}}^T u^{t-2}
// - c_{t-1} A_{I_{t-1}}^T u^{t-1}, so
//   u^t = [A_{I_t} x^{t-3} - b_{I_t} + z^{t-2}_{I_t}] - c_{t-2} G_{I_t,I_{t-2}} u^{t-2} - c_{t-1} G_{I_t,I_{t-1}} u^{t-1}
//         - c'_{t-1} A_{I_t,J_{t-1}} v^{t-1} - c'_t A_{I_t,J_t} v^t,
// and likewise v^{t+1} = [A_{J_{t+1}}^T z^{t-2}] - c'_{t-1} H_{J_{t+1},J_{t-1}} v^{t-1} - c'_t H_{J_{t+1},J_t} v^t,
// with G = A A^T and H = A^T A (FP64, in HBM) and c, c' the row and column step coefficients.  The
// iterates are Algorithm 1's; only the order of the sums differs from the oracle's.
//
// Round t broadcasts B^t = (v^{t+1}, u^t) (and, when a check is due, ||x^{t-3} - x_ref||^2), one
// entry per owning workgroup.  An entry is P^t (the bracket, summed over workgroups: partial sums
// of state two and three iterations old) minus w'_t . B^{t-2} minus w_t . B^{t-1}, where w'_t and
// w_t are the scaled rows of H, G and A above, laid out like B.  Every owner of an entry in use
// publishes it every round (zero when no one reads it).  Wave 0 of the owner reads w_t and
// w'_{t+1} from LDS while its poll of B^{t-1} is in flight; as soon as the poll is complete it forms
// its entry of B^t and publishes it, with no workgroup barrier in between, then hands B^{t-1} to
// the other waves.  Those waves, one round behind, update z and x, publish the partial sums of
// round t + 2, gather the owner's sum of round t + 1 and stage the slabs and the scaled rows of
// later rounds through registers.
constexpr int kPipeSlabs = 5;   // slab buffers of each kind (a slab is read in two rounds three apart)
constexpr int kPipeParts = 4;   // partial vectors kept per workgroup (round t in slot t & 3)
// dwords a helper lane holds in flight per round (the rest: direct copies); with FP64 panels more
// than this pushes the kernel past 256 VGPRs into scratch
template <typename TP>
constexpr int pipe_stage() {
  return 32;
}
static_assert(kPipeMaxStride == 256, "wave 0 holds a broadcast vector in 8 registers per lane pair");

struct PipeLayout {
  int NR, NC;
  int NRS;        // LDS run length of a column-slab run (owned rows rounded up to 16 bytes)
  size_t dbl;     // doubles before the slabs
  size_t slabC, slabR;
};

__host__ __device__ inline PipeLayout pipe_layout(int64_t m, int64_t n, int MI, int MJ, int E, int G, int esz) {
  PipeLayout L;
  // the most rows / columns a workgroup owns: inner ownership boundaries are multiples of al
  // rounded down from floor(w total / G), so two inner ones lie at most al ceil(ceil(total / G) / al)
  // apart; the last range ends at total itself
  auto most = [G](int64_t total, int al) -> int {
    const int64_t q = (total + G - 1) / G;
    const int64_t inner = (q + al - 1) / al * al, last = total - own_lo(G - 1, total, G, al);
    return (int)(inner > last ? inner : last);
  };
  L.NR = most(m, 16 / esz);
  L.NC = most(n, kColOwnAlign);
  L.NRS = L.NR + 16 / esz;
  // z history (4 NR), b (NR), x history (4 NC), x_ref (NC), three broadcast vectors, the scaled
  // vectors W_t and W'_t (two of each), two gathered sums; an even count keeps the slabs 16-byte
  // aligned
  L.dbl = (5 * (size_t)L.NR + 5 * (size_t)L.NC + 7 * (size_t)E + 2 + 1) & ~(size_t)1;
  L.slabC = ((size_t)L.NRS * MJ + 7) / 8 * 8;
  L.slabR = ((size_t)L.NC * MI + 7) / 8 * 8;
  return L;
}

using gdword = const __attribute__((address_space(1))) uint32_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
using gdword4 = const __attribute__((address_space(1))) u32x4;
using gdouble = const __attribute__((address_space(1))) double;

// sum over i < cnt of a[i sa] b[i sb] in FP64, eight loads of each operand issued before the
// products of a step (one wave per SIMD: nothing else hides the LDS latency)
template <typename TP>
__device__ __forceinline__ double dot_strided(const TP* a, int sa, const double* b, int sb, int cnt) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = 0;
  for (; i + 7 < cnt; i += 8) {
    TP av[8];
    double bv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      av[k] = a[(i + k) * sa];
      bv[k] = b[(i + k) * sb];
    }
    s0 += widen(av[0]) * bv[0];
    s1 += widen(av[1]) * bv[1];
    s2 += widen(av[2]) * bv[2];
    s3 += widen(av[3]) * bv[3];
    s0 += widen(av[4]) * bv[4];
    s1 += widen(av[5]) * bv[5];
    s2 += widen(av[6]) * bv[6];
    s3 += widen(av[7]) * bv[7];
  }
  if (i + 3 < cnt) {
    TP av[4];
    double bv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      av[k] = a[(i + k) * sa];
      bv[k] = b[(i + k) * sb];
    }
    s0 += widen(av[0]) * bv[0];
    s1 += widen(av[1]) * bv[1];
    s2 += widen(av[2]) * bv[2];
    s3 += widen(av[3]) * bv[3];
    i += 4;
  }
  for (; i < cnt; ++i) s0 += widen(a[i * sa]) * b[i * sb];
  return (s0 + s1) + (s2 + s3);
}

// One block draw as the pipelined kernel keeps it in LDS (one 32-byte record).
struct PipeDraw {
  int nJ, nI;   // block sizes
  int c0, r0;   // first column of J, first row of I
  double cc, cr;  // alpha / ||A_{:,J}||_F^2, alpha / ||A_{I,:}||_F^2
};
// The record read by every lane of the wave at the same LDS address, made wave-uniform.
__device__ __forceinline__ PipeDraw uniform_draw(const PipeDraw& s) {
  PipeDraw d = s;
  d.nJ = __builtin_amdgcn_readfirstlane(d.nJ);
  d.nI = __builtin_amdgcn_readfirstlane(d.nI);
  d.c0 = __builtin_amdgcn_readfirstlane(d.c0);
  d.r0 = __builtin_amdgcn_readfirstlane(d.r0);
  d.cc = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(d.cc)),
                          __builtin_amdgcn_readfirstlane(__double2loint(d.cc)));
  d.cr = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(d.cr)),
                          __builtin_amdgcn_readfirstlane(__double2loint(d.cr)));
  return d;
}

template <typename TP>
__global__ void __launch_bounds__(kPipeThreads) pipe_solve_kernel(SolveArgs a, GridSync gs,
                                                                  const double* __restrict__ Gm,
                                                                  const double* __restrict__ Hm,
                                                                  const double* __restrict__ Arm) {
  extern __shared__ double lds[];
  __shared__ int s_j[kRing], s_i[kRing];
  __shared__ PipeDraw s_dr[kRing];  // draw of iteration q in slot (q - 1) & (kRing - 1); zero past K
  __shared__ int s_ok;
  // handshakes between the waves (values are round or iteration numbers, nondecreasing)
  __shared__ int s_zflag[2];  // z^t of the owned rows, half h, is in LDS for t <= s_zflag[h]
  __shared__ int s_xflag[2];  // x^t of the owned columns, half h, is in LDS for t <= s_xflag[h]
  __shared__ int s_gflag;     // the owner's gathered sum of round t is in LDS for t <= s_gflag
  const int G = gridDim.x, w = blockIdx.x, tid = threadIdx.x, T = blockDim.x, lane = tid & 63;
  const int wv = tid >> 6;  // wave: 0 broadcast; 1, 2 the z side; 5, 6 the x side; 3 gathers;
                            // 3, 4 and 7 copy slabs and rows (waves w and w + 4 share a SIMD)
  const int64_t m = a.m, n = a.n;
  const int MJ = a.max_nJ, MI = a.max_nI, E = gs.stride;
  const int esz = (int)sizeof(TP);
  const PipeLayout L = pipe_layout(m, n, MI, MJ, E, G, esz);
  const int ra = 16 / esz;
  const int64_t r0 = own_lo(w, m, G, ra), r1 = own_lo(w + 1, m, G, ra);
  const int64_t cA = own_lo(w, n, G, kColOwnAlign), cB = own_lo(w + 1, n, G, kColOwnAlign);
  const int nr = (int)(r1 - r0), nc = (int)(cB - cA);
  const int c16 = (nr * esz + 15) / 16;  // 16-byte chunks of one column-slab run
  const int nrs = c16 * 16 / esz;        // its length in LDS (>= nr)

  double* zh = lds;               // z^t on owned rows at zh + (t & 3) NR
  double* bl = zh + 4 * L.NR;     // b on owned rows
  double* xh = bl + L.NR;         // x^t on owned columns at xh + (t & 3) NC
  double* xr = xh + 4 * L.NC;     // x_ref on owned columns
  double* bv = xr + L.NC;         // B^t at bv + (t % 3) E
  double* wr = bv + 3 * E;        // W_t at wr + (t & 1) E (v part at 0, u part at MJ)
  double* wpr = wr + 2 * E;       // W'_t at wpr + (t & 1) E
  double* gat = wpr + 2 * E;      // gathered sum of round t at gat[t & 1]
  TP* slabC = (TP*)(lds + L.dbl); // column slab of J_t at slabC + (t % 5) slabC (runs of nrs)
  TP* slabR = slabC + kPipeSlabs * L.slabC;

  const TP* __restrict__ Arow = (const TP*)a.Arow;
  const TP* __restrict__ Acol = (const TP*)a.Acol;
  const int64_t K = a.max_iter;
  const int K32 = (int)K;  // (below 2^31; rounds and iterations are 32-bit here)
  const int64_t ce = a.check_every > 0 ? a.check_every : 1;
  const int ce32 = (int)(ce < K ? ce : K);
  const bool checking = a.x_ref != nullptr && a.tol > 0.0;
  const bool final_err = a.x_ref != nullptr;
  const int err_slot = MJ + MI;
  const int EU = MJ + MI + 1;  // entries in use (v, u and the error); their owners publish every round
  const size_t V2 = (size_t)E * 2;
  const int e_own = w < E ? w : -1;  // the entry this workgroup owns (E <= G)
  const bool v_owner = e_own >= 0 && e_own < MJ, u_owner = e_own >= MJ && e_own < MJ + MI;

  for (int q = tid; q < nr; q += T) {
    zh[q] = a.z_in ? a.z_in[r0 + q] : a.b[r0 + q];
    bl[q] = a.b[r0 + q];
  }
  for (int q = tid; q < nc; q += T) {
    xh[q] = a.x_in ? a.x_in[cA + q] : 0.0;
    xr[q] = a.x_ref ? a.x_ref[cA + q] : 0.0;
  }
  for (int q = tid; q < 7 * E + 2; q += T) bv[q] = 0.0;

    auto refill = [&](int64_t first, int t0) {  // draws first .. first + 63 (lanes of the wave at t0)
    const int l = tid - t0;
    if (l >= 0 && l < 64) {
      const int64_t q = first + l;
      const int sl = (int)((q - 1) & (kRing - 1));
      PipeDraw d{0, 0, 0, 0, 0.0, 0.0};
      if (q <= K) {
        int jj, ii;
        draw_pair(a, a.k0 + q, jj, ii);
        s_j[sl] = jj;
        s_i[sl] = ii;
        d.c0 = (int)a.col_off[jj];
        d.nJ = (int)(a.col_off[jj + 1] - a.col_off[jj]);
        d.r0 = (int)a.row_off[ii];
        d.nI = (int)(a.row_off[ii + 1] - a.row_off[ii]);
        d.cc = a.coef_col[jj];
        d.cr = a.coef_row[ii];
      }
      s_dr[sl] = d;
    }
  };
  // draw of iteration t as wave-uniform values (all zero outside 1..K: the records past K are)
  auto drw = [&](int t) -> PipeDraw {
    PipeDraw d{0, 0, 0, 0, 0.0, 0.0};
    if (t >= 1) d = uniform_draw(s_dr[(t - 1) & (kRing - 1)]);
    return d;
  };
  auto nJ_of = [&](int t) -> int { return drw(t).nJ; };
  auto nI_of = [&](int t) -> int { return drw(t).nI; };
  auto cc_of = [&](int t) -> double { return drw(t).cc; };
  auto cr_of = [&](int t) -> double { return drw(t).cr; };
  auto colslab = [&](int t) -> TP* { return slabC + (size_t)(t % kPipeSlabs) * L.slabC; };
  auto rowslab = [&](int t) -> TP* { return slabR + (size_t)(t % kPipeSlabs) * L.slabR; };
  // round t carries the error of x^{t-3} when a check is due (and the last error, of x^K)
  auto err_round = [&](int t) -> bool {
    const int k = t - 3;
    return k >= 1 && k <= K32 && ((checking && k % ce32 == 0) || (final_err && k == K32));
  };
  // entries of round t (polled in the broadcast and gathered by owners)
  // entry e of round t is broadcast: nJn = |J_{t+1}|, nIt = |I_t|, er = err_round(t)
  auto need_d = [&](int e, int nJn, int nIt, bool er) -> bool {  // (false for e < 0: no entry owned)
    return (e >= 0 && e < MJ && e < nJn) || (e >= MJ && e < MJ + MI && e - MJ < nIt) || (e == err_slot && er);
  };
  auto need = [&](int t, int e) -> bool { return need_d(e, nJ_of(t + 1), nI_of(t), err_round(t)); };

  // ---- copies into LDS
  // Column slab of J_t: nJ runs of the owned rows, each c16 16-byte chunks (the column panels are
  // padded to 16 entries, so a rounded-up run stays inside its column); run c at c * nrs.
  auto colsrc = [&](int t) -> const char* { return (const char*)(Acol + a.ldc * drw(t).c0 + r0); };
  auto col_direct = [&](int t, int from, int l0, int nl) {  // chunks from `from` on
    const int nJ = nr > 0 ? nJ_of(t) : 0;
    if (nJ == 0) return;
    const char* src = colsrc(t);
    u32x4* dst = (u32x4*)colslab(t);
    for (int d = from + l0; d < nJ * c16; d += nl) {
      const int c = d / c16, p = d - c * c16;
      dst[c * c16 + p] = *(gdword4*)(src + (int64_t)c * a.ldc * esz + 16 * p);
    }
  };
  // Row slab of I_t: one run of nc x nI entries, copied in dwords when it starts on a dword (2-byte
  // panels at an odd offset and a 2-byte tail go entry by entry).
  auto rowsrc = [&](int t) -> const TP* {
    const PipeDraw d = drw(t);
    return Arow + n * d.r0 + cA * d.nI;
  };
  auto row_dwords = [&](int t) -> int {
    const int nI = nI_of(t);
    if (nI == 0 || nc == 0 || ((uintptr_t)rowsrc(t) & 3) != 0) return 0;
    return nc * nI * esz / 4;
  };
  auto row_direct = [&](int t, int from_dw, int l0, int nl) {  // dwords from `from_dw` on, then entries
    const int nI = nI_of(t);
    if (nI == 0 || nc == 0) return;
    const TP* src = rowsrc(t);
    TP* dst = rowslab(t);
    const int ndw = row_dwords(t);
    for (int d = from_dw + l0; d < ndw; d += nl) ((uint32_t*)dst)[d] = ((gdword*)src)[d];
    for (int e = ndw * 4 / esz + l0; e < nc * nI; e += nl) dst[e] = src[e];
  };
  // Coefficient vectors of this workgroup's entry, scaled, in the layout of the broadcast (E
  // doubles, zero outside the entries they multiply).  W_t multiplies B^{t-1} (the correction
  // -w_t . B^{t-1}): its v part is c'_t times the row over J_t, its u part c_{t-1} times the row of
  // G over I_{t-1}.  W'_t multiplies B^{t-2}: the same rows over J_{t-1} and I_{t-2}, scaled by
  // c'_{t-1} and c_{t-2}.  The rows: a v owner's row c0(J_{t+1}) + e of H; a u owner's row
  // R = r0(I_t) + e - MJ of A (v part) and of G (u part).  Zero when entry e of round t is not
  // broadcast (and for workgroups that own no v or u entry).
  struct WSrc {
    const double *bv, *bu;  // the rows at the first entry of each part
    int nv, nu;             // lengths of the parts (0: none)
    double sv, su;          // scale factors
  };
  auto wsrc = [&](int t, bool prime) -> WSrc {
    WSrc q{nullptr, nullptr, 0, 0, 0.0, 0.0};
    if (!v_owner && !u_owner) return q;
    const PipeDraw dn = drw(t + 1), dt = drw(t);
    if (!need_d(e_own, dn.nJ, dt.nI, err_round(t))) return q;
    const PipeDraw dv = prime ? drw(t - 1) : dt, du = drw(prime ? t - 2 : t - 1);
    q.nv = dv.nJ;
    q.sv = dv.cc;
    if (v_owner) {
      q.bv = Hm + ((int64_t)dn.c0 + e_own) * n + dv.c0;
    } else {
      const int64_t R = (int64_t)dt.r0 + (e_own - MJ);
      q.bv = Arm + R * n + dv.c0;
      q.bu = Gm + R * m + du.r0;
      q.nu = du.nI;
      q.su = du.cr;
    }
    return q;
  };
  // entry q of the vector (q < E): its source, or null for a zero
  auto wsrc_at = [&](const WSrc& v, int q) -> const double* {
    return q < v.nv ? v.bv + q : ((q >= MJ && q - MJ < v.nu) ? v.bu + (q - MJ) : nullptr);
  };
  auto wscale = [&](const WSrc& v, int q) -> double { return q < MJ ? v.sv : v.su; };
  auto wr_of = [&](int t) -> double* { return wr + (size_t)(t & 1) * E; };    // W_t
  auto wpr_of = [&](int t) -> double* { return wpr + (size_t)(t & 1) * E; };  // W'_t

  unsigned spins = 0;
  int ok = 1;
  auto give_up = [&]() -> bool {
    if ((++spins & 63u) == 0) {
      if (__hip_atomic_load(gs.timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
      if (spins > kSpinLimit) {
        __hip_atomic_store(gs.timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
      }
    }
    return false;
  };
  const int p2 = lane & 1;
  const bool first = p2 == 0;
  // Gather: the sum over workgroups of entry e of the partial vectors of round t (one wave).
  auto gather = [&](int t, int e) -> double {
    const unsigned long long* Pp = gs.part + (size_t)(t & (kPipeParts - 1)) * G * V2 + (size_t)e * 2;
    const unsigned ep = (unsigned)(t + 1);
    double acc = 0.0;
    spins = 0;
    for (int q0 = 0; q0 < G; q0 += 256) {
      unsigned long long wd[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      while (ok) {
        // all eight loads in flight before any is inspected (a use between them would make each
        // wait for the previous one)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int q = q0 + k * 32 + (lane >> 1);
          wd[k] = ld_u64(Pp + (size_t)(q < G ? q : G - 1) * V2 + p2);
        }
        bool mine = true;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int q = q0 + k * 32 + (lane >> 1);
          const unsigned tg = first ? (unsigned)(wd[k] >> 32) : (unsigned)wd[k];
          mine = mine && (q >= G || tg == ep);
        }
        if (__all(mine)) break;
        if (give_up()) ok = 0;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int q = q0 + k * 32 + (lane >> 1);
        const unsigned long long o = mirror_word(wd[k]);
        if (first && q < G) acc += tag_value(wd[k], o);
      }
    }
    return group_sum(acc, 64);
  };
  // LDS handshake between waves of the workgroup: the writer's LDS stores are done before the flag
  auto set_flag = [&](int* f, int v) {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    if (lane == 0) __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  auto wait_flag = [&](int* f, int v) {
    unsigned sp = 0;
    while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < v) {
      if (++sp > (kSpinLimit << 2)) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  };

  // ---- partial sums of round t from z (owned rows) and x (owned columns):
  //   v entries A_{J_{t+1}}^T z over owned rows (one wave), u entries A_{I_t} x - b + z (one wave),
  //   and ||x - x_ref||^2 when due (the u wave)
  auto part_v = [&](int t, const double* zc, int c_lo, int c_hi) {  // columns [c_lo, c_hi), whole wave
    unsigned long long* P = gs.part + ((size_t)(t & (kPipeParts - 1)) * G + w) * V2;
    const unsigned ep = (unsigned)(t + 1);
    const int nJn = c_hi < nJ_of(t + 1) ? c_hi : nJ_of(t + 1);
    if (nJn <= c_lo) return;
    const TP* Sl = colslab(t + 1);
    const int tq = lanes_per_item(64, nJn - c_lo), per = 64 / tq, sub = lane % tq;
    for (int c0 = c_lo; c0 < nJn; c0 += per) {
      const int c = c0 + lane / tq;
      const TP* col = Sl + (size_t)(c < nJn ? c : nJn - 1) * nrs;
      const int cnt = sub < nr ? (nr - sub + tq - 1) / tq : 0;
      const double acc = group_sum(dot_strided(col + sub, tq, zc + sub, tq, cnt), tq);
      if (c < nJn && sub == 0) st_tagged(P, c, acc, ep);
    }
  };
  // rows [l_lo, l_hi) of I_t (whole wave); with_err: also ||x - x_ref||^2 when due
  auto part_u = [&](int t, const double* xc, const double* zc, int zready, int l_lo, int l_hi, bool with_err) {
    unsigned long long* P = gs.part + ((size_t)(t & (kPipeParts - 1)) * G + w) * V2;
    const unsigned ep = (unsigned)(t + 1);
    const int nIt = nI_of(t), lend = l_hi < nIt ? l_hi : nIt;
    if (lend > l_lo) {
      const TP* Sr = rowslab(t);
      const int64_t rI = drw(t).r0;
      bool waited = false;
      for (int l0 = l_lo; l0 < lend; l0 += 64) {
        const int l = l0 + lane;
        double acc = l < lend ? dot_strided(Sr + l, nIt, xc, 1, nc) : 0.0;
        // owned rows of I_t add z - b (z from the z-side waves: wait for it once)
        const int64_t lo = rI + l0, hi = rI + (l0 + 64 < lend ? l0 + 64 : lend);
        if (lo < r1 && hi > r0) {
          if (!waited) {
            wait_flag(&s_zflag[0], zready);
            wait_flag(&s_zflag[1], zready);
            waited = true;
          }
          const int64_t gl = rI + l;
          if (l < lend && gl >= r0 && gl < r1) acc += zc[gl - r0] - bl[gl - r0];
        }
        if (l < lend) st_tagged(P, MJ + l, acc, ep);
      }
    }
    if (with_err && err_round(t)) {
      double e = 0.0;
      for (int cc = lane; cc < nc; cc += 64) {
        const double d = xc[cc] - xr[cc];
        e += d * d;
      }
      int width = 1;
      while (width < nc && width < 64) width *= 2;
      e = group_sum(e, width);
      if (lane == 0) st_tagged(P, err_slot, e, ep);
    }
  };
  // z^t = z^{t-1} - c'_t A_{J_t} v^t on owned rows (one wave), v^t = B^{t-1}[0, nJ)
  auto zstep = [&](int t, const double* vB, int p_lo, int p_hi) {  // owned rows [p_lo, p_hi)
    const int nJ = nJ_of(t);
    const TP* Sl = colslab(t);
    const double coef = cc_of(t);
    const double* zo = zh + (size_t)((t - 1) & 3) * L.NR;
    double* zn = zh + (size_t)(t & 3) * L.NR;
    for (int p = p_lo + lane; p < p_hi; p += 64) zn[p] = zo[p] - coef * dot_strided(Sl + p, nrs, vB, 1, nJ);
  };
  // x^t = x^{t-1} - c_t A_{I_t}^T u^t on owned columns (one wave), u^t = B^t[MJ, MJ + nI)
  auto xstep = [&](int t, const double* uB, int c_lo, int c_hi) {  // owned columns [c_lo, c_hi)
    if (c_hi <= c_lo) return;
    const int nI = nI_of(t);
    const TP* Sl = rowslab(t);
    const double coef = cr_of(t);
    const double* xo = xh + (size_t)((t - 1) & 3) * L.NC;
    double* xn = xh + (size_t)(t & 3) * L.NC;
    const int tpc = lanes_per_item(64, c_hi - c_lo), cp = 64 / tpc, sub = lane % tpc;
    for (int c0 = c_lo; c0 < c_hi; c0 += cp) {
      const int cc = c0 + lane / tpc;
      const TP* col = Sl + (size_t)(cc < c_hi ? cc : c_hi - 1) * nI;
      const int cnt = sub < nI ? (nI - sub + tpc - 1) / tpc : 0;
      const double acc = group_sum(dot_strided(col + sub, tpc, uB + sub, tpc, cnt), tpc);
      if (cc < c_hi && sub == 0) xn[cc] = xo[cc] - coef * acc;
    }
  };

  // ---- wave 0: the broadcast (8 entries per lane pair: entry q = 32 k + lane / 2, first lanes)
  double pc = 0.0;  // -w'_{r+1} . B^{r-1} of this workgroup's entry (wave 0)
  // Copies for later rounds, one wave each, all loads issued before any is written to LDS: the
  // column slab of J_t in 16-byte chunks (in two parts, the loads and then the stores into LDS, so
  // the gather can run between them), the row slab of I_t in dwords, and the scaled vectors
  // W_t, W'_{t+1} in doubles.
  auto col_issue = [&](int t, u32x4* v, int* at) -> int {  // returns the chunk count
    const int ncol = nr > 0 ? nJ_of(t) * c16 : 0;
#pragma unroll
    for (int k = 0; k < pipe_stage<TP>() / 4; ++k) at[k] = -1;
    if (ncol == 0) return 0;
    const char* src = colsrc(t);
    const int64_t cstride = a.ldc * esz;
    int c = lane / c16, p = lane - c * c16;
    const int sc = 64 / c16, sp = 64 - sc * c16;
#pragma unroll
    for (int k = 0; k < pipe_stage<TP>() / 4; ++k) {
      if (lane + 64 * k < ncol) {
        v[k] = *(gdword4*)(src + (int64_t)c * cstride + 16 * p);
        at[k] = c * c16 + p;
      }
      p += sp;
      c += sc;
      if (p >= c16) {
        p -= c16;
        ++c;
      }
    }
    return ncol;
  };
  auto col_write = [&](int t, const u32x4* v, const int* at, int ncol) {
    u32x4* const dst = (u32x4*)colslab(t);
#pragma unroll
    for (int k = 0; k < pipe_stage<TP>() / 4; ++k)
      if (at[k] >= 0) dst[at[k]] = v[k];
    if (ncol > 64 * (pipe_stage<TP>() / 4)) col_direct(t, 64 * (pipe_stage<TP>() / 4), lane, 64);
  };
  auto copy_row = [&](int t, auto&& between) {  // `between` runs while the loads are in flight
    const int nrow = row_dwords(t);
    uint32_t v[pipe_stage<TP>()];
    if (nrow > 0) {
      gdword* src = (gdword*)rowsrc(t);
#pragma unroll
      for (int k = 0; k < pipe_stage<TP>(); ++k)
        if (lane + 64 * k < nrow) v[k] = src[lane + 64 * k];
    }
    between();
    if (nrow > 0) {
      uint32_t* const dst = (uint32_t*)rowslab(t);
#pragma unroll
      for (int k = 0; k < pipe_stage<TP>(); ++k)
        if (lane + 64 * k < nrow) dst[lane + 64 * k] = v[k];
    }
    row_direct(t, 64 * pipe_stage<TP>(), lane, 64);
  };
  auto copy_wv = [&](int t) {  // W_t and W'_{t+1} (entries lane + 64 k; E <= 256)
    const WSrc va = wsrc(t, false), vb = wsrc(t + 1, true);
    double xa[4], xb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = lane + 64 * k;
      const double* pa = wsrc_at(va, q);
      const double* pb = wsrc_at(vb, q);
      xa[k] = pa ? *(gdouble*)pa : 0.0;
      xb[k] = pb ? *(gdouble*)pb : 0.0;
    }
    double* da = wr_of(t);
    double* db = wpr_of(t + 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = lane + 64 * k;
      if (q < E) {
        da[q] = wscale(va, q) * xa[k];
        db[q] = wscale(vb, q) * xb[k];
      }
    }
  };

  // ---------------- prologue
  for (int64_t f = 1; f <= 128 && f <= K; f += 64) refill(f, 64 * (int)((f / 64) & 3));
  int64_t filled_to = 128;
  if (tid == 0) {
    s_ok = 1;
    s_zflag[0] = s_zflag[1] = 0;
    s_xflag[0] = s_xflag[1] = 0;
    s_gflag = -1;
  }
  lds_barrier();
  {
    // slabs of J_1..J_4 and I_1..I_3; W_1, W_2, W'_2, W'_3
    for (int64_t t = 1; t <= 4; ++t) col_direct(t, 0, tid, T);
    for (int64_t t = 1; t <= 3; ++t) row_direct(t, 0, tid, T);
    for (int v = 0; v < 4; ++v) {
      const int t = v < 2 ? 1 + v : v;
      const WSrc src = wsrc(t, v >= 2);
      double* dst = v < 2 ? wr_of(t) : wpr_of(t);
      for (int q = tid; q < E; q += T) {
        const double* pq = wsrc_at(src, q);
        dst[q] = pq ? wscale(src, q) * *(gdouble*)pq : 0.0;
      }
    }
  }
  lds_barrier();
  // partial sums of rounds 0, 1, 2 from x^0, z^0; the owner gathers rounds 0 and 1
  if (wv == 1) {
    part_v(0, zh, 0, MJ);
    part_v(1, zh, 0, MJ);
    part_v(2, zh, 0, MJ);
  } else if (wv == 5) {
    part_u(1, xh, zh, 0, 0, MI, true);
    part_u(2, xh, zh, 0, 0, MI, true);
  } else if (wv == 3) {
    const double g0 = need(0, e_own) ? gather(0, e_own) : 0.0;
    const double g1 = need(1, e_own) ? gather(1, e_own) : 0.0;
    if (lane == 0) {
      gat[0] = g0;
      gat[1] = g1;
    }
    set_flag(&s_gflag, 1);
  }
  if (!ok) s_ok = 0;
  lds_barrier();
  if (tid < 64) {
    if (e_own >= 0 && e_own < EU && lane < kCopies) {
      unsigned long long* S0 = gs.gsum + (size_t)(1 % kGridSumRing) * kCopies * V2;
      st_tagged(S0 + (size_t)lane * V2, e_own, gat[0], 1u);
    }
  }

  int status = 0, stopped = 0;
  int64_t last_k = a.k0;
  double last_err2 = -1.0;
  int64_t last_check = -1;
  bool alive = s_ok != 0;
  // After the workgroup barrier of round r (B^r in LDS): the stop rule on the error B^r carries,
  // the same decision in every wave.  Returns true when the solve ends here (outputs written).
  auto round_end = [&](int r) -> bool {
    if (tid == 0 && w == 0 && a.trace_j && r >= 1 && r <= K) {
      a.trace_j[r - 1] = s_j[(r - 1) & (kRing - 1)];
      a.trace_i[r - 1] = s_i[(r - 1) & (kRing - 1)];
    }
    if (!err_round(r)) return false;
    const double e2 = bv[(size_t)(r % 3) * E + err_slot];  // the error of x^{r-3}
    const int64_t k = r - 3;
    last_err2 = e2;
    last_check = a.k0 + k;
    const double rel = sqrt(e2) / sqrt(a.xref_sq);
    const bool stop = checking && (rel < a.tol || !isfinite(e2) || rel > 1e6);
    if (!stop && k != K) return false;
    stopped = stop ? 1 : 0;
    status = !checking ? 0 : (rel < a.tol ? 0 : ((!isfinite(e2) || rel > 1e6) ? 2 : 1));
    last_k = a.k0 + k;
    const double* zk = zh + (size_t)(k & 3) * L.NR;
    const double* xk = xh + (size_t)(k & 3) * L.NC;
    for (int p = tid; p < nr; p += T)
      if (a.z_out) a.z_out[r0 + p] = zk[p];
    for (int p = tid; p < nc; p += T) a.x_out[cA + p] = xk[p];
    return true;
  };

  if (tid < 64) {
    // ---- wave 0: poll B^r, publish this workgroup's entry of B^{r+1}, hand B^r over.  Every
    // owner of an entry in use publishes it every round (zero when no one reads it: its
    // coefficient vectors and its gathered sum are zero then), so the poll waits for all of them.
    const bool owner = e_own >= 0 && e_own < EU;
    for (int r = 0; alive; ++r) {
      const unsigned epB = (unsigned)(r + 1);
      const unsigned long long* Sg =
          gs.gsum + (size_t)(epB % kGridSumRing) * kCopies * V2 + (size_t)(w % kCopies) * V2;
      unsigned long long wd[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int q = k * 32 + (lane >> 1);
        wd[k] = ld_u64(Sg + (size_t)2 * (q < E ? q : E - 1) + p2);
      }
      // while the loads are in flight: W_{r+1} and W'_{r+2} of this workgroup's entry in the
      // layout of the poll (entry 32 k + lane / 2 in register k)
      double W1[8], W2[8];
      if (owner) {
        const double* w1 = wr_of(r + 1);
        const double* w2 = wpr_of(r + 2);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int q = k * 32 + (lane >> 1);
          W1[k] = q < E ? w1[q] : 0.0;
          W2[k] = q < E ? w2[q] : 0.0;
        }
      }
      auto arrived = [&]() -> bool {  // every entry in use carries the epoch of B^r
        bool mine = true;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int q = k * 32 + (lane >> 1);
          const unsigned tg = first ? (unsigned)(wd[k] >> 32) : (unsigned)wd[k];
          mine = mine && (q >= EU || tg == epB);
        }
        return __all(mine);
      };
      spins = 0;
      while (ok && !arrived()) {
        if (give_up()) ok = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int q = k * 32 + (lane >> 1);
          wd[k] = ld_u64(Sg + (size_t)2 * (q < E ? q : E - 1) + p2);
        }
      }
      double vals[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int q = k * 32 + (lane >> 1);
        const unsigned long long o = mirror_word(wd[k]);
        vals[k] = (first && q < EU) ? tag_value(wd[k], o) : 0.0;
      }
      if (owner) {
        double d = 0.0, d2 = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          d += W1[k] * vals[k];   // w_{r+1} . B^r
          d2 += W2[k] * vals[k];  // w'_{r+2} . B^r
        }
        d = group_sum(d, 64);
        wait_flag(&s_gflag, (int)(r + 1));
        const double g = gat[(r + 1) & 1];
        if (lane < kCopies) {
          unsigned long long* Sn = gs.gsum + (size_t)((r + 2) % kGridSumRing) * kCopies * V2;
          st_tagged(Sn + (size_t)lane * V2, e_own, g + pc - d, (unsigned)(r + 2));
        }
        pc = -group_sum(d2, 64);
      }
      double* Bn = bv + (size_t)(r % 3) * E;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int q = k * 32 + (lane >> 1);
        if (first && q < E) Bn[q] = vals[k];
      }
      if (!ok) s_ok = 0;
      lds_barrier();  // B^r in LDS; the helpers' work of round r - 1 is done
      if (s_ok == 0) {
        alive = false;
        break;
      }
      if (round_end(r)) break;
      if (!final_err && r == K) {
        lds_barrier();
        last_k = a.k0 + K;
        break;
      }
    }
  } else {
    // ---- waves 1..3: round r of the helpers, after B^r is in LDS
    for (int r = 0; alive; ++r) {
      if (!ok) s_ok = 0;
      lds_barrier();
      if (s_ok == 0) {
        alive = false;
        break;
      }
      if (round_end(r)) break;
      const double* Bc = bv + (size_t)(r % 3) * E;
      if (!final_err && r == K) {  // the last step: x^K (z^K was formed one round earlier)
        if (wv == 5 && nc > 0) xstep(K, Bc + MJ, 0, nc);
        lds_barrier();
        last_k = a.k0 + K;
        break;
      }
      if (wv == 7 && filled_to < K && r + 40 > filled_to) refill(filled_to + 1, 448);
      if (filled_to < K && r + 40 > filled_to) filled_to += 64;
      const int64_t tz = r + 1 <= K ? r + 1 : K, tx = r <= K ? r : K;
      const double* zc = zh + (size_t)(tz & 3) * L.NR;
      const double* xc = xh + (size_t)(tx & 3) * L.NC;
      if (wv == 1 || wv == 2) {
        // z side, half h: z^{r+1} on half the owned rows, then half the v entries of round r + 3
        const int h = wv - 1, ph = (nr + 1) / 2;
        if (r + 1 <= K && nr > 0) zstep(r + 1, Bc, h == 0 ? 0 : ph, h == 0 ? ph : nr);
        set_flag(&s_zflag[h], (int)(r + 1));
        wait_flag(&s_zflag[1 - h], (int)(r + 1));
        const int nJn = nJ_of(r + 4), ch = (nJn + 1) / 2;
        part_v(r + 3, zc, h == 0 ? 0 : ch, h == 0 ? ch : nJn);
      } else if (wv == 5 || wv == 6) {
        // x side, half h: x^r on half the owned columns, then half the u entries of round r + 3
        const int h = wv - 5, chx = (nc + 1) / 2;
        if (r >= 1 && r <= K && nc > 0) xstep(r, Bc + MJ, h == 0 ? 0 : chx, h == 0 ? chx : nc);
        set_flag(&s_xflag[h], (int)r);
        wait_flag(&s_xflag[1 - h], (int)r);
        const int nIt = nI_of(r + 3), lh = (nIt + 1) / 2;
        part_u(r + 3, xc, zc, (int)(r + 1), h == 0 ? 0 : lh, h == 0 ? lh : nIt, h == 0);
      } else if (wv == 3) {
        // the owner's sum of round r + 2 (wave 0 needs it for its next entry), with the loads of
        // the column slab of J_{r+5} in flight meanwhile
        u32x4 cv[pipe_stage<TP>() / 4];
        int cat[pipe_stage<TP>() / 4];
        const int ncol = col_issue(r + 5, cv, cat);
        const double g = need(r + 2, e_own) ? gather(r + 2, e_own) : 0.0;
        if (lane == 0) gat[(r + 2) & 1] = g;
        set_flag(&s_gflag, (int)(r + 2));
        col_write(r + 5, cv, cat, ncol);
      } else if (wv == 4) {
        copy_row(r + 4, []() {});  // the row slab of I_{r+4}
      } else if (wv == 7) {
        if (v_owner || u_owner) copy_wv(r + 3);  // W_{r+3} and W'_{r+4}
      }
    }
  }
  wait_mem();
  if (alive && !final_err) {  // x^K, z^K
    const double* zk = zh + (size_t)(K & 3) * L.NR;
    const double* xk = xh + (size_t)(K & 3) * L.NC;
    for (int p = tid; p < nr; p += T)
      if (a.z_out) a.z_out[r0 + p] = zk[p];
    for (int p = tid; p < nc; p += T) a.x_out[cA + p] = xk[p];
  }
  if (w == 0 && tid == 0) {
    a.status->status = alive ? status : -4;
    a.status->stopped = stopped;
    a.status->last_k = last_k;
    a.status->err2 = last_err2;
    a.status->check_k = last_check;
  }
}

// A as a row-major FP64 matrix (row r at out + r n) from the row panels (block i: n x |I_i|
// column-major at n row_off[i]); one workgroup per row block, reads along the panel.
template <typename TP>
__global__ void __launch_bounds__(256) unpack_rows_kernel(const TP* __restrict__ Arow, int64_t n,
                                                          const int64_t* __restrict__ row_off, int32_t s,
                                                          double* __restrict__ out) {
  for (int64_t i = blockIdx.x; i < s; i += gridDim.x) {
    const int64_t r0 = row_off[i];
    const int64_t nI = row_off[i + 1] - r0;
    const TP* P = Arow + n * r0;
    for (int64_t e = threadIdx.x; e < nI * n; e += blockDim.x) {
      const int64_t c = e / nI, l = e - c * nI;
      out[(r0 + l) * n + c] = widen(P[e]);
    }
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

namespace rebk {

size_t pipe_solve_lds_bytes(const SolveArgs& a, int grid, int stride, int panel_dtype) {
  const size_t esz = panel_dtype == 0 ? 8 : (panel_dtype == 1 ? 4 : 2);
  const PipeLayout L = pipe_layout(a.m, a.n, a.max_nI, a.max_nJ, stride, grid, (int)esz);
  return L.dbl * sizeof(double) + (size_t)kPipeSlabs * (L.slabC + L.slabR) * esz + 64;
}

hipError_t pipe_solve_max_blocks(int panel_dtype, size_t lds_bytes, int* blocks_per_cu) {
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const void* k = (const void*)pipe_solve_kernel<TP>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, kPipeThreads, lds_bytes);
  });
}

hipError_t launch_unpack_rows(const void* Arow, int panel_dtype, int64_t n, const int64_t* row_off_d, int32_t s,
                              double* out, hipStream_t st) {
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const unsigned g = (unsigned)(s < 65536 ? s : 65536);
    hipLaunchKernelGGL(unpack_rows_kernel<TP>, dim3(g), dim3(256), 0, st, (const TP*)Arow, n, row_off_d, s, out);
    return hipGetLastError();
  });
}

hipError_t launch_pipe_solve(const SolveArgs& a, const GridSync& gs, const double* Gm, const double* Hm,
                             const double* Arm, int panel_dtype, int grid, hipStream_t st) {
  return dev::dispatch_panel(panel_dtype, [&](auto tag) -> hipError_t {
    using TP = typename decltype(tag)::T;
    const void* k = (const void*)pipe_solve_kernel<TP>;
    const size_t lds = pipe_solve_lds_bytes(a, grid, gs.stride, panel_dtype);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    SolveArgs aa = a;
    GridSync gg = gs;
    const double* g = Gm;
    const double* h = Hm;
    const double* ar = Arm;
    void* args[] = {&aa, &gg, (void*)&g, (void*)&h, (void*)&ar};
    return hipLaunchCooperativeKernel(k, dim3(grid), dim3(kPipeThreads), args, (unsigned)lds, st);
  });
}

}  // namespace rebk
