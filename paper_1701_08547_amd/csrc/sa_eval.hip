// gfx950 kernels of the static autotuning model: fused occupancy (Eqs. 1-5),
// instruction-mix score (Eq. 6 with divergence and latency-hiding factors)
// and per-variant top-k selection, streamed over a CSR batch of
// (variant, configuration) evaluations.
//
// Work decomposition.  The flattened evaluation space [0, n_evals) is cut
// into wave-tiles of `tile` evaluations; each wave of a workgroup owns one
// wave-tile and walks the variant segments that overlap it ("pieces").  Per
// piece the variant's record is wave-uniform and computed once.  The body of
// a piece streams in chunks of 256 evaluations, each lane reading 4
// consecutive evaluations of every structure-of-arrays column with one
// 16-byte load, the next chunk's loads issued before the current chunk is
// evaluated; unaligned heads and ragged tails go through a masked row path.
//
// Selection.  Keys are (order-preserving score bits << 32 | local index), a
// total order.  Each wave keeps a threshold theta (the score of its current
// k-th best) and appends only the evaluations at or below it to a per-wave
// LDS candidate buffer (ballot + mbcnt compaction).  When the buffer fills,
// the wave extracts the k smallest keys: every lane sorts its share, then k
// rounds take the wave-wide minimum of the lane heads with DPP row
// reductions.  A piece that is a whole segment writes its result directly;
// pieces of segments that span wave-tiles write k-key fragments that
// sa_merge_kernel combines.
//
// Arithmetic.  Built with -ffp-contract=off and IEEE division, so every
// binary32 step of the score rounds exactly once, in the documented order.
#include <float.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa_dev.h"

namespace sa {
namespace {

// Unconditional stores of one lane's N consecutive 4-byte values at byte
// offset `off` of a buffer resource.  An output that was not asked for gets
// a resource with no records, whose stores the hardware drops; the stores
// stay unconditional in the program, so the compiler knows how many memory
// operations follow each prefetch and can wait for the prefetch alone
// (optional stores behind a branch would make it wait for everything).
typedef uint32_t v2u32_t __attribute__((ext_vector_type(2)));
typedef uint32_t v4u32_t __attribute__((ext_vector_type(4)));
constexpr int kBufFlags = 0x00020000;  // raw 32-bit buffer, gfx9 word 3

__device__ __forceinline__ __amdgpu_buffer_rsrc_t out_rsrc(void *p, int64_t byte0, int bytes) {
  // the offset is wave-uniform; saying so keeps the resource in scalar
  // registers (a possibly divergent resource costs a per-store loop)
  const uint64_t a = p ? (uint64_t)p + (uint64_t)byte0 : 0ull;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), (short)0, p ? bytes : 0, kBufFlags);
}

template <int N, typename T>
__device__ __forceinline__ void buf_store(const T (&x)[N], __amdgpu_buffer_rsrc_t r, int off) {
  constexpr int aux = SA_NT_STORE ? 2 : 0;  // non-temporal
  uint32_t u[N];
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = __builtin_bit_cast(uint32_t, x[i]);
  if constexpr (N == 4) {
    __builtin_amdgcn_raw_buffer_store_b128(v4u32_t{u[0], u[1], u[2], u[3]}, r, off, 0, aux);
  } else if constexpr (N == 2) {
    __builtin_amdgcn_raw_buffer_store_b64(v2u32_t{u[0], u[1]}, r, off, 0, aux);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) __builtin_amdgcn_raw_buffer_store_b32(u[i], r, off + 4 * i, 0, aux);
  }
}

// Values of a product space at local index li (Mode::Product): mixed-radix
// digits, grid fastest.  floor(x / n) for x < 2^24 and n <= 256 is one
// multiply-high by m = ceil(2^32 / n): with m n = 2^32 + r (r < n) and
// x = q n + t, x m / 2^32 = q + t / n + x r / (n 2^32) < q + 1.  m = 0 stands
// for n = 1.  Indices are clamped, so an index past the space reads a valid
// value (such rows are masked out or never reached).
struct ProductDigits {
  const int32_t *pv;  // LDS: four lists of kProductMaxValues values
  uint32_t nG, nR, nU, tmax;
  uint32_t mG, mR, mU;
  __device__ __forceinline__ static uint32_t div(uint32_t x, uint32_t m) { return m ? __umulhi(x, m) : x; }
  __device__ __forceinline__ void at(uint32_t li, int32_t &T, int32_t &U, int32_t &R, int32_t &G) const {
    const uint32_t q1 = div(li, mG);
    const uint32_t q2 = div(q1, mR);
    const uint32_t q3 = div(q2, mU);
    T = pv[min(q3, tmax)];
    U = pv[kProductMaxValues + (q2 - q3 * nU)];
    R = pv[2 * kProductMaxValues + (q1 - q2 * nR)];
    G = pv[3 * kProductMaxValues + (li - q1 * nG)];
  }
};

// Streams one piece [e, pe) of one segment.  ITEMS consecutive evaluations
// per lane per chunk (chunk = 64 ITEMS evaluations), one chunk of loads in
// flight ahead of the one being evaluated.
template <Mode MODE, bool HAS_GRID, bool TOPK, int ITEMS>
struct Evaluator {
  static constexpr int kC = 64 * ITEMS;
  const EvalLaunch &L;
  const Tables &tb;
  const Piece &pc;
  Selector &sel;
  int lane;
  ProductDigits pd{};

  // Masked rows over [base, end): lane l takes base + 64 i + l.  end - base <= 256.
  __device__ __forceinline__ void masked(int64_t base, int64_t end) {
    if constexpr (TOPK) make_room(sel, 256, L.k, lane);
    const int rem = (int)(end - base);
    int32_t Tv[4], Uv[4], Rv[4], Gv[4];
    float Kv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = lane + 64 * i;
      const bool in = j < rem;
      if constexpr (MODE == Mode::Product) {
        pd.at(in ? (uint32_t)(base + j - pc.s0) : 0u, Tv[i], Uv[i], Rv[i], Gv[i]);
        if (!HAS_GRID) Gv[i] = 1;
      } else if constexpr (MODE != Mode::Keys) {
        Tv[i] = in ? L.cfg.block[base + j] : 0;
        Uv[i] = in ? L.cfg.unroll[base + j] : 0;
        Rv[i] = in ? L.cfg.regs[base + j] : 0;
        Gv[i] = (HAS_GRID && in) ? L.cfg.grid[base + j] : 1;
      } else {
        Kv[i] = in ? L.keys[base + j] : __builtin_huge_valf();
      }
    }
    bool cand[4];
    uint64_t key[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = lane + 64 * i;
      const bool in = j < rem;
      const int64_t e = base + j;
      float sc;
      bool ok;
      if constexpr (MODE != Mode::Keys) {
        int32_t W;
        eval_cfg<HAS_GRID>(L.arch, tb, pc, Tv[i], Uv[i], Rv[i], Gv[i], in, L.need_score, W, sc);
        if (L.occ && in) L.occ[e] = W;
        if (L.score && in) L.score[e] = sc;
        ok = W > 0;
      } else {
        sc = Kv[i];
        ok = in && sc < __builtin_huge_valf();
      }
      const uint32_t kk = order_key(sc);
      cand[i] = ok && kk <= sel.theta;
      if constexpr (MODE == Mode::Suggest) cand[i] = cand[i] && in_kept(pc.kept, L.arch, Tv[i]);
      key[i] = ((uint64_t)kk << 32) | (uint32_t)(e - pc.s0);
    }
    if constexpr (TOPK) offer<4>(sel, cand, key);
  }

  struct Cols {
    IVec<ITEMS> T, U, R, G;
    FVec<ITEMS> K;
  };

  // `base` is wave-uniform: each column's chunk address is a scalar base
  // plus the lane's constant offset.
  __device__ __forceinline__ Cols load_chunk(int64_t base) const {
    Cols c;
    const int lo = ITEMS * lane;
    if constexpr (MODE == Mode::Product) {
      const uint32_t li = (uint32_t)(base - pc.s0) + (uint32_t)lo;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        pd.at(li + (uint32_t)i, c.T.v[i], c.U.v[i], c.R.v[i], c.G.v[i]);
        if (!HAS_GRID) c.G.v[i] = 1;
      }
    } else if constexpr (MODE != Mode::Keys) {
      c.T = *(const IVec<ITEMS> *)((L.cfg.block + base) + lo);
      c.U = *(const IVec<ITEMS> *)((L.cfg.unroll + base) + lo);
      c.R = *(const IVec<ITEMS> *)((L.cfg.regs + base) + lo);
      if (HAS_GRID) {
        c.G = *(const IVec<ITEMS> *)((L.cfg.grid + base) + lo);
      } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) c.G.v[i] = 1;
      }
    } else {
      c.K = *(const FVec<ITEMS> *)((L.keys + base) + lo);
    }
    return c;
  }

  __device__ __forceinline__ void chunk(const Cols &c, int64_t base) {
    const int64_t o = base + ITEMS * lane;
    float sc[ITEMS];
    int32_t W[ITEMS];
    bool ok[ITEMS];
    if constexpr (MODE != Mode::Keys) {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        eval_cfg<HAS_GRID>(L.arch, tb, pc, c.T.v[i], c.U.v[i], c.R.v[i], c.G.v[i], true, L.need_score, W[i], sc[i]);
        ok[i] = W[i] > 0;
      }
      const int off = 4 * ITEMS * lane;
      buf_store<ITEMS>(W, out_rsrc(L.occ, 4 * base, 4 * kC), off);
      buf_store<ITEMS>(sc, out_rsrc(L.score, 4 * base, 4 * kC), off);
    } else {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        sc[i] = c.K.v[i];
        ok[i] = sc[i] < __builtin_huge_valf();
      }
    }
    if constexpr (TOPK) {
      const uint32_t li = (uint32_t)(o - pc.s0);
      bool cand[ITEMS];
      uint64_t key[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        // model scores are +0 .. +inf: the key is the bit pattern with the
        // sign bit set, and +inf's key lies above every threshold
        const uint32_t kk = MODE != Mode::Keys ? (__float_as_uint(sc[i]) | 0x80000000u) : order_key(sc[i]);
        cand[i] = MODE != Mode::Keys ? kk <= sel.theta : (ok[i] && kk <= sel.theta);
        if constexpr (MODE == Mode::Suggest) cand[i] = cand[i] && in_kept(pc.kept, L.arch, c.T.v[i]);
        key[i] = ((uint64_t)kk << 32) | (li + (uint32_t)i);
      }
      offer<ITEMS>(sel, cand, key);
    }
  }

  // [e, pe) shared by nw waves, this one being wave w (nw = 1: one wave
  // alone): the unaligned head masked by wave 0, the aligned body's chunks
  // j = w, w + nw, ... vectorised with the next one's loads in flight while
  // the current one is evaluated, and the ragged tail's 256-row blocks dealt
  // out the same way.  Taking chunks in turn keeps the waves of a workgroup
  // on adjacent addresses, as a plain stream's are: each column is read
  // nw x 256 ITEMS contiguous bytes at a time rather than at nw fronts an
  // nw-th of the range apart (measured faster from HBM and from the
  // Infinity Cache alike).
  __device__ void run(int64_t e, int64_t pe, int w = 0, int nw = 1) {
    int64_t body = e;
    if (L.vec) {
      int64_t a0 = (e + ITEMS - 1) & ~(int64_t)(ITEMS - 1);
      a0 = uniform64(a0 < pe ? a0 : pe);  // keep the chunk bases in scalar registers
      if (w == 0 && a0 > e) masked(e, a0);
      const int64_t nfull = (pe - a0) / kC;
      const int64_t cnt = w < nfull ? (nfull - w + nw - 1) / nw : 0;
      if (cnt > 0) {
        const int64_t stride = (int64_t)nw * kC;
        const int64_t b0 = uniform64(a0 + (int64_t)w * kC);
        // Unrolled by two so that the chunk in flight and the chunk being
        // evaluated alternate between two register sets: a loop-carried copy
        // of the prefetched registers would make every iteration wait for all
        // outstanding memory operations, this chunk's stores included.  The
        // prefetches are unconditional (a conditional load would make the
        // compiler wait for it before evaluating); past the last chunk they
        // re-read one that is still cached.
        Cols a = load_chunk(b0);
        if constexpr (MODE != Mode::Keys) {
          // two dropped stores: the loop is entered with the same memory
          // operations behind the first prefetch as every later iteration
          // (a chunk's two output stores), so its waits stay exact
          const int32_t z[ITEMS] = {};
          buf_store<ITEMS>(z, out_rsrc(nullptr, 0, 0), 0);
          buf_store<ITEMS>(z, out_rsrc(nullptr, 0, 0), 4 * ITEMS * 64);
        }
        int64_t it = 0;
        for (; it + 2 <= cnt; it += 2) {
          const int64_t base = b0 + it * stride;
          if constexpr (TOPK) make_room(sel, kC, L.k, lane);
          const Cols b = load_chunk(base + stride);
          // keep the scheduler from hoisting this chunk's first uses above
          // the prefetch: the wait for the current data can then leave the
          // prefetch (and any stores before it) in flight
          __builtin_amdgcn_sched_barrier(0);
          chunk(a, base);
          if constexpr (TOPK) make_room(sel, kC, L.k, lane);
          a = load_chunk(it + 2 < cnt ? base + 2 * stride : base + stride);
          __builtin_amdgcn_sched_barrier(0);
          chunk(b, base + stride);
        }
        if (it < cnt) {
          if constexpr (TOPK) make_room(sel, kC, L.k, lane);
          chunk(a, b0 + it * stride);
        }
      }
      body = a0 + nfull * kC;
    }
    for (int64_t base = body + (int64_t)w * 256; base < pe; base += (int64_t)nw * 256)
      masked(base, (pe - base) < 256 ? pe : base + 256);
  }
};


// The product space travels as a kernel argument of the Product kernels only.
struct NoProduct {};
template <Mode MODE>
struct ProductArg {
  using type = NoProduct;
};
template <>
struct ProductArg<Mode::Product> {
  using type = KProduct;
};

template <Mode MODE, bool HAS_GRID, bool TOPK>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(SA_WAVES_PER_EU)))
void sa_eval_kernel(EvalLaunch L, typename ProductArg<MODE>::type P) {
  // Dynamic LDS: the occupancy table [rg][W_B] followed by waves-by-registers
  // per register-granule count.
  extern __shared__ __align__(16) uint8_t dyn_lds[];
  __shared__ float tab_rcap[kMaxWB + 1];
  __shared__ uint32_t tab_mwb[kMaxWB + 2];
  __shared__ uint8_t tab_blim[kMaxWB + 2];
  __shared__ WaveLds wl[kWavesPerBlock];
  __shared__ int32_t pvals[MODE == Mode::Product ? 4 * kProductMaxValues : 1];

  const KArch &A = L.arch;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int w = tid / kWaveSize;
  (void)A;
  if constexpr (MODE == Mode::Product) {
    for (int i = tid; i < 4 * kProductMaxValues; i += kBlockThreads)
      pvals[i] = P.vals[i / kProductMaxValues][i % kProductMaxValues];
  } else {
    (void)P;
  }
  // (the barrier at the end of build_tables also publishes pvals)
  if constexpr (MODE != Mode::Keys) build_tables(L, dyn_lds, tab_rcap, tab_mwb, tab_blim, tid, kBlockThreads);
  const uint8_t *tab_b = dyn_lds;

  const int64_t wt = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wt >= L.n_tiles) return;
  const int64_t t0 = wt * L.tile;
  const int64_t t1 = (t0 + L.tile < L.n_evals) ? t0 + L.tile : L.n_evals;
  const int64_t *seg = L.cfg.seg;
  const int64_t n_evals = L.n_evals;
  const int k = L.k;

  Selector sel;
  sel.buf = wl[w].cand;
  sel.count = 0;
  sel.theta = kThetaInit;
  const Tables tb{tab_b, tab_rcap};

  // product spaces: every segment has P.size evaluations, no offsets to read
  int64_t v;
  if constexpr (MODE == Mode::Product)
    v = t0 / P.size;
  else
    v = find_segment(seg, L.n_var, n_evals, t0, lane);
  int64_t e = t0;
  for (; v < L.n_var && e < t1; ++v) {
    int64_t s0, s1;
    if constexpr (MODE == Mode::Product) {
      s0 = v * P.size;
      s1 = s0 + P.size;
    } else {
      s0 = uniform64(clamp_off(seg[v], n_evals));
      s1 = uniform64(clamp_off(seg[v + 1], n_evals));
    }
    int64_t pe = s1 > e ? s1 : e;
    pe = pe < t1 ? pe : t1;
    if (pe <= e) continue;

    Piece pc;
    setup_piece<MODE>(L, pc, wl[w], v, s0, lane);
    if constexpr (MODE == Mode::Suggest)
      pc.kept = kept_mask(full_occupancy_mask(A, tab_b), A.nw, L.var.n_fp[v], L.var.n_ld[v], L.var.n_st[v]);

    if constexpr (TOPK) {
      sel.count = 0;
      sel.theta = kThetaInit;
    }
    Evaluator<MODE, HAS_GRID, TOPK, 4> ev{L, tb, pc, sel, lane};
    if constexpr (MODE == Mode::Product)
      ev.pd = ProductDigits{pvals, (uint32_t)P.n[3], (uint32_t)P.n[2], (uint32_t)P.n[1],
                            (uint32_t)P.n[0] - 1u, P.magic[0], P.magic[1], P.magic[2]};
    ev.run(e, pe);

    if constexpr (TOPK) {
      const uint64_t mine = select_k(sel, k, lane);
      if (e == s0 && pe == s1) {
        write_final(mine, k, lane, v, L.topk_idx, L.topk_val, MODE == Mode::Keys ? L.keys : nullptr, s0);
      } else {
        const int64_t slot = 2 * wt + (e == t0 ? 0 : 1);
        if (lane < k) L.frag[slot * k + lane] = mine;
      }
    }
    e = pe;
  }
}

// Combine the k-key fragments of every piece of segment v (which spans the
// wave-tiles ta .. tb, ta < tb) into its final row.
__device__ void merge_segment(const EvalLaunch &L, Selector &sel, int64_t v, int64_t s0, int64_t s1, int lane) {
  const int k = L.k;
  const int64_t T = L.tile;
  const int64_t ta = s0 / T, tb = (s1 - 1) / T;
  sel.count = 0;
  sel.theta = kThetaInit;
  const int64_t n_keys = (tb - ta + 1) * k;
  for (int64_t base = 0; base < n_keys; base += 64) {
    const int64_t j = base + lane;
    uint64_t key = kKeyNone;
    if (j < n_keys) {
      const int64_t p = j / k, r = j - p * k;
      const int64_t t = ta + p;
      const int64_t slot = (t == ta && s0 != ta * T) ? 2 * t + 1 : 2 * t;
      if (slot < 2 * L.n_tiles) key = L.frag[slot * k + r];
    }
    make_room(sel, 64, k, lane);
    const bool cand[1] = {key != kKeyNone && (uint32_t)(key >> 32) <= sel.theta};
    const uint64_t keys1[1] = {key};
    offer<1>(sel, cand, keys1);
  }
  const uint64_t mine = select_k(sel, k, lane);
  write_final(mine, k, lane, v, L.topk_idx, L.topk_val, L.keys, s0);
}

// Second pass of the two-launch path: merge segments that span wave-tiles
// and write the padding row of empty segments.  One wave per variant.
__global__ __launch_bounds__(kBlockThreads) void sa_merge_kernel(EvalLaunch L) {
  __shared__ uint64_t cand[kWavesPerBlock][kCandCap];
  const int lane = lane_id();
  const int w = threadIdx.x / kWaveSize;
  const int64_t n_evals = L.n_evals;
  Selector sel;
  sel.buf = cand[w];
  for (int64_t v = (int64_t)blockIdx.x * kWavesPerBlock + w; v < L.n_var; v += (int64_t)gridDim.x * kWavesPerBlock) {
    const int64_t s0 = uniform64(clamp_off(L.cfg.seg[v], n_evals));
    const int64_t s1 = uniform64(clamp_off(L.cfg.seg[v + 1], n_evals));
    if (s1 <= s0) {
      write_final(kKeyNone, L.k, lane, v, L.topk_idx, L.topk_val, nullptr, 0);
      continue;
    }
    if (s0 / L.tile == (s1 - 1) / L.tile) continue;  // inside one wave-tile: already final
    merge_segment(L, sel, v, s0, s1, lane);
  }
}

// ---------------------------------------------------------------- planned batches

// Persistent kernel over a plan's workgroup items (the plan lists them
// longest first).  Workgroup j takes item j; with more items than workgroups
// the rest are taken from the plan's queue, one ticket per item, the next
// ticket fetched while the current item is evaluated, so that the workgroups
// finish close together whatever the item sizes.  A launch takes exactly
// n_items tickets (n_items - G items, then one empty ticket per workgroup),
// and the workgroup holding the last one returns the counter to zero for the
// next launch (stream-ordered launches of one plan, replayed graphs
// included).  kind 0 items: each wave evaluates whole segments and writes
// their rows.  kind 1 items: the waves take the chunks of one segment's range
// in turn, each selecting over its own, the selections meet in LDS and wave
// 0 writes the row (or the item's fragment).
template <Mode MODE, bool HAS_GRID, bool TOPK, int ITEMS, int WPB>
// (at most 128 registers: four waves per SIMD at every shape that fits them)
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(4))) void sa_plan_kernel(EvalLaunch L,
                                                                                                   PlanDev P) {
  extern __shared__ __align__(16) uint8_t dyn_lds[];
  __shared__ float tab_rcap[kMaxWB + 1];
  __shared__ uint32_t tab_mwb[kMaxWB + 2];
  __shared__ uint8_t tab_blim[kMaxWB + 2];
  __shared__ WaveLds wl[WPB];
  __shared__ uint64_t wgk[WPB][SA_K_MAX];
  __shared__ uint32_t s_ticket;

  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int w = tid / kWaveSize;
  if constexpr (MODE != Mode::Keys) build_tables(L, dyn_lds, tab_rcap, tab_mwb, tab_blim, tid, 64 * WPB);
  const Tables tb{dyn_lds, tab_rcap};
  const int64_t n_evals = L.n_evals;
  const int64_t *seg = L.cfg.seg;
  const int k = L.k;
  Selector sel;
  sel.buf = wl[w].cand;
  sel.count = 0;
  sel.theta = kThetaInit;

  const uint32_t n_items = (uint32_t)P.n_items, n_wg = gridDim.x;
  const bool queued = n_items > n_wg;
  uint32_t ticket = blockIdx.x;
  while (ticket < n_items) {
    const int64_t item = ticket;
    uint32_t next = n_items;
    if (queued) {
      __syncthreads();  // every wave has read s_ticket
      if (tid == 0) {
        const uint32_t t = atomicAdd(&P.queue[0], 1u);
        if (t == n_items - 1u) atomicExch(&P.queue[0], 0u);  // the launch's last ticket
        next = n_wg + t;
      }
    }
    const PlanItem it = P.items[item];
    if (it.kind == 0) {
      const PlanWave pw = P.waves[item * WPB + w];
      const int64_t v1 = pw.v1 < L.n_var ? pw.v1 : L.n_var;
      for (int64_t v = pw.v0 > 0 ? pw.v0 : 0; v < v1; ++v) {
        const int64_t s0 = uniform64(clamp_off(seg[v], n_evals));
        const int64_t s1 = uniform64(clamp_off(seg[v + 1], n_evals));
        if (s1 <= s0) {
          if constexpr (TOPK) write_final(kKeyNone, k, lane, v, L.topk_idx, L.topk_val, nullptr, 0);
          continue;
        }
        Piece pc;
        setup_piece<MODE>(L, pc, wl[w], v, s0, lane);
        sel.count = 0;
        sel.theta = kThetaInit;
        Evaluator<MODE, HAS_GRID, TOPK, ITEMS> ev{L, tb, pc, sel, lane};
        ev.run(s0, s1);
        if constexpr (TOPK) {
          const uint64_t mine = select_k(sel, k, lane);
          write_final(mine, k, lane, v, L.topk_idx, L.topk_val, MODE == Mode::Keys ? L.keys : nullptr, s0);
        }
      }
    } else {
      const int64_t v = it.v < L.n_var ? (it.v > 0 ? it.v : 0) : L.n_var - 1;
      const int64_t s0 = uniform64(clamp_off(seg[v], n_evals));
      const int64_t s1 = uniform64(clamp_off(seg[v + 1], n_evals));
      // the item's range: from its first part's start to its last part's end
      const int64_t f0 = P.waves[item * WPB].e0, f1 = P.waves[item * WPB + WPB - 1].e1;
      const int64_t e0 = f0 > s0 ? f0 : s0;
      const int64_t e1 = f1 < s1 ? f1 : s1;
      uint64_t mine = kKeyNone;
      if (e1 > e0) {
        Piece pc;
        setup_piece<MODE>(L, pc, wl[w], v, s0, lane);
        sel.count = 0;
        sel.theta = kThetaInit;
        Evaluator<MODE, HAS_GRID, TOPK, ITEMS> ev{L, tb, pc, sel, lane};
        ev.run(uniform64(e0), uniform64(e1), w, WPB);
        if constexpr (TOPK) mine = select_k(sel, k, lane);
      }
      if constexpr (TOPK) {
        if (lane < k) wgk[w][lane] = mine;
      }
    }
    // only a split item's waves meet (kind is uniform over the workgroup, so
    // every wave takes the same barriers); a packing item's waves go on to
    // their next item without waiting for each other
    if (TOPK && it.kind == 1) {
      __syncthreads();
      if (w == 0) {
        const int64_t v = it.v < L.n_var ? (it.v > 0 ? it.v : 0) : L.n_var - 1;
        const int64_t s0 = uniform64(clamp_off(seg[v], n_evals));
        // The waves' lists are sorted (kKeyNone last) and their keys distinct
        // (local indices), so a key's place among all of them is its place in
        // its own list plus the keys below it in each other list (a lower
        // bound by bisection); the keys placed below k are the item's k
        // smallest, in order.  Wave 0's candidate buffer is free to hold them.
        uint64_t *out = sel.buf;
        if (lane < k) out[lane] = kKeyNone;
        wave_lds_sync();
        for (int j = lane; j < WPB * k; j += 64) {
          const int a = j / k, r = j - a * k;
          const uint64_t key = wgk[a][r];
          if (key == kKeyNone) continue;
          int place = r;
#pragma unroll 1
          for (int b = 0; b < WPB; ++b) {
            if (b == a) continue;
            int lo = 0, hi = k;
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              if (wgk[b][mid] < key) lo = mid + 1; else hi = mid;
            }
            place += lo;
          }
          if (place < k) out[place] = key;
        }
        wave_lds_sync();
        const uint64_t m = lane < k ? out[lane] : kKeyNone;
        if (it.slot < 0) {
          write_final(m, k, lane, v, L.topk_idx, L.topk_val, MODE == Mode::Keys ? L.keys : nullptr, s0);
        } else if (lane < k) {
          L.frag[(int64_t)it.slot * k + lane] = m;
        }
      }
      __syncthreads();
    }
    if (!queued) break;
    if (tid == 0) s_ticket = next;
    __syncthreads();
    ticket = s_ticket;
  }
}

// Combine the fragments of segments a plan split over several workgroup
// items.  One wave per split record.
__global__ __launch_bounds__(kBlockThreads) void sa_split_merge_kernel(EvalLaunch L, PlanDev P) {
  __shared__ uint64_t cand[kWavesPerBlock][kCandCap];
  const int lane = lane_id();
  const int w = threadIdx.x / kWaveSize;
  const int k = L.k;
  Selector sel;
  sel.buf = cand[w];
  for (int64_t i = (int64_t)blockIdx.x * kWavesPerBlock + w; i < P.n_splits; i += (int64_t)gridDim.x * kWavesPerBlock) {
    const PlanSplit sp = P.splits[i];
    const int64_t v = sp.v;
    if (v < 0 || v >= L.n_var) continue;
    const int64_t s0 = uniform64(clamp_off(L.cfg.seg[v], L.n_evals));
    sel.count = 0;
    sel.theta = kThetaInit;
    const int64_t n_keys = sp.n_slots * k;
    for (int64_t base = 0; base < n_keys; base += 64) {
      const int64_t j = base + lane;
      const uint64_t key = j < n_keys ? L.frag[sp.first_slot * k + j] : kKeyNone;
      make_room(sel, 64, k, lane);
      const bool c[1] = {key != kKeyNone && (uint32_t)(key >> 32) <= sel.theta};
      const uint64_t keys1[1] = {key};
      offer<1>(sel, c, keys1);
    }
    const uint64_t mine = select_k(sel, k, lane);
    write_final(mine, k, lane, v, L.topk_idx, L.topk_val, L.keys, s0);
  }
}

template <Mode M, bool G, bool K, int I, int WPB>
hipError_t launch_plan_one(const EvalLaunch &L, const PlanDev &P, int n_cu, hipStream_t stream) {
  if (P.n_items == 0) return hipSuccess;
  const size_t dyn = M != Mode::Keys ? (size_t)L.dyn_lds_bytes : 0;
  static thread_local int resident = -1;  // workgroups per CU for this instantiation
  static thread_local size_t resident_dyn = (size_t)-1;
  if (resident < 0 || resident_dyn != dyn) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sa_plan_kernel<M, G, K, I, WPB>, 64 * WPB, dyn) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    resident = nb;
    resident_dyn = dyn;
  }
  int64_t grid = (int64_t)resident * n_cu;
  if (grid > P.n_items) grid = P.n_items;
  hipLaunchKernelGGL((sa_plan_kernel<M, G, K, I, WPB>), dim3((uint32_t)grid), dim3(64 * WPB), dyn, stream, L, P);
  return hipGetLastError();
}

template <Mode M, bool G, bool K>
hipError_t launch_plan_shape(const EvalLaunch &L, const PlanDev &P, const PlanShape &S, int n_cu, hipStream_t stream) {
#define SA_SHAPE(I, W) \
  if (S.items == I && S.wpb == W) return launch_plan_one<M, G, K, I, W>(L, P, n_cu, stream);
  SA_SHAPE(1, 4) SA_SHAPE(2, 4) SA_SHAPE(4, 4)
  SA_SHAPE(1, 8) SA_SHAPE(2, 8) SA_SHAPE(4, 8)
  SA_SHAPE(1, 16) SA_SHAPE(2, 16) SA_SHAPE(4, 16)
#undef SA_SHAPE
  return hipErrorInvalidValue;
}

template <Mode M, bool G, bool K>
hipError_t launch_one(const EvalLaunch &L, hipStream_t stream) {
  const int64_t blocks = (L.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks == 0) return hipSuccess;
  const size_t dyn = M != Mode::Keys ? (size_t)L.dyn_lds_bytes : 0;
  hipLaunchKernelGGL((sa_eval_kernel<M, G, K>), dim3((uint32_t)blocks), dim3(kBlockThreads), dyn, stream, L,
                     NoProduct{});
  return hipGetLastError();
}

template <bool G, bool K>
hipError_t launch_one_product(const EvalLaunch &L, const KProduct &P, hipStream_t stream) {
  const int64_t blocks = (L.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((sa_eval_kernel<Mode::Product, G, K>), dim3((uint32_t)blocks), dim3(kBlockThreads),
                     (size_t)L.dyn_lds_bytes, stream, L, P);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eval(const EvalLaunch &L, Mode mode, bool has_grid, bool topk, hipStream_t stream) {
  if (mode == Mode::Suggest) {
    if (!topk) return hipErrorInvalidValue;
    return has_grid ? launch_one<Mode::Suggest, true, true>(L, stream) : launch_one<Mode::Suggest, false, true>(L, stream);
  }
  if (mode == Mode::Keys) {
    return topk ? launch_one<Mode::Keys, false, true>(L, stream) : hipErrorInvalidValue;
  }
  if (has_grid) {
    return topk ? launch_one<Mode::Model, true, true>(L, stream) : launch_one<Mode::Model, true, false>(L, stream);
  }
  return topk ? launch_one<Mode::Model, false, true>(L, stream) : launch_one<Mode::Model, false, false>(L, stream);
}

hipError_t launch_product(const EvalLaunch &L, const KProduct &P, bool has_grid, bool topk, hipStream_t stream) {
  if (has_grid)
    return topk ? launch_one_product<true, true>(L, P, stream) : launch_one_product<true, false>(L, P, stream);
  return topk ? launch_one_product<false, true>(L, P, stream) : launch_one_product<false, false>(L, P, stream);
}

hipError_t launch_plan(const EvalLaunch &L, const PlanDev &P, const PlanShape &S, Mode mode, bool has_grid, bool topk,
                       int n_cu, hipStream_t stream) {
  if (mode == Mode::Keys) {
    return topk ? launch_plan_shape<Mode::Keys, false, true>(L, P, S, n_cu, stream) : hipErrorInvalidValue;
  }
  if (has_grid) {
    return topk ? launch_plan_shape<Mode::Model, true, true>(L, P, S, n_cu, stream)
                : launch_plan_shape<Mode::Model, true, false>(L, P, S, n_cu, stream);
  }
  return topk ? launch_plan_shape<Mode::Model, false, true>(L, P, S, n_cu, stream)
              : launch_plan_shape<Mode::Model, false, false>(L, P, S, n_cu, stream);
}

hipError_t launch_split_merge(const EvalLaunch &L, const PlanDev &P, hipStream_t stream) {
  if (P.n_splits == 0) return hipSuccess;
  int64_t blocks = (P.n_splits + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(sa_split_merge_kernel, dim3((uint32_t)blocks), dim3(kBlockThreads), 0, stream, L, P);
  return hipGetLastError();
}

namespace {
// Per variant, the block sizes the paper's reduction keeps (bit j = T of
// ws (j + 1) threads).
__global__ __launch_bounds__(kBlockThreads) void sa_suggest_kernel(EvalLaunch L, uint64_t *kept) {
  extern __shared__ __align__(16) uint8_t dyn_lds[];
  __shared__ float tab_rcap[kMaxWB + 1];
  __shared__ uint32_t tab_mwb[kMaxWB + 2];
  __shared__ uint8_t tab_blim[kMaxWB + 2];
  build_tables(L, dyn_lds, tab_rcap, tab_mwb, tab_blim, threadIdx.x, kBlockThreads);
  const uint64_t full = full_occupancy_mask(L.arch, dyn_lds);
  for (int64_t v = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x; v < L.n_var;
       v += (int64_t)gridDim.x * kBlockThreads)
    kept[v] = kept_mask(full, L.arch.nw, L.var.n_fp[v], L.var.n_ld[v], L.var.n_st[v]);
}

// Headroom at full occupancy for each row's block size (Sec. III-C): the last
// register-granule row of the occupancy table that keeps full occupancy at
// this W_B (rows never gain occupancy as registers grow), and the largest LDS
// allocation that leaves room for the table's block count, floor(floor(pool /
// B) / granule) granules (Eq. 5 with a floor).
__global__ __launch_bounds__(kBlockThreads) void sa_headroom_kernel(EvalLaunch L, const int32_t *block,
                                                                    const int32_t *regs, int64_t n, int32_t *r_star,
                                                                    int32_t *s_star) {
  extern __shared__ __align__(16) uint8_t dyn_lds[];
  __shared__ float tab_rcap[kMaxWB + 1];
  __shared__ uint32_t tab_mwb[kMaxWB + 2];
  __shared__ uint8_t tab_blim[kMaxWB + 2];
  build_tables(L, dyn_lds, tab_rcap, tab_mwb, tab_blim, threadIdx.x, kBlockThreads);
  const KArch &A = L.arch;
  const uint8_t *tab_b = dyn_lds;
  const int32_t row = A.nw + 2;
  for (int64_t i = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlockThreads) {
    const int32_t T = block[i];
    const int32_t R = regs ? regs[i] : 0;
    int32_t rs = 0, ss = 0;
    if ((uint32_t)(T - 1) < (uint32_t)A.max_threads && (uint32_t)R <= (uint32_t)A.max_vgprs) {
      const int32_t WB = (T + A.ws - 1) >> A.ws_shift;
      const int32_t B0 = tab_b[WB];
      if (B0 * WB == A.max_waves) {
        int32_t g = 0;
        for (int32_t rg = 1; rg <= A.nr && (int32_t)tab_b[rg * row + WB] * WB == A.max_waves; ++rg) g = rg;
        const int32_t rmax = g << A.gran_shift;
        rs = rmax > R ? rmax - R : 0;
        const int32_t alloc = (A.lds_cu / B0) / A.lds_gran * A.lds_gran;
        ss = alloc < A.max_lds ? alloc : A.max_lds;
      }
    }
    if (r_star) r_star[i] = rs;
    if (s_star) s_star[i] = ss;
  }
}
}  // namespace

hipError_t launch_headroom(const EvalLaunch &L, const int32_t *block, const int32_t *regs, int64_t n, int32_t *r_star,
                           int32_t *s_star, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + kBlockThreads - 1) / kBlockThreads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(sa_headroom_kernel, dim3((uint32_t)blocks), dim3(kBlockThreads), (size_t)L.dyn_lds_bytes,
                     stream, L, block, regs, n, r_star, s_star);
  return hipGetLastError();
}

hipError_t launch_suggest(const EvalLaunch &L, uint64_t *kept, hipStream_t stream) {
  if (L.n_var == 0) return hipSuccess;
  int64_t blocks = (L.n_var + kBlockThreads - 1) / kBlockThreads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(sa_suggest_kernel, dim3((uint32_t)blocks), dim3(kBlockThreads), (size_t)L.dyn_lds_bytes, stream,
                     L, kept);
  return hipGetLastError();
}

hipError_t launch_merge(const EvalLaunch &L, hipStream_t stream) {
  if (L.n_var == 0) return hipSuccess;
  int64_t blocks = (L.n_var + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(sa_merge_kernel, dim3((uint32_t)blocks), dim3(kBlockThreads), 0, stream, L);
  return hipGetLastError();
}

}  // namespace sa
