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

#include "sa_internal.h"

namespace sa {
namespace {

constexpr uint64_t kKeyNone = ~0ull;
constexpr uint32_t kThetaInit = 0xFF7FFFFFu;  // order key of FLT_MAX
constexpr int32_t kUnlimited = 1 << 30;
#ifndef SA_NT_STORE
#define SA_NT_STORE 1
#endif
#ifndef SA_WAVES_PER_EU
#define SA_WAVES_PER_EU 4
#endif

typedef int32_t v4i32 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

// Streaming 16-byte stores of the per-evaluation outputs.
__device__ __forceinline__ void store4(int32_t *p, int32_t a, int32_t b, int32_t c, int32_t d) {
  const v4i32 v = {a, b, c, d};
  if (SA_NT_STORE) __builtin_nontemporal_store(v, (v4i32 *)p);
  else *(v4i32 *)p = v;
}
__device__ __forceinline__ void store4(float *p, float a, float b, float c, float d) {
  const v4f32 v = {a, b, c, d};
  if (SA_NT_STORE) __builtin_nontemporal_store(v, (v4f32 *)p);
  else *(v4f32 *)p = v;
}

// Order-preserving map of binary32 to uint32 (negative values flipped, -0
// ordered as +0 so equal values tie and fall back to the index).
__device__ __forceinline__ uint32_t order_key(float f) {
  uint32_t b = __float_as_uint(f);
  b = (b == 0x80000000u) ? 0u : b;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float order_key_inv(uint32_t k) {
  uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(b);
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Orders this wave's LDS accesses before/after (LDS ops of one wave complete
// in order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Minimum over the 64 lanes: four DPP steps leave every lane of a 16-lane row
// holding the row minimum, then the four row minima are combined.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_min(uint32_t v) {
  uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false);
  return o < v ? o : v;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = dpp_min<0xB1>(v);   // quad_perm [1,0,3,2]
  v = dpp_min<0x4E>(v);   // quad_perm [2,3,0,1]
  v = dpp_min<0x141>(v);  // row_half_mirror
  v = dpp_min<0x140>(v);  // row_mirror
  uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
  uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
  uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
  uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
  a = a < b ? a : b;
  c = c < d ? c : d;
  return a < c ? a : c;
}

// Clamp a segment offset into [0, n]: keeps every access in bounds even when
// the offsets are not a valid CSR.
__device__ __forceinline__ int64_t clamp_off(int64_t s, int64_t n) { return s < 0 ? 0 : (s > n ? n : s); }

// Largest v in [0, n_var) with seg[v] <= e (the segment containing e).  A
// 64-ary search: each step probes 64 offsets at once.
__device__ int64_t find_segment(const int64_t *seg, int64_t n_var, int64_t n_evals, int64_t e, int lane) {
  int64_t lo = 0, hi = n_var;
  while (hi - lo > 1) {
    int64_t step = (hi - lo + 63) / 64;
    int64_t p = lo + (int64_t)lane * step;
    bool pred = (p < hi) && clamp_off(seg[p < hi ? p : lo], n_evals) <= e;
    uint64_t m = __ballot(pred);
    int c = __popcll(m);
    if (c == 0) c = 1;
    lo = uniform64(lo + (int64_t)(c - 1) * step);
    int64_t nh = lo + step;
    hi = uniform64(nh < hi ? nh : hi);
  }
  return lo;
}

// Floor division a / b for 0 <= a < 2^21, 1 <= b < 2^21, given rcp ~ 1/b to
// within a few ulp: the float estimate is within 1 of the quotient, one
// correction step each way makes it exact.
__device__ __forceinline__ int32_t udiv_rcp(int32_t a, int32_t b, float rcp) {
  int32_t q = (int32_t)((float)a * rcp);
  int32_t r = a - (int32_t)__umul24((uint32_t)q, (uint32_t)b);
  q = (r < 0) ? q - 1 : q;
  r = (r < 0) ? r + b : r;
  q = (r >= b) ? q + 1 : q;
  return q;
}

// ---------------------------------------------------------------- selection

struct Selector {
  uint64_t *buf;   // this wave's candidate buffer (kCandCap keys, LDS)
  uint32_t count;  // keys in buf (uniform)
  uint32_t theta;  // order key of the current k-th best score (uniform)
};

__device__ __forceinline__ void cas64(uint64_t &a, uint64_t &b) {
  uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
  a = lo;
  b = hi;
}

// Reduce buf[0, count) to its k smallest keys: afterwards lane r < found holds
// the r-th smallest (kKeyNone elsewhere), buf[0, found) holds them too and
// theta is the k-th smallest score when k keys exist.  Each lane sorts its
// eight keys (Batcher's odd-even merge network); each of the k rounds takes
// the minimum of the lane heads and the owner pops its head.
__device__ uint64_t select_k(Selector &s, int k, int lane) {
  static_assert(kCandCap == 8 * 64, "select_k holds eight keys per lane");
  wave_lds_sync();
  const uint32_t i0 = 8u * (uint32_t)lane;
  uint64_t r[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = i0 + j < s.count ? s.buf[i0 + j] : kKeyNone;
  cas64(r[0], r[1]); cas64(r[2], r[3]); cas64(r[4], r[5]); cas64(r[6], r[7]);
  cas64(r[0], r[2]); cas64(r[1], r[3]); cas64(r[4], r[6]); cas64(r[5], r[7]);
  cas64(r[1], r[2]); cas64(r[5], r[6]);
  cas64(r[0], r[4]); cas64(r[1], r[5]); cas64(r[2], r[6]); cas64(r[3], r[7]);
  cas64(r[2], r[4]); cas64(r[3], r[5]);
  cas64(r[1], r[2]); cas64(r[3], r[4]); cas64(r[5], r[6]);
  uint64_t mine = kKeyNone;
  int found = 0;
  uint32_t last_hi = 0;
  for (int q = 0; q < k; ++q) {
    const uint32_t hi = (uint32_t)(r[0] >> 32), lo = (uint32_t)r[0];
    const uint32_t mh = wave_min_u32(hi);
    if (mh == 0xFFFFFFFFu) break;
    const uint64_t tie = __ballot(hi == mh);
    int owner;
    uint32_t ml;
    if (__popcll(tie) == 1) {
      owner = __ffsll((long long)tie) - 1;
      ml = (uint32_t)__builtin_amdgcn_readlane((int)lo, owner);
    } else {
      ml = wave_min_u32(hi == mh ? lo : 0xFFFFFFFFu);
      owner = __ffsll((long long)__ballot(hi == mh && lo == ml)) - 1;
    }
    if (lane == q) mine = ((uint64_t)mh << 32) | ml;
    if (lane == owner) {
#pragma unroll
      for (int j = 0; j < 7; ++j) r[j] = r[j + 1];
      r[7] = kKeyNone;
    }
    last_hi = mh;
    ++found;
  }
  wave_lds_sync();
  if (lane < found) s.buf[lane] = mine;
  s.count = (uint32_t)found;
  if (found == k) s.theta = last_hi;
  wave_lds_sync();
  return mine;
}

// Flush the buffer when fewer than `need` slots are free.  Called before a
// batch is evaluated, where few registers are live.
__device__ __forceinline__ void make_room(Selector &s, uint32_t need, int k, int lane) {
  if (s.count + need > (uint32_t)kCandCap) select_k(s, k, lane);
}

// Offer N rows of 64 keys (`cand[i]` marks the lanes offering key[i]) by
// ballot + mbcnt compaction; make_room(64 N) must have run first.
template <int N>
__device__ __forceinline__ void offer(Selector &s, const bool (&cand)[N], const uint64_t (&key)[N]) {
  static_assert(N * 64 + SA_K_MAX <= kCandCap, "buffer must hold k keys plus one batch");
  uint64_t bal[N];
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    bal[i] = __ballot(cand[i]);
    c += (uint32_t)__popcll(bal[i]);
  }
  if (c == 0) return;
  uint32_t pos = s.count;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (cand[i]) s.buf[pos + mbcnt64(bal[i])] = key[i];
    pos += (uint32_t)__popcll(bal[i]);
  }
  s.count = pos;
}

// Final row of variant v.  Values come from the key, or (keys mode) from the
// caller's array so that the sign of a zero key survives.
__device__ __forceinline__ void write_final(uint64_t mine, int k, int lane, int64_t v, int32_t *idx, float *val,
                                            const float *keys, int64_t s0) {
  if (lane < k) {
    const bool none = (mine == kKeyNone);
    const int32_t li = (int32_t)(uint32_t)mine;
    if (idx) idx[v * k + lane] = none ? -1 : li;
    if (val) {
      float x = __builtin_huge_valf();
      if (!none) x = keys ? keys[s0 + li] : order_key_inv((uint32_t)(mine >> 32));
      val[v * k + lane] = x;
    }
  }
}

// ---------------------------------------------------------------- evaluation

struct __align__(16) WaveLds {
  float a4[kMaxUnroll];  // (c_ctrl n_br) / U for U = 1 .. max_unroll
  float a5[kMaxWB + 1];  // c_sync (n_bar W_B)    for W_B = 1 .. nw
  uint64_t cand[kCandCap];
};

// Wave-uniform state of the piece being evaluated.
struct Piece {
  bool valid;      // variant counts in range
  int32_t gs;      // Eq. 5 bound for the variant's LDS
  float P, D;      // Eq. 6 per-variant sum, divergence weight 1 + d
  int64_t s0;      // segment start (local index origin)
  const float *a4, *a5;
};

struct Tables {
  const uint8_t *tab_b;  // [rg][W_B] -> min(G_W, G_R)
  const float *rcap;     // [B] -> 1 / (n_cu B)
};

// One configuration: W* (0 if illegal) and the binary32 score (+inf if
// illegal or not asked for).  Products of small non-negative integers use
// the full-rate 24-bit multiplier (every operand here is below 2^24).
template <bool HAS_GRID>
__device__ __forceinline__ void eval_cfg(const KArch &A, const Tables &tb, const Piece &pc, int32_t T, int32_t U,
                                         int32_t R, int32_t G, bool in, bool need_score, int32_t &W, float &sc) {
  // bitwise '&' keeps the legality test free of branches
  bool ok = in & pc.valid & ((uint32_t)(T - 1) < (uint32_t)A.max_threads) &
            ((uint32_t)(U - 1) < (uint32_t)A.max_unroll) & ((uint32_t)R <= (uint32_t)A.max_vgprs);
  if (HAS_GRID) ok = ok & ((uint32_t)(G - 1) < (uint32_t)A.max_grid);
  // only the table indices need sanitising; G of an illegal lane is discarded
  T = ok ? T : 1;
  U = ok ? U : 1;
  R = ok ? R : 0;
  // Eqs. 1-5: waves per block, register granules, bound table, LDS bound
  const int32_t WB = (T + A.ws - 1) >> A.ws_shift;
  const int32_t rg = (R + (1 << A.gran_shift) - 1) >> A.gran_shift;
  int32_t B = tb.tab_b[__umul24(rg, A.nw + 1) + WB];
  B = B < pc.gs ? B : pc.gs;
  B = ok ? B : 0;
  W = __umul24(B, WB);
  sc = __builtin_huge_valf();
  if (need_score) {
    // Eq. 6 per-configuration part, fixed binary32 order
    float E = pc.P + pc.a4[U - 1];
    E = E + pc.a5[WB];
    const float Ed = E * pc.D;
    const int32_t x = __umul24(W, U);
    const int32_t hide = x > A.w_sat ? x : A.w_sat;
    int32_t num, den;
    if (HAS_GRID) {
      const int32_t cap = __umul24(A.n_cu, B);
      const int32_t rounds = udiv_rcp(G + cap - 1, cap, tb.rcap[B]);
      num = __umul24(__umul24(rounds, cap), hide);
      den = __umul24(G, x);
    } else {
      num = hide;
      den = x;
    }
    const float F = (float)num / (float)den;
    sc = (B > 0) ? Ed * F : __builtin_huge_valf();
  }
}

// N consecutive int32 / binary32 values of one lane (one 4N-byte access).
template <int N>
struct alignas(4 * N) IVec {
  int32_t v[N];
};
template <int N>
struct alignas(4 * N) FVec {
  float v[N];
};

template <int N>
__device__ __forceinline__ void store_n(int32_t *p, const int32_t (&x)[N]) {
  if constexpr (N == 4) {
    store4(p, x[0], x[1], x[2], x[3]);
  } else {
    IVec<N> t;
#pragma unroll
    for (int i = 0; i < N; ++i) t.v[i] = x[i];
    *(IVec<N> *)p = t;
  }
}
template <int N>
__device__ __forceinline__ void store_n(float *p, const float (&x)[N]) {
  if constexpr (N == 4) {
    store4(p, x[0], x[1], x[2], x[3]);
  } else {
    FVec<N> t;
#pragma unroll
    for (int i = 0; i < N; ++i) t.v[i] = x[i];
    *(FVec<N> *)p = t;
  }
}

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
      if constexpr (MODE == Mode::Model) {
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
      if constexpr (MODE == Mode::Model) {
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
      key[i] = ((uint64_t)kk << 32) | (uint32_t)(e - pc.s0);
    }
    if constexpr (TOPK) offer<4>(sel, cand, key);
  }

  struct Cols {
    IVec<ITEMS> T, U, R, G;
    FVec<ITEMS> K;
  };

  __device__ __forceinline__ Cols load_chunk(int64_t base) const {
    Cols c;
    const int64_t o = base + ITEMS * lane;
    if constexpr (MODE == Mode::Model) {
      c.T = *(const IVec<ITEMS> *)(L.cfg.block + o);
      c.U = *(const IVec<ITEMS> *)(L.cfg.unroll + o);
      c.R = *(const IVec<ITEMS> *)(L.cfg.regs + o);
      if (HAS_GRID) {
        c.G = *(const IVec<ITEMS> *)(L.cfg.grid + o);
      } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) c.G.v[i] = 1;
      }
    } else {
      c.K = *(const FVec<ITEMS> *)(L.keys + o);
    }
    return c;
  }

  __device__ __forceinline__ void chunk(const Cols &c, int64_t base) {
    const int64_t o = base + ITEMS * lane;
    float sc[ITEMS];
    int32_t W[ITEMS];
    bool ok[ITEMS];
    if constexpr (MODE == Mode::Model) {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        eval_cfg<HAS_GRID>(L.arch, tb, pc, c.T.v[i], c.U.v[i], c.R.v[i], c.G.v[i], true, L.need_score, W[i], sc[i]);
        ok[i] = W[i] > 0;
      }
      if (L.occ) store_n<ITEMS>(L.occ + o, W);
      if (L.score) store_n<ITEMS>(L.score + o, sc);
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
        const uint32_t kk = MODE == Mode::Model ? (__float_as_uint(sc[i]) | 0x80000000u) : order_key(sc[i]);
        cand[i] = MODE == Mode::Model ? kk <= sel.theta : (ok[i] && kk <= sel.theta);
        key[i] = ((uint64_t)kk << 32) | (li + (uint32_t)i);
      }
      offer<ITEMS>(sel, cand, key);
    }
  }

  // [e, pe): unaligned head and ragged tail masked, aligned body vectorised
  // with the next chunk's loads in flight while the current one is evaluated.
  __device__ void run(int64_t e, int64_t pe) {
    int64_t body = e;
    if (L.vec) {
      int64_t a0 = (e + ITEMS - 1) & ~(int64_t)(ITEMS - 1);
      a0 = a0 < pe ? a0 : pe;
      if (a0 > e) masked(e, a0);
      body = a0;
      const int64_t nfull = (pe - a0) / kC;
      if (nfull > 0) {
        Cols cur = load_chunk(a0);
        for (int64_t it = 0; it < nfull; ++it) {
          const int64_t base = a0 + it * kC;
          if constexpr (TOPK) make_room(sel, kC, L.k, lane);
          // the prefetch is unconditional (a conditional load would make the
          // compiler wait for every load before evaluating cur); past the
          // last chunk it re-reads the current one, which is still cached
          const bool more = it + 1 < nfull;
          const Cols nxt = load_chunk(more ? base + kC : base);
          chunk(cur, base);
          cur = nxt;
        }
        body = a0 + nfull * kC;
      }
    }
    for (int64_t base = body; base < pe; base += 256) masked(base, (pe - base) < 256 ? pe : base + 256);
  }
};

// Per-workgroup tables: min(G_W, G_R) by (register granules, W_B), and
// 1 / (n_cu B) for the grid-round division.  Ends with a barrier.
__device__ void build_tables(const EvalLaunch &L, uint8_t *dyn_lds, float *tab_rcap, uint32_t *tab_mwb,
                             uint8_t *tab_blim, int tid, int nthreads) {
  const KArch &A = L.arch;
  const int row = A.nw + 1;
  uint8_t *tab_b = dyn_lds;
  uint8_t *tab_wtot = dyn_lds + L.tab_wtot_off;
  // waves the register file admits per register-granule count (Eq. 4 plain
  // reading), all slots when no registers are named
  const int slots = A.max_waves / A.simd;
  for (int rg = tid; rg <= A.nr; rg += nthreads) {
    int wtot = A.max_waves;
    if (rg > 0) {
      const int per_simd = A.vgprs / (rg * A.vgpr_gran);
      wtot = A.simd * (per_simd < slots ? per_simd : slots);
    }
    tab_wtot[rg] = (uint8_t)wtot;
  }
  // Eq. 3 block slots, and ceil(2^16 / W_B) for exact small divisions
  for (int wb = tid; wb <= A.nw; wb += nthreads) {
    tab_mwb[wb] = wb > 0 ? (65536u + (uint32_t)wb - 1u) / (uint32_t)wb : 0u;
    const int blim = (wb == 1 && A.exempt) ? 255 : (A.max_blocks < 255 ? A.max_blocks : 255);
    tab_blim[wb] = (uint8_t)blim;
  }
  for (int i = tid; i <= A.max_waves; i += nthreads) tab_rcap[i] = i > 0 ? 1.0f / (float)(A.n_cu * i) : 0.0f;
  __syncthreads();
  // min(G_W, G_R) = min(B_lim, floor(wtot / W_B)): the register bound never
  // exceeds floor(max_waves / W_B), the wave-slot part of Eq. 3
  const int n_tab = (A.nr + 1) * row;
  for (int i = tid; i < n_tab; i += nthreads) {
    const int rg = i / row, wb = i - rg * row;
    uint32_t b = 0;
    if (wb >= 1) {
      b = ((uint32_t)tab_wtot[rg] * tab_mwb[wb]) >> 16;
      b = b < tab_blim[wb] ? b : tab_blim[wb];
    }
    tab_b[i] = (uint8_t)b;
  }
  __syncthreads();
}

// The wave-uniform record of variant v (Eq. 5 bound, Eq. 6 per-variant sum,
// divergence weight) and its per-U / per-W_B tables in this wave's LDS.
template <Mode MODE>
__device__ __forceinline__ void setup_piece(const EvalLaunch &L, Piece &pc, WaveLds &wl, int64_t v, int64_t s0,
                                            int lane) {
  const KArch &A = L.arch;
  pc.valid = true;
  pc.gs = 0;
  pc.P = 0.f;
  pc.D = 1.f;
  pc.s0 = s0;
  pc.a4 = wl.a4;
  pc.a5 = wl.a5;
  if constexpr (MODE == Mode::Model) {
    const int32_t nfp = L.var.n_fp[v], nint = L.var.n_int[v], nld = L.var.n_ld[v], nst = L.var.n_st[v];
    const int32_t nbr = L.var.n_br[v], nbar = L.var.n_bar[v];
    const int32_t nreg = L.var.n_reg ? L.var.n_reg[v] : 0;
    const int32_t S = L.var.lds[v];
    const float d = L.var.div[v];
    const uint32_t cmax = 1u << 24;
    pc.valid = (uint32_t)nfp < cmax && (uint32_t)nint < cmax && (uint32_t)nld < cmax && (uint32_t)nst < cmax &&
               (uint32_t)nbr < cmax && (uint32_t)nreg < cmax && (uint32_t)nbar <= (1u << 14) && d >= 0.0f &&
               d <= 1.0f;
    // Eq. 5 with a floor; S = 0 does not limit
    if (S == 0) {
      pc.gs = kUnlimited;
    } else if (S < 0 || S > A.max_lds) {
      pc.gs = 0;
    } else {
      const int32_t alloc = ((S + A.lds_gran - 1) / A.lds_gran) * A.lds_gran;
      pc.gs = A.lds_cu / alloc;
    }
    // Eq. 6 per-variant part, fixed binary32 order
    const float s1f = A.cfp * (float)nfp;
    const float s2f = A.cint * (float)nint;
    const float s3f = A.cmem * (float)(nld + nst);
    const float s6f = A.creg * (float)nreg;
    float P = s1f + s2f;
    P = P + s3f;
    P = P + s6f;
    pc.P = P;
    const float A4 = A.cctrl * (float)nbr;
    pc.D = 1.0f + d;
    // branch term per U, barrier term per W_B
    wave_lds_sync();
    if (lane < A.max_unroll) wl.a4[lane] = A4 / (float)(lane + 1);
    if (lane < A.nw) wl.a5[lane + 1] = A.csync * (float)(nbar * (lane + 1));
    wave_lds_sync();
  }
}

template <Mode MODE, bool HAS_GRID, bool TOPK>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(SA_WAVES_PER_EU)))
void sa_eval_kernel(EvalLaunch L) {
  // Dynamic LDS: the occupancy table [rg][W_B] followed by waves-by-registers
  // per register-granule count.
  extern __shared__ __align__(16) uint8_t dyn_lds[];
  __shared__ float tab_rcap[kMaxWB + 1];
  __shared__ uint32_t tab_mwb[kMaxWB + 1];
  __shared__ uint8_t tab_blim[kMaxWB + 1];
  __shared__ WaveLds wl[kWavesPerBlock];

  const KArch &A = L.arch;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int w = tid / kWaveSize;
  (void)A;
  if constexpr (MODE == Mode::Model) build_tables(L, dyn_lds, tab_rcap, tab_mwb, tab_blim, tid, kBlockThreads);
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

  int64_t v = find_segment(seg, L.n_var, n_evals, t0, lane);
  int64_t e = t0;
  for (; v < L.n_var && e < t1; ++v) {
    const int64_t s0 = uniform64(clamp_off(seg[v], n_evals));
    const int64_t s1 = uniform64(clamp_off(seg[v + 1], n_evals));
    int64_t pe = s1 > e ? s1 : e;
    pe = pe < t1 ? pe : t1;
    if (pe <= e) continue;

    Piece pc;
    setup_piece<MODE>(L, pc, wl[w], v, s0, lane);

    if constexpr (TOPK) {
      sel.count = 0;
      sel.theta = kThetaInit;
    }
    Evaluator<MODE, HAS_GRID, TOPK, 4> ev{L, tb, pc, sel, lane};
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

// Persistent kernel over a plan's workgroup items (static stride over the
// grid).  kind 0 items: each wave evaluates whole segments and writes their
// rows.  kind 1 items: each wave selects over its part of one segment, the
// parts meet in LDS and wave 0 writes the row (or the item's fragment).
template <Mode MODE, bool HAS_GRID, bool TOPK, int ITEMS, int WPB>
__global__ __launch_bounds__(64 * WPB) void sa_plan_kernel(EvalLaunch L, PlanDev P) {
  extern __shared__ __align__(16) uint8_t dyn_lds[];
  __shared__ float tab_rcap[kMaxWB + 1];
  __shared__ uint32_t tab_mwb[kMaxWB + 1];
  __shared__ uint8_t tab_blim[kMaxWB + 1];
  __shared__ WaveLds wl[WPB];
  __shared__ uint64_t wgk[WPB][SA_K_MAX];

  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int w = tid / kWaveSize;
  if constexpr (MODE == Mode::Model) build_tables(L, dyn_lds, tab_rcap, tab_mwb, tab_blim, tid, 64 * WPB);
  const Tables tb{dyn_lds, tab_rcap};
  const int64_t n_evals = L.n_evals;
  const int64_t *seg = L.cfg.seg;
  const int k = L.k;
  Selector sel;
  sel.buf = wl[w].cand;
  sel.count = 0;
  sel.theta = kThetaInit;

  for (int64_t item = blockIdx.x; item < P.n_items; item += gridDim.x) {
    const PlanItem it = P.items[item];
    const PlanWave pw = P.waves[item * WPB + w];
    if (it.kind == 0) {
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
      int64_t e0 = pw.e0 > s0 ? pw.e0 : s0;
      int64_t e1 = pw.e1 < s1 ? pw.e1 : s1;
      uint64_t mine = kKeyNone;
      if (e1 > e0) {
        Piece pc;
        setup_piece<MODE>(L, pc, wl[w], v, s0, lane);
        sel.count = 0;
        sel.theta = kThetaInit;
        Evaluator<MODE, HAS_GRID, TOPK, ITEMS> ev{L, tb, pc, sel, lane};
        ev.run(e0, e1);
        if constexpr (TOPK) mine = select_k(sel, k, lane);
      }
      if constexpr (TOPK) {
        if (lane < k) wgk[w][lane] = mine;
      }
    }
    if constexpr (TOPK) {
      __syncthreads();
      if (it.kind == 1 && w == 0) {
        const int64_t v = it.v < L.n_var ? (it.v > 0 ? it.v : 0) : L.n_var - 1;
        const int64_t s0 = uniform64(clamp_off(seg[v], n_evals));
        sel.count = 0;
        sel.theta = kThetaInit;
        for (int base = 0; base < WPB * k; base += 64) {
          const int j = base + lane;
          const uint64_t key = j < WPB * k ? wgk[j / k][j % k] : kKeyNone;
          make_room(sel, 64, k, lane);
          const bool cand[1] = {key != kKeyNone && (uint32_t)(key >> 32) <= sel.theta};
          const uint64_t keys1[1] = {key};
          offer<1>(sel, cand, keys1);
        }
        const uint64_t m = select_k(sel, k, lane);
        if (it.slot < 0) {
          write_final(m, k, lane, v, L.topk_idx, L.topk_val, MODE == Mode::Keys ? L.keys : nullptr, s0);
        } else if (lane < k) {
          L.frag[(int64_t)it.slot * k + lane] = m;
        }
      }
      __syncthreads();
    }
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
  const size_t dyn = M == Mode::Model ? (size_t)L.dyn_lds_bytes : 0;
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
  const size_t dyn = M == Mode::Model ? (size_t)L.dyn_lds_bytes : 0;
  hipLaunchKernelGGL((sa_eval_kernel<M, G, K>), dim3((uint32_t)blocks), dim3(kBlockThreads), dyn, stream, L);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eval(const EvalLaunch &L, Mode mode, bool has_grid, bool topk, hipStream_t stream) {
  if (mode == Mode::Keys) {
    return topk ? launch_one<Mode::Keys, false, true>(L, stream) : hipErrorInvalidValue;
  }
  if (has_grid) {
    return topk ? launch_one<Mode::Model, true, true>(L, stream) : launch_one<Mode::Model, true, false>(L, stream);
  }
  return topk ? launch_one<Mode::Model, false, true>(L, stream) : launch_one<Mode::Model, false, false>(L, stream);
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

hipError_t launch_merge(const EvalLaunch &L, hipStream_t stream) {
  if (L.n_var == 0) return hipSuccess;
  int64_t blocks = (L.n_var + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(sa_merge_kernel, dim3((uint32_t)blocks), dim3(kBlockThreads), 0, stream, L);
  return hipGetLastError();
}

}  // namespace sa
