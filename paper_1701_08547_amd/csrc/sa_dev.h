// Device building blocks shared by the gfx950 kernels: lane helpers, the
// per-wave top-k selector, the occupancy / score evaluation of one
// configuration (Eqs. 1-6) and the per-workgroup occupancy tables.
// Everything has internal linkage: each kernel source gets its own copy.
#pragma once

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

// Floor division a / b for 0 <= a < 2^19, 1 <= b <= 2^17, given r = 1/b
// rounded to binary32 and then raised by three units in the last place.  The
// binary32 estimate a r is then above a/b by a factor in (1, 1 + 2^-21], i.e.
// by less than 1/4: its integer part is the quotient or one more, and one
// test makes it exact.
__device__ __forceinline__ int32_t udiv_up(int32_t a, int32_t b, float r) {
  const int32_t q = (int32_t)((float)a * r);
  return q - (int32_t)(__umul24((uint32_t)q, (uint32_t)b) > (uint32_t)a);
}

// a / b in binary32 for the grid factor's operands: integers from 0 to 2^31
// converted to binary32, b > 0 where the quotient is used.  These are the
// steps of the IEEE division the compiler emits for `a / b` (reciprocal
// estimate, one refinement, the quotient and two corrections from exact
// remainders) without its operand scaling and special-value fix-up, which
// operands in this range never trigger, so the quotient is the same, in
// eight instructions instead of eleven.
__device__ __forceinline__ float div_grid(float a, float b) {
  float y = __builtin_amdgcn_rcpf(b);
  const float e = fmaf(-b, y, 1.0f);
  y = fmaf(e, y, y);
  float q = a * y;
  float r = fmaf(-b, q, a);
  q = fmaf(r, y, q);
  r = fmaf(-b, q, a);
  return fmaf(r, y, q);
}

// ---------------------------------------------------------------- selection

struct Selector {
  uint64_t *buf;   // this wave's candidate buffer (CAP keys, LDS)
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
// CAP / 64 keys (Batcher's odd-even merge network for 8, its first stages for
// 4 and 2); each of the k rounds takes the minimum of the lane heads and the
// owner pops its head.
template <int CAP = kCandCap>
__device__ uint64_t select_k(Selector &s, int k, int lane) {
  constexpr int PER = CAP / 64;
  static_assert(PER == 2 || PER == 4 || PER == 8, "two, four or eight keys per lane");
  wave_lds_sync();
  const uint32_t i0 = (uint32_t)PER * (uint32_t)lane;
  uint64_t r[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) r[j] = i0 + j < s.count ? s.buf[i0 + j] : kKeyNone;
  if constexpr (PER == 2) {
    cas64(r[0], r[1]);
  } else if constexpr (PER == 4) {
    cas64(r[0], r[1]); cas64(r[2], r[3]);
    cas64(r[0], r[2]); cas64(r[1], r[3]);
    cas64(r[1], r[2]);
  } else {
    cas64(r[0], r[1]); cas64(r[2], r[3]); cas64(r[4], r[5]); cas64(r[6], r[7]);
    cas64(r[0], r[2]); cas64(r[1], r[3]); cas64(r[4], r[6]); cas64(r[5], r[7]);
    cas64(r[1], r[2]); cas64(r[5], r[6]);
    cas64(r[0], r[4]); cas64(r[1], r[5]); cas64(r[2], r[6]); cas64(r[3], r[7]);
    cas64(r[2], r[4]); cas64(r[3], r[5]);
    cas64(r[1], r[2]); cas64(r[3], r[4]); cas64(r[5], r[6]);
  }
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
      for (int j = 0; j < PER - 1; ++j) r[j] = r[j + 1];
      r[PER - 1] = kKeyNone;
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
template <int CAP = kCandCap>
__device__ __forceinline__ void make_room(Selector &s, uint32_t need, int k, int lane) {
  if (s.count + need > (uint32_t)CAP) select_k<CAP>(s, k, lane);
}

// Offer N rows of 64 keys (`cand[i]` marks the lanes offering key[i]) by
// ballot + mbcnt compaction; make_room(64 N) must have run first.
template <int N, int CAP = kCandCap>
__device__ __forceinline__ void offer(Selector &s, const bool (&cand)[N], const uint64_t (&key)[N]) {
  static_assert(N * 64 + SA_K_MAX <= CAP, "buffer must hold k keys plus one batch");
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

template <int CAP>
struct __align__(16) WaveLdsT {
  float a4[kMaxUnroll];  // (c_ctrl n_br) / U for U = 1 .. max_unroll
  float a5[kMaxWB + 2];  // c_sync (n_bar W_B)    for W_B = 1 .. nw (nw + 1: unused)
  uint64_t cand[CAP];
};
using WaveLds = WaveLdsT<kCandCap>;

// Wave-uniform state of the piece being evaluated.
struct Piece {
  uint64_t kept;   // reduced search space: bit j keeps block size ws (j + 1)
  bool valid;      // variant counts in range
  int32_t gs;      // Eq. 5 bound for the variant's LDS
  float P, D;      // Eq. 6 per-variant sum, divergence weight 1 + d
  int64_t s0;      // segment start (local index origin)
  const float *a4, *a5;
};

struct Tables {
  const uint8_t *tab_b;  // [rg][W_B] -> min(G_W, G_R)
  const float *rcap;     // [B] -> 1 / (n_cu B), raised 3 ulp (udiv_up)
};

// One configuration: W* (0 if illegal) and the binary32 score (+inf if
// illegal or not asked for).  Products of small non-negative integers use
// the full-rate 24-bit multiplier (every operand here is below 2^24).
template <bool HAS_GRID>
__device__ __forceinline__ void eval_cfg(const KArch &A, const Tables &tb, const Piece &pc, int32_t T, int32_t U,
                                         int32_t R, int32_t G, bool in, bool need_score, int32_t &W, float &sc) {
  // Block sizes and register counts outside their limits (negative ones
  // included, as unsigned) are clamped one past the limit, which lands in the
  // table's zero column (W_B = nw + 1) or zero row (granules = nr + 1): the
  // thread and register limits are multiples of the wave size and granule.
  const uint32_t Tc = min((uint32_t)T, (uint32_t)A.max_threads + 1u);
  const uint32_t Rc = min((uint32_t)R, (uint32_t)A.max_vgprs + 1u);
  // bitwise '&' keeps the remaining legality test free of branches
  bool ok = in & pc.valid & ((uint32_t)(U - 1) < (uint32_t)A.max_unroll);
  if (HAS_GRID) ok = ok & ((uint32_t)(G - 1) < (uint32_t)A.max_grid);
  U = ok ? U : 1;  // table index; G of an illegal lane is discarded
  // Eqs. 1-5: waves per block, register granules, bound table, LDS bound
  const int32_t WB = (int32_t)((Tc + (uint32_t)A.ws - 1u) >> A.ws_shift);
  const int32_t rg = (int32_t)((Rc + (1u << A.gran_shift) - 1u) >> A.gran_shift);
  int32_t B = tb.tab_b[__umul24(rg, A.nw + 2) + WB];
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
      const int32_t rounds = udiv_up(G + cap - 1, cap, tb.rcap[B]);
      num = __umul24(__umul24(rounds, cap), hide);
      den = __umul24(G, x);
    } else {
      num = hide;
      den = x;
    }
    const float F = div_grid((float)num, (float)den);
    sc = (B > 0) ? Ed * F : __builtin_huge_valf();
  }
}

// Every term of one configuration, for the learned correction's features:
// the same binary32 sequence as eval_cfg (need_score set), plus W_B, the
// bound B*, the separate wave-slot (G_W) and register (G_R) bounds, E' and
// F.  `wsimd`, `mwb` and `blim` are build_tables' per-granule waves per
// partition, ceil(2^16 / W_B) and block limits.  Illegal: B = W = 0, scores
// +inf.
struct Terms {
  int32_t WB, gw, gr, gs, B, W;
  float Ed, F, sc;
};

template <bool HAS_GRID>
__device__ __forceinline__ Terms eval_terms(const KArch &A, const Tables &tb, const uint8_t *wsimd, const uint32_t *mwb,
                                            const uint8_t *blim, const Piece &pc, int32_t T, int32_t U, int32_t R,
                                            int32_t G, bool in) {
  Terms t;
  bool ok = in & pc.valid & ((uint32_t)(T - 1) < (uint32_t)A.max_threads) &
            ((uint32_t)(U - 1) < (uint32_t)A.max_unroll) & ((uint32_t)R <= (uint32_t)A.max_vgprs);
  if (HAS_GRID) ok = ok & ((uint32_t)(G - 1) < (uint32_t)A.max_grid);
  T = ok ? T : 1;
  U = ok ? U : 1;
  R = ok ? R : 0;
  const int32_t WB = (T + A.ws - 1) >> A.ws_shift;
  const int32_t rg = (R + (1 << A.gran_shift) - 1) >> A.gran_shift;
  int32_t B = tb.tab_b[__umul24(rg, A.nw + 2) + WB];
  B = B < pc.gs ? B : pc.gs;
  B = ok ? B : 0;
  const int32_t W = __umul24(B, WB);
  const int32_t gwv = blocks_on_partitions_m(A.max_waves >> A.simd_shift, WB, A.simd_shift, mwb[WB]);
  t.WB = WB;
  t.gw = gwv < (int32_t)blim[WB] ? gwv : (int32_t)blim[WB];
  t.gr = rg == 0 ? kUnlimited : blocks_on_partitions_m(wsimd[rg], WB, A.simd_shift, mwb[WB]);
  t.gs = pc.gs;
  t.B = B;
  t.W = W;
  float E = pc.P + pc.a4[U - 1];
  E = E + pc.a5[WB];
  const float Ed = E * pc.D;
  const int32_t x = __umul24(W, U);
  const int32_t hide = x > A.w_sat ? x : A.w_sat;
  int32_t num, den;
  if (HAS_GRID) {
    const int32_t cap = __umul24(A.n_cu, B);
    const int32_t rounds = udiv_up(G + cap - 1, cap, tb.rcap[B]);
    num = __umul24(__umul24(rounds, cap), hide);
    den = __umul24(G, x);
  } else {
    num = hide;
    den = x;
  }
  const float F = div_grid((float)num, (float)den);
  t.Ed = B > 0 ? Ed : __builtin_huge_valf();
  t.F = B > 0 ? F : 0.0f;
  t.sc = B > 0 ? Ed * F : __builtin_huge_valf();
  return t;
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

// Per-workgroup tables: min(G_W, G_R) by (register granules, W_B), and
// 1 / (n_cu B) for the grid-round division.  Ends with a barrier.
__device__ void build_tables(const EvalLaunch &L, uint8_t *dyn_lds, float *tab_rcap, uint32_t *tab_mwb,
                             uint8_t *tab_blim, int tid, int nthreads) {
  const KArch &A = L.arch;
  const int row = A.nw + 2;
  uint8_t *tab_b = dyn_lds;
  uint8_t *tab_wsimd = dyn_lds + L.tab_wsimd_off;
  // waves one partition's register file admits per register-granule count
  // (Eq. 4 plain reading), capped by its wave slots; all slots when no
  // registers are named; granule count nr + 1 stands for every illegal
  // register count and admits none
  const int slots = A.max_waves / A.simd;
  for (int rg = tid; rg <= A.nr + 1; rg += nthreads) {
    int w = slots;
    if (rg > A.nr) {
      w = 0;
    } else if (rg > 0) {
      const int per_simd = A.vgprs / (rg * A.vgpr_gran);
      w = per_simd < slots ? per_simd : slots;
    }
    tab_wsimd[rg] = (uint8_t)w;
  }
  // Eq. 3 block slots, and ceil(2^16 / W_B) for exact small divisions; W_B =
  // nw + 1 stands for every illegal block size and admits no block
  for (int wb = tid; wb <= A.nw + 1; wb += nthreads) {
    tab_mwb[wb] = wb > 0 ? (65536u + (uint32_t)wb - 1u) / (uint32_t)wb : 0u;
    int blim = (wb == 1 && A.exempt) ? 255 : (A.max_blocks < 255 ? A.max_blocks : 255);
    tab_blim[wb] = (uint8_t)(wb > A.nw ? 0 : blim);
  }
  // 1 / (n_cu B) raised by three ulp for udiv_up
  for (int i = tid; i <= A.max_waves; i += nthreads)
    tab_rcap[i] = i > 0 ? __uint_as_float(__float_as_uint(1.0f / (float)(A.n_cu * i)) + 3u) : 0.0f;
  __syncthreads();
  // min(G_W, G_R) = min(B_lim, blocks on min(slots, register waves) places
  // per partition): the block count grows with the places, so the smaller
  // of the two place counts decides
  const int n_tab = (A.nr + 2) * row;
  for (int i = tid; i < n_tab; i += nthreads) {
    const int rg = i / row, wb = i - rg * row;
    uint32_t b = 0;
    if (wb >= 1) {
      b = (uint32_t)blocks_on_partitions_m(tab_wsimd[rg], wb, A.simd_shift, tab_mwb[wb]);
      b = b < tab_blim[wb] ? b : tab_blim[wb];
    }
    tab_b[i] = (uint8_t)b;
  }
  __syncthreads();
}

// The wave-uniform record of variant v (Eq. 5 bound, Eq. 6 per-variant sum,
// divergence weight) and its per-U / per-W_B tables in this wave's LDS.
template <Mode MODE, class WL>
__device__ __forceinline__ void setup_piece(const EvalLaunch &L, Piece &pc, WL &wl, int64_t v, int64_t s0,
                                            int lane) {
  const KArch &A = L.arch;
  pc.kept = 0;
  pc.valid = true;
  pc.gs = 0;
  pc.P = 0.f;
  pc.D = 1.f;
  pc.s0 = s0;
  pc.a4 = wl.a4;
  pc.a5 = wl.a5;
  if constexpr (MODE != Mode::Keys) {
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


// ---------------------------------------------------------------- reduced search space

// Sec. III-C / IV-C: T* = the block sizes (multiples of the wave size) whose
// occupancy is full when registers and LDS do not limit; bit j of the result
// stands for T = ws (j + 1).  Read from row 0 (no register limit) of the
// workgroup's occupancy table.
__device__ __forceinline__ uint64_t full_occupancy_mask(const KArch &A, const uint8_t *tab_b) {
  uint64_t m = 0;
  for (int wb = 1; wb <= A.nw; ++wb)
    if ((int32_t)tab_b[wb] * wb == A.max_waves) m |= 1ull << (wb - 1);
  return m;
}

// The paper's rule: keep the upper half of T* (by thread count) when the
// kernel's intensity n_fp / max(1, n_ld + n_st) exceeds 4, else the lower
// half; an odd-length T* drops its median.  The comparison is made on the
// integers (n_fp > 4 max(1, m)), which is exact.
__device__ __forceinline__ uint64_t kept_mask(uint64_t full, int nw, int32_t nfp, int32_t nld, int32_t nst) {
  const int32_t mem = nld + nst;
  const bool upper = nfp > 4 * (mem > 1 ? mem : 1);
  const int n = __popcll(full), h = n / 2;
  uint64_t kept = 0;
  int seen = 0;
  for (int j = 0; j < nw; ++j) {
    if ((full >> j) & 1ull) {
      if (upper ? seen >= n - h : seen < h) kept |= 1ull << j;
      ++seen;
    }
  }
  return kept;
}

// Whether block size T lies in the kept set.
__device__ __forceinline__ bool in_kept(uint64_t kept, const KArch &A, int32_t T) {
  const uint32_t j = ((uint32_t)T >> A.ws_shift) - 1u;
  return ((T & (A.ws - 1)) == 0) & (j < 64u) & (((kept >> (j & 63u)) & 1ull) != 0);
}

}  // namespace
}  // namespace sa
