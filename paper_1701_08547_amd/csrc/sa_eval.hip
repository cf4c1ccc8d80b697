// gfx950 kernels of the static autotuning model: fused occupancy (Eqs. 1-5),
// instruction-mix score (Eq. 6 with divergence and latency-hiding factors)
// and per-variant top-k selection, streamed over a CSR batch of
// (variant, configuration) evaluations.
//
// Work decomposition.  The flattened evaluation space [0, n_evals) is cut
// into wave-tiles of `tile` evaluations; each wave of a workgroup owns one
// wave-tile and walks the variant segments that overlap it ("pieces").  Per
// piece the variant's record is wave-uniform (scalar loads, computed once),
// and the wave streams its evaluations in rows of 64 lanes, kItems rows in
// flight, reading each structure-of-arrays column with coalesced dword loads.
//
// Selection.  Keys are (order-preserving score bits << 32 | local index), a
// total order.  Each wave keeps a threshold theta (the score of its current
// k-th best) and appends only the evaluations at or below it to a per-wave
// LDS candidate buffer (ballot + mbcnt compaction).  When the buffer fills,
// the wave extracts the k smallest keys by k rounds of a wave-wide minimum
// and tightens theta.  A piece that is a whole segment writes its result
// directly; pieces of segments that span wave-tiles write k-key fragments
// that sa_merge_kernel combines.
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

// Order-preserving map of binary32 to uint32 (negative values flipped).
__device__ __forceinline__ uint32_t order_key(float f) {
  uint32_t b = __float_as_uint(f);
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
__device__ __forceinline__ int32_t uniform32(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Orders this wave's LDS accesses before/after (LDS ops of one wave complete
// in order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int mask) {
  int lo = __shfl_xor((int)(uint32_t)v, mask, 64);
  int hi = __shfl_xor((int)(uint32_t)(v >> 32), mask, 64);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    uint64_t o = shfl_xor64(v, m);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ uint64_t min64(uint64_t a, uint64_t b) { return a < b ? a : b; }

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
  int32_t r = a - q * b;
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

// Reduce buf[0, count) to its k smallest keys: afterwards lane r < found holds
// the r-th smallest (kKeyNone elsewhere), buf[0, found) holds them too and
// theta is the k-th smallest score when k keys exist.
__device__ uint64_t select_k(Selector &s, int k, int lane) {
  wave_lds_sync();
  constexpr int J = kCandCap / 64;
  uint64_t r[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    uint32_t i = (uint32_t)lane + 64u * j;
    r[j] = i < s.count ? s.buf[i] : kKeyNone;
  }
  uint64_t mine = kKeyNone;
  int found = 0;
  for (int q = 0; q < k; ++q) {
    uint64_t m = r[0];
#pragma unroll
    for (int j = 1; j < J; ++j) m = min64(m, r[j]);
    m = wave_min64(m);
    if (m == kKeyNone) break;
    if (lane == q) mine = m;
#pragma unroll
    for (int j = 0; j < J; ++j) r[j] = (r[j] == m) ? kKeyNone : r[j];
    ++found;
  }
  wave_lds_sync();
  if (lane < found) s.buf[lane] = mine;
  s.count = (uint32_t)found;
  if (found == k) {
    uint32_t hi = (uint32_t)(mine >> 32);
    s.theta = (uint32_t)__builtin_amdgcn_readlane((int)hi, k - 1);
  }
  wave_lds_sync();
  return mine;
}

// Offer one row of 64 keys (one per lane, `cand` marks the lanes to offer).
__device__ __forceinline__ void offer(Selector &s, bool cand, uint64_t key, int k, int lane) {
  uint64_t bal = __ballot(cand);
  if (bal == 0) return;
  uint32_t c = (uint32_t)__popcll(bal);
  if (s.count + c > (uint32_t)kCandCap) select_k(s, k, lane);
  uint32_t pos = s.count + mbcnt64(bal);
  if (cand) s.buf[pos] = key;
  s.count += c;
}

__device__ __forceinline__ void write_final(uint64_t mine, int k, int lane, int64_t v, int32_t *idx, float *val) {
  if (lane < k) {
    bool none = (mine == kKeyNone);
    if (idx) idx[v * k + lane] = none ? -1 : (int32_t)(uint32_t)mine;
    if (val) val[v * k + lane] = none ? __builtin_huge_valf() : order_key_inv((uint32_t)(mine >> 32));
  }
}

// ---------------------------------------------------------------- main kernel

struct __align__(16) WaveLds {
  float a4[kMaxUnroll];        // (c_ctrl n_br) / U for U = 1 .. max_unroll
  float a5[kMaxWB + 1];        // c_sync (n_bar W_B)    for W_B = 1 .. nw
  uint64_t cand[kCandCap];
};

template <Mode MODE, bool HAS_GRID, bool TOPK>
__global__ __launch_bounds__(kBlockThreads) void sa_eval_kernel(EvalLaunch L) {
  // Per-workgroup tables: occupancy bound by (register granules, W_B) and
  // 1/(n_cu B*) for the grid-round division.
  extern __shared__ __align__(16) uint8_t tab_b[];  // (nr + 1) x (nw + 1) bytes, dynamic
  __shared__ float tab_rcap[kMaxWB + 1];
  __shared__ WaveLds wl[kWavesPerBlock];

  const KArch &A = L.arch;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int w = tid / kWaveSize;

  if constexpr (MODE == Mode::Model) {
    const int row = A.nw + 1;
    const int n_tab = (A.nr + 1) * row;
    for (int i = tid; i < n_tab; i += kBlockThreads) {
      int rg = i / row, wb = i - rg * row;
      int b = 0;
      if (wb >= 1) {
        // waves the register file admits (Eq. 4 plain reading), all when R = 0
        int wtot = A.max_waves;
        if (rg > 0) {
          int per_simd = A.vgprs / (rg * A.vgpr_gran);
          int slots = A.max_waves / A.simd;
          wtot = A.simd * (per_simd < slots ? per_simd : slots);
        }
        // Eq. 3 wave slots and block slots (min over both); registers bound
        // floor(wtot / W_B) never exceeds floor(max_waves / W_B).
        int by_regs = wtot / wb;
        int by_slots = (wb == 1 && A.exempt) ? kUnlimited : A.max_blocks;
        b = by_regs < by_slots ? by_regs : by_slots;
      }
      tab_b[i] = (uint8_t)b;
    }
    for (int i = tid; i <= A.max_waves; i += kBlockThreads)
      tab_rcap[i] = i > 0 ? 1.0f / (float)(A.n_cu * i) : 0.0f;
  }
  __syncthreads();  // the only workgroup barrier: waves are independent below

  const int64_t wt = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wt >= L.n_tiles) return;
  const int64_t t0 = wt * L.tile;
  const int64_t t1 = (t0 + L.tile < L.n_evals) ? t0 + L.tile : L.n_evals;
  const int64_t *seg = L.cfg.seg;
  const int64_t n_evals = L.n_evals;
  const int k = L.k;

  Selector sel;
  sel.buf = wl[w].cand;

  int64_t v = find_segment(seg, L.n_var, n_evals, t0, lane);
  int64_t e = t0;
  for (; v < L.n_var && e < t1; ++v) {
    const int64_t s0 = clamp_off(seg[v], n_evals);
    const int64_t s1 = clamp_off(seg[v + 1], n_evals);
    int64_t pe = s1 > e ? s1 : e;
    pe = pe < t1 ? pe : t1;
    if (pe <= e) continue;

    // ---- per-variant record (wave-uniform)
    bool valid = true;
    int32_t gs = 0;
    float P = 0.f, D = 1.f;
    if constexpr (MODE == Mode::Model) {
      const int32_t nfp = L.var.n_fp[v], nint = L.var.n_int[v], nld = L.var.n_ld[v], nst = L.var.n_st[v];
      const int32_t nbr = L.var.n_br[v], nbar = L.var.n_bar[v];
      const int32_t nreg = L.var.n_reg ? L.var.n_reg[v] : 0;
      const int32_t S = L.var.lds[v];
      const float d = L.var.div[v];
      const uint32_t cmax = 1u << 24;
      valid = (uint32_t)nfp < cmax && (uint32_t)nint < cmax && (uint32_t)nld < cmax && (uint32_t)nst < cmax &&
              (uint32_t)nbr < cmax && (uint32_t)nreg < cmax && (uint32_t)nbar <= (1u << 14) && d >= 0.0f &&
              d <= 1.0f;
      // Eq. 5 with a floor; S = 0 does not limit
      if (S == 0) {
        gs = kUnlimited;
      } else if (S < 0 || S > A.max_lds) {
        gs = 0;
      } else {
        int32_t alloc = ((S + A.lds_gran - 1) / A.lds_gran) * A.lds_gran;
        gs = A.lds_cu / alloc;
      }
      // Eq. 6 per-variant part, fixed binary32 order
      float s1f = A.cfp * (float)nfp;
      float s2f = A.cint * (float)nint;
      float s3f = A.cmem * (float)(nld + nst);
      float s6f = A.creg * (float)nreg;
      P = s1f + s2f;
      P = P + s3f;
      P = P + s6f;
      const float A4 = A.cctrl * (float)nbr;
      D = 1.0f + d;
      // per-wave tables for this variant
      wave_lds_sync();
      if (lane < A.max_unroll) wl[w].a4[lane] = A4 / (float)(lane + 1);
      if (lane < A.nw) wl[w].a5[lane + 1] = A.csync * (float)(nbar * (lane + 1));
      wave_lds_sync();
    }

    if constexpr (TOPK) {
      sel.count = 0;
      sel.theta = kThetaInit;
    }

    for (int64_t base = e; base < pe; base += 64 * kItems) {
      const int64_t rem64 = pe - base;
      const int rem = rem64 < 64 * kItems ? (int)rem64 : 64 * kItems;
      int32_t Tv[kItems], Uv[kItems], Rv[kItems], Gv[kItems];
      float Kv[kItems];
      if constexpr (MODE == Mode::Model) {
        const int32_t *pT = L.cfg.block + base;
        const int32_t *pU = L.cfg.unroll + base;
        const int32_t *pR = L.cfg.regs + base;
        const int32_t *pG = HAS_GRID ? L.cfg.grid + base : nullptr;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
          const int j = lane + 64 * i;
          const bool in = j < rem;
          Tv[i] = in ? pT[j] : 0;
          Uv[i] = in ? pU[j] : 0;
          Rv[i] = in ? pR[j] : 0;
          Gv[i] = (HAS_GRID && in) ? pG[j] : 1;
        }
      } else {
        const float *pK = L.keys + base;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
          const int j = lane + 64 * i;
          Kv[i] = j < rem ? pK[j] : __builtin_huge_valf();
        }
      }
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        const int j = lane + 64 * i;
        const bool in = j < rem;
        const int64_t eidx = base + j;
        float sc = __builtin_huge_valf();
        bool ok;
        if constexpr (MODE == Mode::Model) {
          int32_t T = Tv[i], U = Uv[i], R = Rv[i], G = Gv[i];
          ok = in && valid && (uint32_t)(T - 1) < (uint32_t)A.max_threads &&
               (uint32_t)(U - 1) < (uint32_t)A.max_unroll && (uint32_t)R <= (uint32_t)A.max_vgprs;
          if (HAS_GRID) ok = ok && (uint32_t)(G - 1) < (uint32_t)A.max_grid;
          T = ok ? T : 1;
          U = ok ? U : 1;
          R = ok ? R : 0;
          G = ok ? G : 1;
          // Eqs. 1-5: W_B, register granules, bound table, LDS bound
          const int32_t WB = (int32_t)__umulhi((uint32_t)(T + A.ws - 1), A.m_ws);
          const int32_t rg = A.m_gran ? (int32_t)__umulhi((uint32_t)(R + A.vgpr_gran - 1), A.m_gran) : R;
          int32_t B = tab_b[rg * (A.nw + 1) + WB];
          B = B < gs ? B : gs;
          B = ok ? B : 0;
          const int32_t W = B * WB;
          if (L.occ && in) L.occ[eidx] = W;
          if (L.need_score) {
            const int32_t Bs = B > 0 ? B : 1;
            const float a4 = wl[w].a4[U - 1];
            const float a5 = wl[w].a5[WB];
            float E = P + a4;
            E = E + a5;
            const float Ed = E * D;
            const int32_t x = Bs * WB * U;
            const int32_t hide = x > A.w_sat ? x : A.w_sat;
            int32_t num, den;
            if (HAS_GRID) {
              const int32_t cap = A.n_cu * Bs;
              const int32_t rounds = udiv_rcp(G + cap - 1, cap, tab_rcap[Bs]);
              num = rounds * cap * hide;
              den = G * x;
            } else {
              num = hide;
              den = x;
            }
            const float F = (float)num / (float)den;
            sc = (B > 0) ? Ed * F : __builtin_huge_valf();
            if (L.score && in) L.score[eidx] = sc;
          }
          ok = B > 0;
        } else {
          sc = Kv[i];
          ok = in && sc < __builtin_huge_valf();
        }
        if constexpr (TOPK) {
          const uint32_t kk = order_key(sc);
          const bool cand = ok && kk <= sel.theta;
          const uint64_t key = ((uint64_t)kk << 32) | (uint32_t)(eidx - s0);
          offer(sel, cand, key, k, lane);
        }
      }
    }

    if constexpr (TOPK) {
      const uint64_t mine = select_k(sel, k, lane);
      if (e == s0 && pe == s1) {
        write_final(mine, k, lane, v, L.topk_idx, L.topk_val);
      } else {
        const int64_t slot = 2 * wt + (e == t0 ? 0 : 1);
        if (lane < k) L.frag[slot * k + lane] = mine;
      }
    }
    e = pe;
  }
}

// Combine the fragments of segments that span several wave-tiles, and write
// the padding row of empty segments.  One wave per variant.
__global__ __launch_bounds__(kBlockThreads) void sa_merge_kernel(EvalLaunch L) {
  __shared__ uint64_t cand[kWavesPerBlock][kCandCap];
  const int lane = lane_id();
  const int w = threadIdx.x / kWaveSize;
  const int64_t n_evals = L.n_evals;
  const int k = L.k;
  const int64_t T = L.tile;
  Selector sel;
  sel.buf = cand[w];
  for (int64_t v = (int64_t)blockIdx.x * kWavesPerBlock + w; v < L.n_var;
       v += (int64_t)gridDim.x * kWavesPerBlock) {
    const int64_t s0 = clamp_off(L.cfg.seg[v], n_evals);
    const int64_t s1 = clamp_off(L.cfg.seg[v + 1], n_evals);
    if (s1 <= s0) {
      write_final(kKeyNone, k, lane, v, L.topk_idx, L.topk_val);
      continue;
    }
    const int64_t ta = s0 / T, tb = (s1 - 1) / T;
    if (ta == tb) continue;  // whole segment inside one wave-tile: already final
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
      const bool cand_ok = key != kKeyNone && (uint32_t)(key >> 32) <= sel.theta;
      offer(sel, cand_ok, key, k, lane);
    }
    const uint64_t mine = select_k(sel, k, lane);
    write_final(mine, k, lane, v, L.topk_idx, L.topk_val);
  }
}

template <Mode M, bool G, bool K>
hipError_t launch_one(const EvalLaunch &L, hipStream_t stream) {
  const int64_t blocks = (L.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks == 0) return hipSuccess;
  size_t dyn = 0;
  if (M == Mode::Model) dyn = (((size_t)(L.arch.nr + 1) * (size_t)(L.arch.nw + 1)) + 15) & ~(size_t)15;
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

hipError_t launch_merge(const EvalLaunch &L, hipStream_t stream) {
  if (L.n_var == 0) return hipSuccess;
  int64_t blocks = (L.n_var + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(sa_merge_kernel, dim3((uint32_t)blocks), dim3(kBlockThreads), 0, stream, L);
  return hipGetLastError();
}

}  // namespace sa
