// Learned correction of the static model on gfx950: the 24-feature builder,
// the BF16 MFMA forward pass for rows of features (24 -> 128 -> 128 -> 1,
// GELU, fp32 accumulation) and the training step.
//
// A training step is one fused kernel and one update kernel.  Each workgroup
// of the fused kernel takes passes of 64 rows, one 16-row tile per wave: the
// forward pass exactly as inference computes it (same staged weights, GELU
// pieces and MFMA order, so the training forward's Delta equals the served
// one bit for bit), the loss gradient, the backward pass in registers (dL/da2,
// dL/dh1 = W2^T dL/da2 on the matrix cores, dL/da1), and the weight-gradient
// contractions over the pass's rows from LDS; the workgroup writes its
// gradient sums once.  The update kernel adds the workgroups' partial sums in
// a fixed order (deterministic) and applies Adam.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "sa_internal.h"
#include "sa_mlp_dev.h"
#include "sa_train.h"

namespace sa {
namespace {

constexpr int kF = 24;  // features

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Sum over the 16 lanes of a lane group (lanes with equal l / 16), left in
// every lane of the group: four additions of the value rotated within the
// row by 8, 4, 2 and 1 lanes (DPP row_ror, no LDS traffic).  After the
// rotation by 2^s every lane holds the sum over the lanes congruent to it
// modulo 2^s, the same pairs of partial sums a butterfly over lane l xor 2^s
// adds, so the result is the butterfly's bit for bit.
template <int CTRL>
__device__ __forceinline__ float row_ror_add(float v) {
  return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float sum16(float v) {
  v = row_ror_add<0x128>(v);  // row_ror:8
  v = row_ror_add<0x124>(v);  // row_ror:4
  v = row_ror_add<0x122>(v);  // row_ror:2
  return row_ror_add<0x121>(v);  // row_ror:1
}

// ---------------------------------------------------------------- features

// The 24 features of one legal evaluation (binary32; see the oracle's
// definition).  gw, gr, gs may be kUnlimitedFeat when not limiting.
__device__ __forceinline__ void make_features(float *f, int32_t nfp, int32_t nint, int32_t nld, int32_t nst,
                                              int32_t nbr, int32_t nbar, int32_t nreg, int32_t S, float d, int32_t T,
                                              int32_t U, int32_t R, int32_t G, bool has_grid, int32_t n_cu, int32_t WB,
                                              int32_t gw, int32_t gr, int32_t gs, int32_t B, int32_t W, float Ed,
                                              float F, float sc) {
  variant_features(f, nfp, nint, nld, nst, nbr, nbar, nreg, S, d);
  config_features(f, T, U, R, G, has_grid, n_cu, WB, gw, gr, gs, B, W, Ed, F, sc);
}

// Standalone feature builder over a CSR batch (training data, tests): one
// thread per evaluation; the occupancy and score terms follow the same
// binary32 sequence as the scoring kernel.  Illegal evaluations get +inf in
// feature 22 (ln score).
__global__ void sa_features_kernel(EvalLaunch L, float *feat) {
  const KArch &A = L.arch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < L.n_evals;
       e += (int64_t)gridDim.x * blockDim.x) {
    // variant of e: binary search in seg
    int64_t lo = 0, hi = L.n_var;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) / 2;
      if (L.cfg.seg[mid] <= e) lo = mid; else hi = mid;
    }
    const int64_t v = lo;
    const int32_t nfp = L.var.n_fp[v], nint = L.var.n_int[v], nld = L.var.n_ld[v], nst = L.var.n_st[v];
    const int32_t nbr = L.var.n_br[v], nbar = L.var.n_bar[v], nreg = L.var.n_reg ? L.var.n_reg[v] : 0;
    const int32_t S = L.var.lds[v];
    const float d = L.var.div[v];
    const int32_t T = L.cfg.block[e], U = L.cfg.unroll[e], R = L.cfg.regs[e];
    const bool has_grid = L.cfg.grid != nullptr;
    const int32_t G = has_grid ? L.cfg.grid[e] : 1;
    const uint32_t cmax = 1u << 24;
    bool ok = (uint32_t)nfp < cmax && (uint32_t)nint < cmax && (uint32_t)nld < cmax && (uint32_t)nst < cmax &&
              (uint32_t)nbr < cmax && (uint32_t)nreg < cmax && (uint32_t)nbar <= (1u << 14) && d >= 0.0f &&
              d <= 1.0f && (uint32_t)(T - 1) < (uint32_t)A.max_threads && (uint32_t)(U - 1) < (uint32_t)A.max_unroll &&
              (uint32_t)R <= (uint32_t)A.max_vgprs && (!has_grid || (uint32_t)(G - 1) < (uint32_t)A.max_grid) &&
              S >= 0 && S <= A.max_lds;
    float *f = feat + e * kF;
    const int32_t Tc = ok ? T : 1, Rc = ok ? R : 0, Uc = ok ? U : 1;
    const int32_t WB = (Tc + A.ws - 1) / A.ws;
    const int32_t slots = A.max_waves / A.simd;
    const int32_t gw_waves = blocks_on_partitions(slots, WB, A.simd);
    const int32_t blim = (WB == 1 && A.exempt) ? (1 << 30) : A.max_blocks;
    const int32_t gw = gw_waves < blim ? gw_waves : blim;
    int32_t gr = 1 << 30;
    if (Rc > 0) {
      const int32_t per = ((Rc + A.vgpr_gran - 1) / A.vgpr_gran) * A.vgpr_gran;
      const int32_t wv = A.vgprs / per < slots ? A.vgprs / per : slots;
      gr = blocks_on_partitions(wv, WB, A.simd);
    }
    int32_t gs = 1 << 30;
    if (S > 0) gs = A.lds_cu / (((S + A.lds_gran - 1) / A.lds_gran) * A.lds_gran);
    int32_t B = gw < gr ? gw : gr;
    B = B < gs ? B : gs;
    if (!ok) B = 0;
    const int32_t W = B * WB;
    float Ed = __builtin_huge_valf(), F = 0.0f, sc = __builtin_huge_valf();
    if (B > 0) {
      const float s1f = A.cfp * (float)nfp, s2f = A.cint * (float)nint, s3f = A.cmem * (float)(nld + nst);
      const float s6f = A.creg * (float)nreg;
      float P = s1f + s2f;
      P = P + s3f;
      P = P + s6f;
      const float A4 = A.cctrl * (float)nbr;
      const float a4 = A4 / (float)Uc;
      const float a5 = A.csync * (float)(nbar * WB);
      float E = P + a4;
      E = E + a5;
      Ed = E * (1.0f + d);
      const int32_t x = W * Uc;
      const int32_t hide = x > A.w_sat ? x : A.w_sat;
      int32_t num = hide, den = x;
      if (has_grid) {
        const int32_t cap = A.n_cu * B;
        const int32_t rounds = (G + cap - 1) / cap;
        num = rounds * cap * hide;
        den = G * x;
      }
      F = (float)num / (float)den;
      sc = Ed * F;
    }
    make_features(f, nfp, nint, nld, nst, nbr, nbar, nreg, S, d, Tc, Uc, Rc, G, has_grid, A.n_cu, WB, gw, gr, gs, B, W,
                  Ed, F, sc);
  }
}

// ---------------------------------------------------------------- inference

// Delta for n rows of raw features (n x 24 fp32): each wave takes blocks of
// 64 rows, one row per lane.
constexpr int kFwdWaves = 8;

__global__ __launch_bounds__(64 * kFwdWaves) void sa_mlp_fwd_kernel(MlpDev M, const float *feat, int64_t n,
                                                                    float *delta) {
  __shared__ MlpLdsT s;
  __shared__ __align__(16) uint16_t X[kFwdWaves][64 * kLdXin];
  const int tid = threadIdx.x, lane = lane_id(), w = tid / 64;
  load_weights_t(M, s, tid, 64 * kFwdWaves);
  __syncthreads();
  const int64_t n_blocks = (n + 63) / 64;
  for (int64_t blk = (int64_t)blockIdx.x * kFwdWaves + w; blk < n_blocks; blk += (int64_t)gridDim.x * kFwdWaves) {
    const int64_t row = blk * 64 + lane;
    const bool in = row < n;
    float f[kF];
#pragma unroll
    for (int i = 0; i < kF; ++i) f[i] = in ? feat[row * kF + i] : 0.0f;
    put_x(s, X[w], lane, f, !in);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const float d = mlp_rows<false, 2>(s, X[w], lane, u32x4_t{0u, 0u, 0u, 0u});
    if (in) delta[row] = d;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
}

// ---------------------------------------------------------------- training

constexpr int kTrainWaves = 4;                // one 16-row tile per wave
constexpr int kTrainRows = 16 * kTrainWaves;  // rows per pass of a workgroup
constexpr int kTrainThreads = 64 * kTrainWaves;
constexpr int kMaxPartials = 256;             // workgroups (gradient partials) of one step
constexpr int kLdR = kTrainRows + 8;          // row stride of the per-pass blocks (bf16), padded

struct __align__(16) TrainLds {
  MlpLdsT f;                        // forward: the inference staging (scaled weights, GELU pieces)
  uint16_t W2b[kMH * kLdW2];        // backward: W2b[k][p] = W2[w2_column(p)][k]
  float w3[kMH];                    // w3 as the forward uses it (its bf16 value)
  uint16_t gA2t[kMH * kLdR];        // dL/da2 [hidden][row of the pass], bf16
  uint16_t gA1t[kMH * kLdR];        // dL/da1
  uint16_t H1t[kMH * kLdR];         // h1
  uint16_t Xt[kMK * kLdR];          // normalised inputs, columns 24..31 zero
  float sums[kTrainWaves][3][kMH];  // per-wave column sums: b1, b2, w3 gradients
  float tail[kTrainWaves][2];       // per-wave b3 gradient and loss
};

// a of a scaled pre-activation u = a / 16 + 1/2.
__device__ __forceinline__ float unscale(float t) { return (t - kTOrigin) * (1.0f / kTScale); }

// LOSS 0: squared error against target (dL/dDelta = 2 (Delta - r) / n).
// LOSS 1: dL/dDelta and the loss terms given per row (pairwise ranking loss,
// computed beforehand from this step's Delta).
template <int LOSS>
__global__ __launch_bounds__(kTrainThreads) void sa_train_kernel(MlpDev M, const float *feat, const float *target,
                                                                 int64_t n, TrainBufs T, int64_t *step_counter) {
  __shared__ TrainLds s;
  const int tid = threadIdx.x, lane = lane_id(), w = tid / 64;
  const int r = lane & 15, q = lane >> 4;
  // the backward's W2 staged beside the forward's: W2b[k][p] = W2[w2_column(p)][k]
  load_weights_t(M, s.f, tid, kTrainThreads, s.W2b);
  for (int i = tid; i < kMH; i += kTrainThreads) s.w3[i] = bf2f(M.w3[i]);
  if (step_counter && blockIdx.x == 0 && tid == 0) *step_counter += 1;  // read by the update kernel
  __syncthreads();
  const float inv_n2 = 2.0f / (float)n;
  // per-lane running sums over this workgroup's rows (reduced at the end)
  float g_b1[8][4], g_b2[8][4], g_w3[8][4];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) g_b1[t][j] = g_b2[t][j] = g_w3[t][j] = 0.0f;
  float g_b3 = 0.0f, loss = 0.0f;
  f32x4_t accW2[16], accW1[4];
#pragma unroll
  for (int i = 0; i < 16; ++i) accW2[i] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int i = 0; i < 4; ++i) accW1[i] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  const int col = 16 * w + r;  // this lane's row within the pass

  for (int64_t base = (int64_t)blockIdx.x * kTrainRows; base < n; base += (int64_t)gridDim.x * kTrainRows) {
    const int64_t row = base + col;
    const bool in = row < n;
    // inputs: slice q (features 8 q .. 8 q + 7) of this lane's row, as inference packs them
    u32x4_t xb = {0u, 0u, 0u, 0u};
    if (q < 3 && in) {
      const float *fr = feat + row * kF + 8 * q;
      const float *mu = s.f.mean + 8 * q, *is = s.f.inv_std + 8 * q;
      uint32_t p[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        p[i] = pack_bf16((fr[2 * i] - mu[2 * i]) * is[2 * i], (fr[2 * i + 1] - mu[2 * i + 1]) * is[2 * i + 1]);
      xb = u32x4_t{p[0], p[1], p[2], p[3]};
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s.Xt[(8 * q + 2 * i) * kLdR + col] = (uint16_t)(xb[i] & 0xFFFFu);
      s.Xt[(8 * q + 2 * i + 1) * kLdR + col] = (uint16_t)(xb[i] >> 16);
    }
    // the contraction's operand carries the folded first-layer bias in
    // inputs 24..26, as inference's does (the weight gradient above sees the
    // network's zeros there)
    if (q == 3) xb = u32x4_t{kOnes24, kOnes26, 0u, 0u};
    // layer 1 (scaled pre-activations kept for the backward pass)
    // (each layer's contractions all issued before its GELU: the pre-activations
    // are kept for the backward pass anyway)
    f32x4_t t1[8];
    uint32_t h1[8][2];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const u32x4_t a = *(const u32x4_t *)(s.f.W1 + (16 * t + r) * kLdW1 + 8 * q);
      t1[t] = mfma32(a, xb, f32x4_t{0.0f, 0.0f, 0.0f, 0.0f});
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      float v[4] = {t1[t][0], t1[t][1], t1[t][2], t1[t][3]};
      gelu_t_n<4>(v, s.f.gelu);
      h1[t][0] = pack_bf16(v[0], v[1]);
      h1[t][1] = pack_bf16(v[2], v[3]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        s.H1t[(16 * t + 4 * q + j) * kLdR + col] = (uint16_t)(h1[t][j >> 1] >> (16 * (j & 1)));
    }
    // layer 2
    f32x4_t t2[8];
    uint32_t h2[8][2];
#pragma unroll
    for (int ot = 0; ot < 8; ++ot) {
      f32x4_t acc = *(const f32x4_t *)(s.f.b2 + 16 * ot + 4 * q);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const u32x4_t a = *(const u32x4_t *)(s.f.W2 + (16 * ot + r) * kLdW2 + 32 * c + 8 * q);
        acc = mfma32(a, u32x4_t{h1[2 * c][0], h1[2 * c][1], h1[2 * c + 1][0], h1[2 * c + 1][1]}, acc);
      }
      t2[ot] = acc;
    }
#pragma unroll
    for (int ot = 0; ot < 8; ++ot) {
      float v[4] = {t2[ot][0], t2[ot][1], t2[ot][2], t2[ot][3]};
      gelu_t_n<4>(v, s.f.gelu);
      h2[ot][0] = pack_bf16(v[0], v[1]);
      h2[ot][1] = pack_bf16(v[2], v[3]);
    }
    // layer 3: every A row is w3, so each lane of column r receives Delta of row r
    f32x4_t acc3 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c3 = 0; c3 < 4; ++c3) {
      const u32x4_t a3 = *(const u32x4_t *)(s.f.w3p + 32 * c3 + 8 * q);
      acc3 = mfma32(a3, u32x4_t{h2[2 * c3][0], h2[2 * c3][1], h2[2 * c3 + 1][0], h2[2 * c3 + 1][1]}, acc3);
    }
    const float delta = acc3[0] + s.f.b3;
    // the loss gradient of this lane's row
    float gd = 0.0f;
    if (in) {
      if constexpr (LOSS == 0) {
        const float e = delta - target[row];
        gd = inv_n2 * e;
        if (q == 0) loss += e * e;
      } else {
        gd = T.gdelta[row];
        if (q == 0) loss += T.loss[row];
      }
    }
    if (q == 0) g_b3 += gd;
    // dL/da2 = dL/dDelta w3 GELU'(a2), packed as the next contraction's B operand
    uint32_t g2[8][2];
#pragma unroll
    for (int ot = 0; ot < 8; ++ot) {
      float g[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int hid = 16 * ot + 4 * q + j;
        const float hv = bf2f((uint16_t)(h2[ot][j >> 1] >> (16 * (j & 1))));
        g[j] = gd * s.w3[hid] * gelu_grad(unscale(t2[ot][j]));
        g_b2[ot][j] += g[j];
        g_w3[ot][j] += gd * hv;
      }
      g2[ot][0] = pack_bf16(g[0], g[1]);
      g2[ot][1] = pack_bf16(g[2], g[3]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        s.gA2t[(16 * ot + 4 * q + j) * kLdR + col] = (uint16_t)(g2[ot][j >> 1] >> (16 * (j & 1)));
    }
    // dL/dh1 = W2^T dL/da2 (matrix cores), then dL/da1 = dL/dh1 GELU'(a1)
#pragma unroll
    for (int kt = 0; kt < 8; ++kt) {
      f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const u32x4_t a = *(const u32x4_t *)(s.W2b + (16 * kt + r) * kLdW2 + 32 * c + 8 * q);
        acc = mfma32(a, u32x4_t{g2[2 * c][0], g2[2 * c][1], g2[2 * c + 1][0], g2[2 * c + 1][1]}, acc);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float g = acc[j] * gelu_grad(unscale(t1[kt][j]));
        g_b1[kt][j] += g;
        s.gA1t[(16 * kt + 4 * q + j) * kLdR + col] = f2bf(g);
      }
    }
    __syncthreads();
    // weight gradients over the pass's 64 rows: dW2 = dA2^T H1 (64 tiles, 16 per
    // wave), dW1 = dA1^T X (16 tiles, 4 per wave)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int tile = 16 * w + i, mt = tile >> 3, nt = tile & 7;
#pragma unroll
      for (int kk = 0; kk < kTrainRows; kk += 32) {
        const u32x4_t a = *(const u32x4_t *)(s.gA2t + (16 * mt + r) * kLdR + kk + 8 * q);
        const u32x4_t b = *(const u32x4_t *)(s.H1t + (16 * nt + r) * kLdR + kk + 8 * q);
        accW2[i] = mfma32(a, b, accW2[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int tile = 4 * w + i, mt = tile >> 1, nt = tile & 1;
#pragma unroll
      for (int kk = 0; kk < kTrainRows; kk += 32) {
        const u32x4_t a = *(const u32x4_t *)(s.gA1t + (16 * mt + r) * kLdR + kk + 8 * q);
        const u32x4_t b = *(const u32x4_t *)(s.Xt + (16 * nt + r) * kLdR + kk + 8 * q);
        accW1[i] = mfma32(a, b, accW1[i]);
      }
    }
    __syncthreads();
  }

  // this workgroup's sums: the weight tiles as they stand, the column sums
  // reduced over each wave's 16 rows and then over the waves
  float *part = T.part + (int64_t)blockIdx.x * kPartStride;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int tile = 16 * w + i, mt = tile >> 3, nt = tile & 7;
#pragma unroll
    for (int j = 0; j < 4; ++j) part[kPartW2 + (16 * mt + 4 * q + j) * kMH + 16 * nt + r] = accW2[i][j];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int tile = 4 * w + i, mt = tile >> 1, nt = tile & 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) part[kPartW1 + (16 * mt + 4 * q + j) * kMK + 16 * nt + r] = accW1[i][j];
  }
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float b1 = sum16(g_b1[t][j]), b2 = sum16(g_b2[t][j]), w3 = sum16(g_w3[t][j]);
      if (r == 0) {
        const int hid = 16 * t + 4 * q + j;
        s.sums[w][0][hid] = b1;
        s.sums[w][1][hid] = b2;
        s.sums[w][2][hid] = w3;
      }
    }
  // q == 0 lanes hold one row each: sum over the wave's 16 rows
  const float b3w = sum16(g_b3), lw = sum16(loss);
  if (lane == 0) {
    s.tail[w][0] = b3w;
    s.tail[w][1] = lw;
  }
  __syncthreads();
  for (int i = tid; i < kMH; i += kTrainThreads) {
    float b1 = 0.0f, b2 = 0.0f, w3 = 0.0f;
#pragma unroll
    for (int v = 0; v < kTrainWaves; ++v) {
      b1 += s.sums[v][0][i];
      b2 += s.sums[v][1][i];
      w3 += s.sums[v][2][i];
    }
    part[kPartB1 + i] = b1;
    part[kPartB2 + i] = b2;
    part[kPartW3 + i] = w3;
  }
  if (tid == 0) {
    float b3 = 0.0f, l = 0.0f;
#pragma unroll
    for (int v = 0; v < kTrainWaves; ++v) {
      b3 += s.tail[v][0];
      l += s.tail[v][1];
    }
    part[kPartB3] = b3;
    part[kPartLoss] = l;
  }
  for (int64_t i = kPartLoss + 1 + tid; i < kPartStride; i += kTrainThreads) part[i] = 0.0f;
}

// Pairwise ranking loss, one workgroup per group of `group` consecutive rows
// (one kernel instance's configurations).  z = ln score (feature 22, raw) +
// Delta is the corrected key; every ordered pair (i, j) with y_i < y_j (y the
// measured log runtime) costs softplus(z_i - z_j), and the loss is the mean
// over pairs within each group, averaged over the groups.  dL/dz_i =
// (sum over j after i of sigma(z_i - z_j) - sum over j before i of
// sigma(z_j - z_i)) / (groups x pairs of the group); dL/dDelta = dL/dz.
__global__ __launch_bounds__(256) void sa_train_rank_kernel(const float *feat, const float *target, int32_t group,
                                                            float inv_groups, TrainBufs T) {
  extern __shared__ float zy[];  // z[group], y[group]
  __shared__ int pairs;
  const int64_t g0 = (int64_t)blockIdx.x * group;
  if (threadIdx.x == 0) pairs = 0;
  for (int i = threadIdx.x; i < group; i += blockDim.x) {
    zy[i] = feat[(g0 + i) * kF + 22] + T.delta[g0 + i];
    zy[group + i] = target[g0 + i];
  }
  __syncthreads();
  int mine = 0;
  for (int i = threadIdx.x; i < group; i += blockDim.x)
    for (int j = 0; j < group; ++j) mine += zy[group + i] < zy[group + j] ? 1 : 0;
  atomicAdd(&pairs, mine);
  __syncthreads();
  const float w = pairs > 0 ? inv_groups / (float)pairs : 0.0f;
  for (int i = threadIdx.x; i < group; i += blockDim.x) {
    const float zi = zy[i], yi = zy[group + i];
    float g = 0.0f, l = 0.0f;
    for (int j = 0; j < group; ++j) {
      const float zj = zy[j], yj = zy[group + j];
      if (yi < yj) {
        const float x = zi - zj;
        g += 1.0f / (1.0f + expf(-x));
        l += fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
      } else if (yj < yi) {
        g -= 1.0f / (1.0f + expf(zi - zj));
      }
    }
    T.gdelta[g0 + i] = g * w;
    T.loss[g0 + i] = l * w;
  }
}

// Sum the workgroups' partials (fixed order: deterministic), then Adam on the
// fp32 master weights and the bf16 shadow.  A workgroup takes 64 parameters:
// each of its four waves adds every fourth partial (into four running sums,
// up to 16 loads in flight per lane), and the four sums are added in wave
// order.  With a step counter,
// the bias corrections follow the count the training kernel has just
// advanced.
constexpr int kAdamParams = 64;

__global__ __launch_bounds__(256) void sa_train_adam_kernel(TrainState S, MlpDev Mw, const float *part,
                                                            int64_t n_parts, AdamArgs h, float *grad_out) {
  __shared__ float red[4][kAdamParams];
  const int j = threadIdx.x & (kAdamParams - 1), wv = threadIdx.x / kAdamParams;
  const int64_t i = (int64_t)blockIdx.x * kAdamParams + j;
  // the bias corrections first (wave 0 applies the update): their binary64
  // powers then overlap the partials' loads instead of following the barrier
  float bc1 = h.bc1, bc2 = h.bc2;
  if (h.step_counter && wv == 0) {
    const double t = (double)*h.step_counter;
    bc1 = (float)(1.0 - pow(h.beta1_d, t));
    bc2 = (float)(1.0 - pow(h.beta2_d, t));
  }
  float g = 0.0f;
  if (i < kPartStride) {
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int64_t p = wv;
#pragma unroll 4
    for (; p + 12 < n_parts; p += 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += part[(p + 4 * u) * kPartStride + i];
    }
    for (; p < n_parts; p += 4) acc[0] += part[p * kPartStride + i];
    g = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
  red[wv][j] = g;
  __syncthreads();
  if (wv != 0 || i >= kPartStride) return;
  g = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
  if (grad_out) grad_out[i] = i == kPartLoss ? g * h.inv_n : g;
  if (i >= kPartUsed) return;
  const float m = h.beta1 * S.m[i] + (1.0f - h.beta1) * g;
  const float v = h.beta2 * S.v[i] + (1.0f - h.beta2) * g * g;
  S.m[i] = m;
  S.v[i] = v;
  const float mh = m / bc1, vh = v / bc2;
  const float p = S.master[i] - h.lr * mh / (sqrtf(vh) + h.eps);
  S.master[i] = p;
  uint16_t *W1 = (uint16_t *)Mw.W1, *W2 = (uint16_t *)Mw.W2, *w3 = (uint16_t *)Mw.w3;
  float *b1 = (float *)Mw.b1, *b2 = (float *)Mw.b2, *b3 = (float *)Mw.b3;
  if (i < kPartW1 + kMH * kMK && i >= kPartW1) {
    const int64_t jw = i - kPartW1;
    W1[jw] = (jw % kMK) < kF ? f2bf(p) : 0;  // padding inputs stay zero
    if ((jw % kMK) >= kF) S.master[i] = 0.0f;
  } else if (i >= kPartW2 && i < kPartW2 + kMH * kMH) {
    W2[i - kPartW2] = f2bf(p);
  } else if (i >= kPartW3 && i < kPartW3 + kMH) {
    w3[i - kPartW3] = f2bf(p);
  } else if (i >= kPartB1 && i < kPartB1 + kMH) {
    b1[i - kPartB1] = p;
  } else if (i >= kPartB2 && i < kPartB2 + kMH) {
    b2[i - kPartB2] = p;
  } else if (i == kPartB3) {
    b3[0] = p;
  }
}

}  // namespace

hipError_t launch_features(const EvalLaunch &L, float *feat, hipStream_t stream) {
  if (L.n_evals == 0) return hipSuccess;
  int64_t blocks = (L.n_evals + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(sa_features_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, L, feat);
  return hipGetLastError();
}

hipError_t launch_mlp_fwd(const MlpDev &M, const float *feat, int64_t n, float *delta, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const int64_t n_blocks = (n + 63) / 64;
  int64_t grid = (n_blocks + kFwdWaves - 1) / kFwdWaves;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(sa_mlp_fwd_kernel, dim3((uint32_t)grid), dim3(64 * kFwdWaves), 0, stream, M, feat, n, delta);
  return hipGetLastError();
}

int64_t train_partials(int64_t n) {
  const int64_t passes = (n + kTrainRows - 1) / kTrainRows;
  return passes < kMaxPartials ? passes : kMaxPartials;
}

hipError_t launch_train_step(const MlpDev &M, TrainState S, const float *feat, const float *target, int64_t n,
                             TrainBufs T, AdamArgs h, float *grad_out, int32_t group, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const int64_t parts = train_partials(n);
  hipError_t e;
  if (group > 0) {
    // this step's Delta (the same values the fused kernel recomputes), then the
    // ranking loss's per-row gradients
    if ((e = launch_mlp_fwd(M, feat, n, T.delta, stream)) != hipSuccess) return e;
    const int64_t groups = n / group;
    hipLaunchKernelGGL(sa_train_rank_kernel, dim3((uint32_t)groups), dim3(256), (size_t)(2 * group) * sizeof(float),
                       stream, feat, target, group, 1.0f / (float)groups, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(sa_train_kernel<1>, dim3((uint32_t)parts), dim3(kTrainThreads), 0, stream, M, feat, target, n, T,
                       h.step_counter);
  } else {
    hipLaunchKernelGGL(sa_train_kernel<0>, dim3((uint32_t)parts), dim3(kTrainThreads), 0, stream, M, feat, target, n, T,
                       h.step_counter);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(sa_train_adam_kernel, dim3((uint32_t)((kPartStride + kAdamParams - 1) / kAdamParams)), dim3(256),
                     0, stream, S, M, T.part, parts, h, grad_out);
  return hipGetLastError();
}

}  // namespace sa
