// Device building blocks of the learned correction shared by the standalone
// inference kernel and the fused corrected scoring pass: bfloat16 rounding,
// GELU, the 24 features and the forward pass of one wave's 64 rows.
//
// Forward layout.  The hidden units are the M dimension and the rows the N
// dimension of v_mfma_f32_16x16x32_bf16: for D (16 x 16) += A (16 x 32) B
// (32 x 16), lane l = 16 q + r supplies A[r][8 q .. 8 q + 7] and
// B[8 q .. 8 q + 7][r] as eight bf16 each and receives D[4 q + j][r],
// j = 0..3.  The first layer's output tile (hidden 16 t + 4 q + j, row r)
// is then already where the second layer wants its B operand: for the
// contraction chunk of hidden units 32 c .. 32 c + 31 a lane's eight slots
// hold the four values of tile 2 c and the four of tile 2 c + 1, and the
// second layer's weights are stored with their columns permuted the same
// way.  The first hidden layer never leaves registers; only the inputs go
// through LDS (each lane writes its row, then reads the slices MFMA needs).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa_internal.h"

namespace sa {
namespace {

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kMH = 128;          // hidden width
constexpr int kMK = 32;           // padded input width
constexpr int kMF = 24;           // features
constexpr int kLdW1 = kMK + 8;    // LDS row strides in bf16 elements (16-byte padding)
constexpr int kLdW2 = kMH + 8;
constexpr int kLdXT = kMK + 8;

// Two binary32 values rounded to bfloat16 (nearest, ties to even), packed
// low half first.
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  const bf16x2_t p = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, p);
}

// erf for x = |a| / sqrt 2 by Abramowitz & Stegun 7.1.26 (absolute error at
// most 1.5e-7): 1 - erf(x) = t P(t) exp(-x^2), t = 1 / (1 + p x).  Returns
// half of it, the normal upper tail Q(|a|), and exp(-a^2 / 2) in e.
__device__ __forceinline__ float normal_tail(float a, float &e) {
  const float ax = fabsf(a);
  const float t = __builtin_amdgcn_rcpf(fmaf(ax, 0.23164189f, 1.0f));  // p / sqrt 2
  float y = fmaf(t, 1.061405429f, -1.453152027f);
  y = fmaf(t, y, 1.421413741f);
  y = fmaf(t, y, -0.284496736f);
  y = fmaf(t, y, 0.254829592f);
  y = y * t;
  e = __builtin_amdgcn_exp2f((a * a) * -0.72134752f);  // exp(-a^2 / 2) = 2^(-a^2 / (2 ln 2))
  return 0.5f * (y * e);
}

// GELU(a) = a Phi(a) = relu(a) - |a| Q(|a|).
__device__ __forceinline__ float gelu(float a) {
  float e;
  const float q = normal_tail(a, e);
  return fmaf(-fabsf(a), q, fmaxf(a, 0.0f));
}

// GELU'(a) = Phi(a) + a phi(a).
__device__ __forceinline__ float gelu_grad(float a) {
  float e;
  const float q = normal_tail(a, e);
  const float phi_cdf = a >= 0.0f ? 1.0f - q : q;
  return fmaf(a * e, 0.39894228f, phi_cdf);
}

// Inference GELU from an LDS table of the normal CDF: Phi sampled at
// a_i = -8 + i / 32 (i = 0..512, exact erfc at table build), linearly
// interpolated; a Phi(a) outside [-8, 8] is relu(a) to within 1e-14.  The
// interpolation error of Phi is at most h^2 / 8 max|Phi''| = 3.0e-5 (h = 1/32),
// far below the bfloat16 rounding that follows.
constexpr int kGeluN = 512;
typedef float f32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float phi_exact(float x) { return 0.5f * erfcf(-x * 0.70710678118654752f); }

// GELU of N values in place.  All table positions are computed first and all
// reads issued before the first interpolation, so that the reads' latency
// overlaps instead of being paid once per value.  For t in [0, 512) the
// fractional part t - floor(t) is exact.
template <int N>
__device__ __forceinline__ void gelu_tab_n(float (&a)[N], const f32x2_t *tab) {
  int idx[N];
  float fr[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float t = __builtin_amdgcn_fmed3f(fmaf(a[i], 32.0f, 256.0f), 0.0f, 511.99997f);
    idx[i] = (int)t;
    fr[i] = __builtin_amdgcn_fractf(t);
  }
  f32x2_t e[N];
#pragma unroll
  for (int i = 0; i < N; ++i) e[i] = tab[idx[i]];
#pragma unroll
  for (int i = 0; i < N; ++i) a[i] = a[i] * fmaf(fr[i], e[i].y, e[i].x);
}

// ---------------------------------------------------------------- features

// The variant's features (binary32): f0-f8, f19 and f23.
__device__ __forceinline__ void variant_features(float *f, int32_t nfp, int32_t nint, int32_t nld, int32_t nst,
                                                 int32_t nbr, int32_t nbar, int32_t nreg, int32_t S, float d) {
  f[0] = log1pf((float)nfp);
  f[1] = log1pf((float)nint);
  f[2] = log1pf((float)nld);
  f[3] = log1pf((float)nst);
  f[4] = log1pf((float)nbr);
  f[5] = (float)nbar / 4.0f;
  f[6] = log1pf((float)nreg);
  f[7] = (float)S / 65536.0f;
  f[8] = d;
  const int32_t mem = nld + nst;
  const float inten = (float)nfp / (float)(mem > 1 ? mem : 1);
  f[19] = log1pf(inten);
  // decided on the integers: n_fp / m > 4 exactly when n_fp > 4 m
  f[23] = nfp > 4 * (mem > 1 ? mem : 1) ? 1.0f : 0.0f;
}

// The configuration's features: f9-f18 and f20-f22.
__device__ __forceinline__ void config_features(float *f, int32_t T, int32_t U, int32_t R, int32_t G, bool has_grid,
                                                int32_t n_cu, int32_t WB, int32_t gw, int32_t gr, int32_t gs,
                                                int32_t B, int32_t W, float Ed, float F, float sc) {
  f[9] = log2f((float)T) / 10.0f;
  f[10] = (float)(U - 1) / 7.0f;
  f[11] = (float)R / 512.0f;
  f[12] = has_grid ? log2f((float)G / (float)n_cu) / 3.0f : 0.0f;
  f[13] = (float)WB / 16.0f;
  f[14] = (float)(gw < 32 ? gw : 32) / 32.0f;
  f[15] = (float)(gr < 32 ? gr : 32) / 32.0f;
  f[16] = (float)(gs < 32 ? gs : 32) / 32.0f;
  f[17] = (float)B / 32.0f;
  f[18] = (float)W / 32.0f;
  f[20] = logf(Ed);
  f[21] = 1.0f / F;
  f[22] = logf(sc);
}

// ---------------------------------------------------------------- forward pass

struct __align__(16) MlpLdsT {
  uint16_t W1[kMH * kLdW1];  // W1[h][k]
  uint16_t W2[kMH * kLdW2];  // W2[o][.], columns permuted per 32-wide chunk (see w2_column)
  uint16_t w3p[kMH];         // w3 in the same permuted order
  float b1[kMH], b2[kMH];
  f32x2_t phi[kGeluN + 1];   // (Phi(a_i), Phi(a_i+1) - Phi(a_i))
  float mean[kMF], inv_std[kMF];
  float b3;
};

// Hidden unit stored at position p of a second-layer weight row: in chunk
// c = p / 32, slot 8 q + j holds unit 32 c + 4 q + j (j < 4) or
// 32 c + 16 + 4 q + (j - 4) (j >= 4).
__device__ __forceinline__ int w2_column(int p) {
  const int c = p >> 5, q = (p >> 3) & 3, j = p & 7;
  return 32 * c + (j < 4 ? 4 * q + j : 12 + 4 * q + j);
}

__device__ void load_weights_t(const MlpDev &M, MlpLdsT &s, int tid, int nthreads) {
  for (int i = tid; i < kMH * kMK; i += nthreads) s.W1[(i / kMK) * kLdW1 + (i % kMK)] = M.W1[i];
  for (int i = tid; i < kMH * kMH; i += nthreads) {
    const int o = i / kMH, p = i % kMH;
    s.W2[o * kLdW2 + p] = M.W2[o * kMH + w2_column(p)];
  }
  for (int i = tid; i < kMH; i += nthreads) {
    s.b1[i] = M.b1[i];
    s.b2[i] = M.b2[i];
    s.w3p[i] = M.w3[w2_column(i)];
  }
  for (int i = tid; i < kMF; i += nthreads) {
    s.mean[i] = M.mean[i];
    s.inv_std[i] = M.inv_std[i];
  }
  for (int i = tid; i <= kGeluN; i += nthreads) {
    const float p0 = phi_exact(-8.0f + (float)i / 32.0f);
    const float p1 = i < kGeluN ? phi_exact(-8.0f + (float)(i + 1) / 32.0f) : p0;
    s.phi[i] = f32x2_t{p0, p1 - p0};
  }
  if (tid == 0) s.b3 = M.b3[0];
}

// Row `row` of the wave's input block: bf16((f - mean) * inv_std) for the 24
// features, then eight zeros.  `zero` writes an all-zero row (rows that do
// not exist or are illegal).
__device__ __forceinline__ void put_x(const MlpLdsT &s, uint16_t *X, int row, const float *f, bool zero) {
  uint32_t p[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const float lo = (f[2 * i] - s.mean[2 * i]) * s.inv_std[2 * i];
    const float hi = (f[2 * i + 1] - s.mean[2 * i + 1]) * s.inv_std[2 * i + 1];
    p[i] = zero ? 0u : pack_bf16(lo, hi);
  }
  u32x4_t *dst = (u32x4_t *)(X + row * kLdXT);
  dst[0] = u32x4_t{p[0], p[1], p[2], p[3]};
  dst[1] = u32x4_t{p[4], p[5], p[6], p[7]};
  dst[2] = u32x4_t{p[8], p[9], p[10], p[11]};
  dst[3] = u32x4_t{0u, 0u, 0u, 0u};
}

__device__ __forceinline__ f32x4_t mfma32(u32x4_t a, u32x4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                 0, 0, 0);
}

// Delta of row `lane` of the wave's 64-row input block X (put_x rows; the
// caller orders the writes before this call).  h1 = bf16(GELU(W1 x + b1)),
// h2 = bf16(GELU(W2 h1 + b2)), Delta = w3 . h2 + b3, all three layers on the
// matrix cores with fp32 accumulation.  A layer's output tiles (hidden units
// 16 t + 4 q + j of row r at lane 16 q + r) are, packed in pairs, the B
// operands of the next layer once its weight columns are permuted as in
// w2_column.  The third layer multiplies every A row by w3, so row 4 q of its
// result, which lane 16 q + r holds, is the sum for row r of the row tile.
__device__ __forceinline__ float mlp_rows(const MlpLdsT &s, const uint16_t *X, int lane) {
  const int r = lane & 15, q = lane >> 4;
  u32x4_t xb[4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) xb[rt] = *(const u32x4_t *)(X + (16 * rt + r) * kLdXT + 8 * q);
  // layer 1: h-tile t, row tile rt -> 4 packed bf16 (two dwords)
  uint32_t h1[8][4][2];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const u32x4_t a = *(const u32x4_t *)(s.W1 + (16 * t + r) * kLdW1 + 8 * q);
    const f32x4_t bias = *(const f32x4_t *)(s.b1 + 16 * t + 4 * q);
    float v[16];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const f32x4_t d = mfma32(a, xb[rt], bias);
#pragma unroll
      for (int j = 0; j < 4; ++j) v[4 * rt + j] = d[j];
    }
    gelu_tab_n<16>(v, s.phi);
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      h1[t][rt][0] = pack_bf16(v[4 * rt], v[4 * rt + 1]);
      h1[t][rt][1] = pack_bf16(v[4 * rt + 2], v[4 * rt + 3]);
    }
  }
  // layers 2 and 3, one 32-unit chunk of the second hidden layer at a time
  f32x4_t acc3[4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) acc3[rt] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
  for (int c3 = 0; c3 < 4; ++c3) {
    uint32_t h2[2][4][2];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int ot = 2 * c3 + half;
      const f32x4_t bias = *(const f32x4_t *)(s.b2 + 16 * ot + 4 * q);
      f32x4_t acc[4] = {bias, bias, bias, bias};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const u32x4_t a = *(const u32x4_t *)(s.W2 + (16 * ot + r) * kLdW2 + 32 * c + 8 * q);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
          const u32x4_t b = {h1[2 * c][rt][0], h1[2 * c][rt][1], h1[2 * c + 1][rt][0], h1[2 * c + 1][rt][1]};
          acc[rt] = mfma32(a, b, acc[rt]);
        }
      }
      float v[16];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int j = 0; j < 4; ++j) v[4 * rt + j] = acc[rt][j];
      gelu_tab_n<16>(v, s.phi);
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        h2[half][rt][0] = pack_bf16(v[4 * rt], v[4 * rt + 1]);
        h2[half][rt][1] = pack_bf16(v[4 * rt + 2], v[4 * rt + 3]);
      }
    }
    const u32x4_t a3 = *(const u32x4_t *)(s.w3p + 32 * c3 + 8 * q);
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const u32x4_t b = {h2[0][rt][0], h2[0][rt][1], h2[1][rt][0], h2[1][rt][1]};
      acc3[rt] = mfma32(a3, b, acc3[rt]);
    }
  }
  // lane l = 16 q + r owns row l, which is row r of row tile q
  float d = acc3[0][0];
  d = q == 1 ? acc3[1][0] : d;
  d = q == 2 ? acc3[2][0] : d;
  d = q == 3 ? acc3[3][0] : d;
  return d + s.b3;
}

}  // namespace
}  // namespace sa
