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

// Inference GELU from an LDS table of linear pieces.  The forward pass works
// on the scaled pre-activation u = a / 16 + 1/2: the weights of the first two
// layers are staged multiplied by 1/16 (exact in bfloat16) and their biases
// as b / 16 + 1/2, so the matrix cores deliver u directly, and u in [0, 1)
// covers a in [-8, 8).  Piece i covers u in [i, i + 1) / 1024 (a width of
// 1/64 in a) and holds the chord of GELU between a_i = (i - 512) / 64 and
// a_i+1 as GELU ~ g0_i + u g1_i, so one multiply-add gives the value: the
// chord's error is at most h^2 / 8 max|GELU''| = 2.4e-5 (h = 1/64, GELU'' =
// phi(a) (2 - a^2) peaks at 2 phi(0)), well below the bfloat16 rounding that
// follows.  Piece 0 (a < -8 + 1/64) is zero and piece 1023 (a >= 8 - 1/64)
// is the identity a = 16 (u - 1/2); so an index clamped to [0, 1023] also
// covers every u outside [0, 1): GELU(a) differs from 0 below a = -8 and
// from a above a = 8 by less than 1e-14.  The index of two values comes from
// one conversion: v_cvt_pknorm_u16_f32 clamps both to [0, 1] and rounds
// them to 16-bit fractions m = round(65535 u), whose top ten bits are the
// piece (m / 64 differs from 1024 u by less than 1/64 + 1/128 of a piece, so
// near a piece's edge the neighbouring chord may be taken: both pass through
// the edge, and the chord extended by that much stays within 1e-7 of GELU).
constexpr int kGeluN = 1024;
constexpr float kTScale = 1.0f / 16.0f;
constexpr float kTOrigin = 0.5f;
typedef float f32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double gelu_exact(double a) { return 0.5 * a * erfc(-a * 0.70710678118654752440); }

// Binary64 GELU at the edge a_i = (i - 512) / 64 of pieces i - 1 and i.
__device__ __forceinline__ double gelu_edge(int i) { return gelu_exact((double)(i - 512) / 64.0); }

// (g0, g1) of piece i, from the binary64 GELU at its ends y0 = gelu_edge(i)
// and y1 = gelu_edge(i + 1) (not read for the first and last piece).
__device__ __forceinline__ f32x2_t gelu_piece(int i, double y0, double y1) {
  if (i <= 0) return f32x2_t{0.0f, 0.0f};
  if (i >= kGeluN - 1) return f32x2_t{-kTOrigin / kTScale, 1.0f / kTScale};
  const double g1 = (y1 - y0) * kGeluN;  // per unit of u
  return f32x2_t{(float)(y0 - (double)i / kGeluN * g1), (float)g1};
}

// GELU of N (even) scaled pre-activations in place.  All table positions
// are computed and all reads issued before the first multiply-add, so that
// the reads' latency overlaps.
template <int N>
__device__ __forceinline__ void gelu_t_n(float (&t)[N], const f32x2_t *tab) {
  static_assert(N % 2 == 0, "pairs of values");
  const char *base = (const char *)tab;
  f32x2_t c[N];
#pragma unroll
  for (int i = 0; i < N; i += 2) {
    uint32_t m = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pknorm_u16(t[i], t[i + 1]));
    // Both 16-bit fractions cut to their piece (the top ten bits) at once;
    // the byte offsets 8 piece are then one field extract (low half) and one
    // shift (high half).  The empty statement keeps the compiler from folding
    // the mask into each offset, which takes two instructions apiece.
    m &= 0xFFC0FFC0u;
    __asm__ volatile("" : "+v"(m));
    c[i] = *(const f32x2_t *)(base + __builtin_amdgcn_ubfe(m, 3u, 13u));
    c[i + 1] = *(const f32x2_t *)(base + (m >> 19));
  }
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = fmaf(t[i], c[i].y, c[i].x);
}


// ---------------------------------------------------------------- features

// The variant's features (binary32): f0-f8, f19 and f23.
// Natural logarithm by the device's base-2 logarithm (v_log_f32, about one
// ulp) times ln 2: two instructions where the library's logf takes about
// twenty, within the features' tolerance for the positive, normal arguments
// used here.
__device__ __forceinline__ float dev_ln(float x) { return __builtin_amdgcn_logf(x) * 0.693147182f; }

// ln(1 + n) of a count (1 + n is exact in binary32 below 2^24).
__device__ __forceinline__ float ln1p_count(int32_t n) { return dev_ln(1.0f + (float)n); }

// The variant's features (binary32): f0-f8, f19 and f23.
__device__ __forceinline__ void variant_features(float *f, int32_t nfp, int32_t nint, int32_t nld, int32_t nst,
                                                 int32_t nbr, int32_t nbar, int32_t nreg, int32_t S, float d) {
  f[0] = ln1p_count(nfp);
  f[1] = ln1p_count(nint);
  f[2] = ln1p_count(nld);
  f[3] = ln1p_count(nst);
  f[4] = ln1p_count(nbr);
  f[5] = (float)nbar * 0.25f;
  f[6] = ln1p_count(nreg);
  f[7] = (float)S * (1.0f / 65536.0f);
  f[8] = d;
  const int32_t mem = nld + nst;
  const float inten = (float)nfp / (float)(mem > 1 ? mem : 1);
  f[19] = dev_ln(1.0f + inten);
  // decided on the integers: n_fp / m > 4 exactly when n_fp > 4 m
  f[23] = nfp > 4 * (mem > 1 ? mem : 1) ? 1.0f : 0.0f;
}

// The configuration's features: f9-f18 and f20-f22.  Per evaluation, so the
// logarithms are the device's and the divisions are products with binary32
// reciprocals (constants, or v_rcp_f32 for 1/F): each within an ulp or two
// of the correctly rounded value, far inside the features' tolerance, at a
// tenth of the instructions of the library's logf and IEEE division.
__device__ __forceinline__ void config_features(float *f, int32_t T, int32_t U, int32_t R, int32_t G, bool has_grid,
                                                int32_t n_cu, int32_t WB, int32_t gw, int32_t gr, int32_t gs,
                                                int32_t B, int32_t W, float Ed, float F, float sc) {
  f[9] = __builtin_amdgcn_logf((float)T) * 0.1f;
  f[10] = (float)(U - 1) * (1.0f / 7.0f);
  f[11] = (float)R * (1.0f / 512.0f);
  f[12] = has_grid ? (__builtin_amdgcn_logf((float)G) - __builtin_amdgcn_logf((float)n_cu)) * (1.0f / 3.0f) : 0.0f;
  f[13] = (float)WB * (1.0f / 16.0f);
  f[14] = (float)(gw < 32 ? gw : 32) * (1.0f / 32.0f);
  f[15] = (float)(gr < 32 ? gr : 32) * (1.0f / 32.0f);
  f[16] = (float)(gs < 32 ? gs : 32) * (1.0f / 32.0f);
  f[17] = (float)B * (1.0f / 32.0f);
  f[18] = (float)W * (1.0f / 32.0f);
  f[20] = dev_ln(Ed);
  f[21] = __builtin_amdgcn_rcpf(F);
  f[22] = dev_ln(sc);
}

// ---------------------------------------------------------------- forward pass

constexpr int kLdXin = kMF;  // input row stride (bf16): the 24 features, no padding
// MFMA operand slice of inputs 24..31: 1, 1 | 1, 0 | 0, 0 | 0, 0 (bfloat16
// pairs, low half first), the ones that carry the folded first-layer bias
constexpr uint32_t kOnes24 = 0x3F803F80u, kOnes26 = 0x00003F80u;

struct __align__(16) MlpLdsT {
  uint16_t W1[kMH * kLdW1];  // W1[h][k] / 16
  uint16_t W2[kMH * kLdW2];  // W2[o][.] / 16, columns permuted per 32-wide chunk (see w2_column)
  uint16_t w3p[kMH];         // w3 in the same permuted order
  float b2[kMH];             // b2 / 16 + 1/2 (b1 is folded into W1, see load_weights_t)
  union {
    f32x2_t gelu[kGeluN];    // pieces (g0, g1)
    double edge[kGeluN];     // while staging: GELU at the inner piece edges
  };
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

// Position of hidden unit u in a permuted row: the inverse of w2_column.
__device__ __forceinline__ int w2_position(int u) {
  const int c = u >> 5, m = u & 31;
  return m < 16 ? 32 * c + 8 * (m >> 2) + (m & 3) : 32 * c + 8 * ((m - 16) >> 2) + 4 + (m & 3);
}

// bfloat16 bits times kTScale (exact: only the exponent changes; zero stays
// zero; weights this small never reach the subnormals).
__device__ __forceinline__ uint16_t bf16_scaled(uint16_t b) {
  const float x = __builtin_bit_cast(float, (uint32_t)b << 16) * kTScale;
  return (uint16_t)(__builtin_bit_cast(uint32_t, x) >> 16);
}

// The first layer's bias enters its contraction: inputs 24..26 of every row
// (padding, zero in the network) are 1 in the MFMA operand (kOnes24 / kOnes26,
// the slice of inputs 24..31), and the staged W1 columns 24..26 hold the scaled
// bias v = b1 / 16 + 1/2 split into three bfloat16 parts, hi + mid + lo = v
// exactly (each part takes the next 8 significant bits of the remainder), so
// the first layer reads no bias tile.  W1's own columns 24..31 multiply
// zero inputs in the network and are not staged for 24..26.
__device__ __forceinline__ uint16_t bf16_rn(float x) { return (uint16_t)(pack_bf16(x, 0.0f) & 0xFFFFu); }
__device__ __forceinline__ float bf16_value(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// Two bfloat16 (low half first) times kTScale each.
__device__ __forceinline__ uint32_t bf16x2_scaled(uint32_t u) {
  return (uint32_t)bf16_scaled((uint16_t)(u & 0xFFFFu)) | ((uint32_t)bf16_scaled((uint16_t)(u >> 16)) << 16);
}
__device__ __forceinline__ u32x4_t bf16x8_scaled(u32x4_t x) {
  return u32x4_t{bf16x2_scaled(x[0]), bf16x2_scaled(x[1]), bf16x2_scaled(x[2]), bf16x2_scaled(x[3])};
}

// The first layer's scaled bias for hidden unit h as its three bfloat16
// parts hi, mid, lo (hi + mid + lo = b1 / 16 + 1/2 exactly).
__device__ __forceinline__ void bias_split(const MlpDev &M, int h, uint16_t &hi, uint16_t &mid, uint16_t &lo) {
  const float v = fmaf(M.b1[h], kTScale, kTOrigin);
  hi = bf16_rn(v);
  const float r1 = v - bf16_value(hi);
  mid = bf16_rn(r1);
  lo = bf16_rn(r1 - bf16_value(mid));
}

// Staging of the weights in LDS.  With 16-byte aligned weight arrays (the
// usual case) every thread moves whole 16-byte pieces, all of its loads in
// flight at once: a W1 row is four pieces (the last one's first three slots
// take the bias split), a W2 row sixteen, each splitting into two 4-column
// runs whose positions w2_column permutes as a whole (run a of a 32-wide
// chunk, columns 32 c + 4 a .. + 3, lands at 32 c + 8 (a mod 4) + 4 (a / 4)).
// Otherwise element by element, to the same result.  With W2t (training's
// backward), W2 is also written there transposed, unscaled and with its rows
// permuted as the forward's columns are: W2t[k][w2_position(o)] = W2[o][k]
// (rows of kLdW2 elements), each loaded piece's eight values stored at once
// from the same registers.
__device__ void load_weights_t(const MlpDev &M, MlpLdsT &s, int tid, int nthreads, uint16_t *W2t = nullptr) {
  const bool vec = (((uintptr_t)M.W1 | (uintptr_t)M.W2) & 15u) == 0;
  if (vec) {
    for (int i = tid; i < kMH * (kMK / 8); i += nthreads) {
      const int h = i / (kMK / 8), m = i % (kMK / 8);
      u32x4_t x = bf16x8_scaled(*(const u32x4_t *)(M.W1 + h * kMK + 8 * m));
      if (8 * m == kMF) {
        uint16_t hi, mid, lo;
        bias_split(M, h, hi, mid, lo);
        x[0] = (uint32_t)hi | ((uint32_t)mid << 16);
        x[1] = (uint32_t)lo | (x[1] & 0xFFFF0000u);
      }
      *(u32x4_t *)(s.W1 + h * kLdW1 + 8 * m) = x;
    }
    typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
    for (int i = tid; i < kMH * (kMH / 8); i += nthreads) {
      const int o = i / (kMH / 8), m = i % (kMH / 8), a0 = 2 * (m & 3), a1 = a0 + 1;
      const u32x4_t raw = *(const u32x4_t *)(M.W2 + o * kMH + 8 * m);
      const u32x4_t x = bf16x8_scaled(raw);
      uint16_t *row = s.W2 + o * kLdW2 + 32 * (m >> 2);
      *(u32x2_t *)(row + 8 * (a0 & 3) + 4 * (a0 >> 2)) = u32x2_t{x[0], x[1]};
      *(u32x2_t *)(row + 8 * (a1 & 3) + 4 * (a1 >> 2)) = u32x2_t{x[2], x[3]};
      if (W2t) {
        uint16_t *col = W2t + 8 * m * kLdW2 + w2_position(o);
#pragma unroll
        for (int j = 0; j < 8; ++j) col[j * kLdW2] = (uint16_t)(raw[j >> 1] >> (16 * (j & 1)));
      }
    }
  } else {
    for (int i = tid; i < kMH * kMK; i += nthreads) {
      const int k = i % kMK;
      if (k >= kMF && k < kMF + 3) continue;
      s.W1[(i / kMK) * kLdW1 + k] = bf16_scaled(M.W1[i]);
    }
    for (int i = tid; i < kMH; i += nthreads) {
      uint16_t hi, mid, lo;
      bias_split(M, i, hi, mid, lo);
      s.W1[i * kLdW1 + kMF] = hi;
      s.W1[i * kLdW1 + kMF + 1] = mid;
      s.W1[i * kLdW1 + kMF + 2] = lo;
    }
    for (int i = tid; i < kMH * kMH; i += nthreads) {
      const int o = i / kMH, p = i % kMH;
      s.W2[o * kLdW2 + p] = bf16_scaled(M.W2[o * kMH + w2_column(p)]);
      if (W2t) W2t[p * kLdW2 + w2_position(o)] = M.W2[o * kMH + p];
    }
  }
  for (int i = tid; i < kMH; i += nthreads) {
    s.b2[i] = fmaf(M.b2[i], kTScale, kTOrigin);
    s.w3p[i] = M.w3[w2_column(i)];
  }
  for (int i = tid; i < kMF; i += nthreads) {
    s.mean[i] = M.mean[i];
    s.inv_std[i] = M.inv_std[i];
  }
  // GELU pieces: each inner edge's value once (binary64, held in the table's
  // own storage), then every piece from its two edges.  nthreads >= 256.
  for (int i = 1 + tid; i < kGeluN; i += nthreads) s.edge[i] = gelu_edge(i);
  __syncthreads();
  f32x2_t piece[kGeluN / 256];
#pragma unroll
  for (int r = 0; r < kGeluN / 256; ++r) {
    const int i = tid + r * nthreads;
    if (i < kGeluN) {
      const bool inner = i > 0 && i < kGeluN - 1;
      piece[r] = gelu_piece(i, inner ? s.edge[i] : 0.0, inner ? s.edge[i + 1] : 0.0);
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kGeluN / 256; ++r) {
    const int i = tid + r * nthreads;
    if (i < kGeluN) s.gelu[i] = piece[r];
  }
  if (tid == 0) s.b3 = M.b3[0];
}

// Features i0 .. i0 + 2 n - 1 as network inputs: bf16((f - mean) * inv_std),
// packed in pairs.  (One multiply-add with a precomputed -mean inv_std
// would lose the exact difference f - mean: near-constant features, whose
// inv_std is large, then come out visibly wrong.)
template <int N>
__device__ __forceinline__ void pack_inputs(const MlpLdsT &s, const float *f, int i0, uint32_t *p) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int a = i0 + 2 * i;
    p[i] = pack_bf16((f[a] - s.mean[a]) * s.inv_std[a], (f[a + 1] - s.mean[a + 1]) * s.inv_std[a + 1]);
  }
}

// Row `row` of the wave's input block: the 24 inputs (three 16-byte slices).
// `zero` writes an all-zero row (rows that do not exist).
__device__ __forceinline__ void put_x(const MlpLdsT &s, uint16_t *X, int row, const float *f, bool zero) {
  uint32_t p[12];
  pack_inputs<12>(s, f, 0, p);
  u32x4_t *dst = (u32x4_t *)(X + row * kLdXin);
#pragma unroll
  for (int j = 0; j < 3; ++j)
    dst[j] = zero ? u32x4_t{0u, 0u, 0u, 0u} : u32x4_t{p[4 * j], p[4 * j + 1], p[4 * j + 2], p[4 * j + 3]};
}

// The same row when inputs 0..7 (slice 0) are the variant's and shared by
// every row of the block: only slices 1 and 2 (inputs 8..23) are written.
// Rows of illegal configurations keep their non-finite inputs: every
// column of a contraction is one row, so they reach only their own Delta,
// which the caller discards.
__device__ __forceinline__ void put_x_cfg(const MlpLdsT &s, uint16_t *X, int row, const float *f) {
  uint32_t p[8];
  pack_inputs<8>(s, f, 8, p);
  u32x4_t *dst = (u32x4_t *)(X + row * kLdXin);
#pragma unroll
  for (int j = 0; j < 2; ++j) dst[j + 1] = u32x4_t{p[4 * j], p[4 * j + 1], p[4 * j + 2], p[4 * j + 3]};
}

__device__ __forceinline__ f32x4_t mfma32(u32x4_t a, u32x4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                 0, 0, 0);
}

// The values of RT row tiles of an MFMA output through GELU, packed to
// bfloat16 in pairs: out[i][0..1] for row tile i.  Eight values at a time,
// so that eight table reads are in flight before the first multiply-add.
template <int RT>
__device__ __forceinline__ void gelu_pack(const f32x4_t (&d)[RT], const f32x2_t *tab, uint32_t (&out)[RT][2]) {
#pragma unroll
  for (int i0 = 0; i0 < RT; i0 += 2) {
    float v[8];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) v[4 * i + j] = d[i0 + i][j];
    gelu_t_n<8>(v, tab);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      out[i0 + i][0] = pack_bf16(v[4 * i], v[4 * i + 1]);
      out[i0 + i][1] = pack_bf16(v[4 * i + 2], v[4 * i + 3]);
    }
  }
}

// Delta of row `lane` of the wave's 64-row input block X (put_x rows; the
// caller orders the writes before this call).  h1 = bf16(GELU(W1 x + b1)),
// h2 = bf16(GELU(W2 h1 + b2)), Delta = w3 . h2 + b3, all three layers on the
// matrix cores with fp32 accumulation, in 4 / RT passes of RT row tiles (16
// rows each): every weight tile read from LDS serves the RT row tiles of a
// pass, so more row tiles per pass read fewer weight bytes per row, and one
// pass's first hidden layer takes 16 RT registers.  A layer's output tiles
// (hidden units 16 t + 4 q + j of row r at lane 16 q + r) are, packed in
// pairs, the B operands of the next layer once its weight columns are
// permuted as in w2_column.  Input slice q = 3 (inputs 24..31) is
// kOnes24 / kOnes26: the first layer's bias is part of its contraction.
// The third layer multiplies every A row by w3, so row 4 q of its result,
// which lane 16 q + r holds, is the sum for row r of the row tile.  SHARED:
// slice 0 of every row is `xv` (put_x_cfg rows), not read from X.
template <bool SHARED, int RT>
__device__ __forceinline__ float mlp_rows(const MlpLdsT &s, const uint16_t *X, int lane, u32x4_t xv) {
  static_assert(RT == 2 || RT == 4, "row tiles per pass");
  const int r = lane & 15, q = lane >> 4;
  const int qx = q == 0 ? (SHARED ? 1 : 0) : (q < 3 ? q : 2);
  float delta = 0.0f;
#pragma unroll 1
  for (int p = 0; p < 4 / RT; ++p) {
    u32x4_t xb[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const u32x4_t x = *(const u32x4_t *)(X + (16 * (RT * p + i) + r) * kLdXin + 8 * qx);
      xb[i] = q == 3 ? u32x4_t{kOnes24, kOnes26, 0u, 0u} : ((SHARED && q == 0) ? xv : x);
    }
    // layer 1: hidden tile t -> RT row tiles x 4 packed bf16 (two dwords).
    // Software-pipelined: tile t + 1's MFMAs are issued before tile t's GELU,
    // so that the matrix cores work while the vector unit does the table GELU.
    uint32_t h1[8][RT][2];
    auto l1 = [&](int t, f32x4_t (&d)[RT]) {
      const u32x4_t a = *(const u32x4_t *)(s.W1 + (16 * t + r) * kLdW1 + 8 * q);
#pragma unroll
      for (int i = 0; i < RT; ++i) d[i] = mfma32(a, xb[i], f32x4_t{0.0f, 0.0f, 0.0f, 0.0f});
    };
    f32x4_t d_cur[RT], d_nxt[RT];
    l1(0, d_cur);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (t < 7) l1(t + 1, d_nxt);
      gelu_pack<RT>(d_cur, s.gelu, h1[t]);
      if (t < 7) {
#pragma unroll
        for (int i = 0; i < RT; ++i) d_cur[i] = d_nxt[i];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // layers 2 and 3, pipelined the same way over the 8 output tiles; each
    // pair of tiles (a 32-unit chunk) feeds the third layer at once
    auto l2 = [&](int ot, f32x4_t (&acc)[RT]) {
      const f32x4_t bias = *(const f32x4_t *)(s.b2 + 16 * ot + 4 * q);
#pragma unroll
      for (int i = 0; i < RT; ++i) acc[i] = bias;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const u32x4_t a = *(const u32x4_t *)(s.W2 + (16 * ot + r) * kLdW2 + 32 * c + 8 * q);
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          const u32x4_t b = {h1[2 * c][i][0], h1[2 * c][i][1], h1[2 * c + 1][i][0], h1[2 * c + 1][i][1]};
          acc[i] = mfma32(a, b, acc[i]);
        }
      }
    };
    f32x4_t acc3[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) acc3[i] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
    f32x4_t a_cur[RT], a_nxt[RT];
    uint32_t h2[2][RT][2];
    l2(0, a_cur);
#pragma unroll
    for (int ot = 0; ot < 8; ++ot) {
      if (ot < 7) l2(ot + 1, a_nxt);
      gelu_pack<RT>(a_cur, s.gelu, h2[ot & 1]);
      if (ot & 1) {
        const u32x4_t a3 = *(const u32x4_t *)(s.w3p + 32 * (ot >> 1) + 8 * q);
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          const u32x4_t b = {h2[0][i][0], h2[0][i][1], h2[1][i][0], h2[1][i][1]};
          acc3[i] = mfma32(a3, b, acc3[i]);
        }
      }
      if (ot < 7) {
#pragma unroll
        for (int i = 0; i < RT; ++i) a_cur[i] = a_nxt[i];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // lane l = 16 q + r owns row l, which is row r of row tile q
#pragma unroll
    for (int i = 0; i < RT; ++i) delta = q == RT * p + i ? acc3[i][0] : delta;
  }
  return delta + s.b3;
}

}  // namespace
}  // namespace sa
