// Learned correction of the static model on gfx950: the 24-feature builder,
// BF16 MFMA forward pass (24 -> 128 -> 128 -> 1, GELU, fp32 accumulation)
// and the training step (forward, MSE, backward with MFMA weight-gradient
// contractions, deterministic two-pass reduction, Adam).
//
// MFMA tiles use v_mfma_f32_16x16x16_bf16: for a 16x16 output tile D (rows
// i, columns j) += A (16 x 16, rows i, k) x B (16 x 16, k, columns j), lane l
// supplies A[l % 16][4 (l / 16) + 0..3] and B[4 (l / 16) + 0..3][l % 16] as
// four bf16 each, and receives D[4 (l / 16) + 0..3][l % 16].  Operands are
// kept in LDS row-major with the contraction index contiguous, rows padded
// so that the sixteen rows a lane group reads fall in different banks.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "sa_internal.h"
#include "sa_mlp_dev.h"

namespace sa {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kH = 128;             // hidden width
constexpr int kK1 = 32;             // padded input width
constexpr int kF = 24;              // features
constexpr int kRows = 64;           // rows per wave block
constexpr int kLdX = kK1 + 4;       // padded LDS row strides (bf16 elements)
constexpr int kLdH = kH + 4;
constexpr int kMlpWaves = 4;        // waves per workgroup
constexpr int kMlpThreads = 64 * kMlpWaves;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }


__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// D(16x16) += A[m0.., k0..k0+16) x B, with B given transposed (Bt[n][k]).
__device__ __forceinline__ v4f mfma_tile(const uint16_t *A, int lda, int m0, const uint16_t *Bt, int ldb, int n0,
                                         int k0, v4f acc, int lane) {
  const int r = lane & 15, q = lane >> 4;
  const v4s a = *(const v4s *)(A + (m0 + r) * lda + k0 + 4 * q);
  const v4s b = *(const v4s *)(Bt + (n0 + r) * ldb + k0 + 4 * q);
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
}

// Sum over the 16 lanes of a lane group (lanes with equal l / 16).
__device__ __forceinline__ float sum16(float v) {
#pragma unroll
  for (int m = 8; m >= 1; m >>= 1) v += __shfl_xor(v, m, 16);
  return v;
}

struct __align__(16) MlpLds {
  uint16_t W1[kH * kLdX];  // W1[n][k], k < 32
  uint16_t W2[kH * kLdH];  // W2[n][k]
  float w3[kH], b1[kH], b2[kH], b3, mean[kF], inv_std[kF];
};

struct __align__(16) WaveBufs {
  uint16_t X[kRows * kLdX];   // normalised inputs, bf16
  uint16_t H1[kRows * kLdH];  // first hidden layer, bf16
};

__device__ void load_weights(const MlpDev &M, MlpLds &s, int tid, int nthreads) {
  for (int i = tid; i < kH * kK1; i += nthreads) s.W1[(i / kK1) * kLdX + (i % kK1)] = M.W1[i];
  for (int i = tid; i < kH * kH; i += nthreads) s.W2[(i / kH) * kLdH + (i % kH)] = M.W2[i];
  for (int i = tid; i < kH; i += nthreads) {
    s.w3[i] = bf2f(M.w3[i]);
    s.b1[i] = M.b1[i];
    s.b2[i] = M.b2[i];
  }
  for (int i = tid; i < kF; i += nthreads) {
    s.mean[i] = M.mean[i];
    s.inv_std[i] = M.inv_std[i];
  }
  if (tid == 0) s.b3 = M.b3[0];
}

// Row `row` of the wave block gets the features f (fp32) normalised and
// rounded to bf16; the padding inputs are zero.
__device__ __forceinline__ void put_row(const MlpLds &s, WaveBufs &wb, int row, const float *f) {
#pragma unroll
  for (int i = 0; i < kF; ++i) wb.X[row * kLdX + i] = f2bf((f[i] - s.mean[i]) * s.inv_std[i]);
#pragma unroll
  for (int i = kF; i < kK1; ++i) wb.X[row * kLdX + i] = 0;
}

// Optional per-row outputs of the forward pass (training): pre-activations
// and activations, row-major [row][128].
struct FwdStash {
  float *a1, *a2;
  uint16_t *h1, *h2;
  int64_t row0;   // global row of the block's first row
  int64_t n_rows; // rows that exist
};

// Forward pass of the wave's 64-row block held in wb.X.  Returns Delta of
// row 4 q + j of M-tile m in d[m][j] on every lane of group q.
template <bool STASH>
__device__ void forward_block(const MlpLds &s, WaveBufs &wb, int lane, float (&d)[4][4], const FwdStash &st) {
  const int r = lane & 15, q = lane >> 4;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  // layer 1: X (64 x 32) . W1^T -> 128, bias, GELU, bf16
  for (int nt = 0; nt < kH / 16; ++nt) {
    v4f acc[4] = {};
#pragma unroll
    for (int kk = 0; kk < kK1; kk += 16)
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m] = mfma_tile(wb.X, kLdX, 16 * m, s.W1, kLdX, 16 * nt, kk, acc[m], lane);
    const int col = 16 * nt + r;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * m + 4 * q + j;
        const float a = acc[m][j] + s.b1[col];
        const uint16_t h = f2bf(gelu(a));
        wb.H1[row * kLdH + col] = h;
        if (STASH && st.row0 + row < st.n_rows) {
          st.a1[(st.row0 + row) * kH + col] = a;
          st.h1[(st.row0 + row) * kH + col] = h;
        }
      }
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  // layer 2 with layer 3 folded into its epilogue
  float part[4][4] = {};
  for (int nt = 0; nt < kH / 16; ++nt) {
    v4f acc[4] = {};
    for (int kk = 0; kk < kH; kk += 16)
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m] = mfma_tile(wb.H1, kLdH, 16 * m, s.W2, kLdH, 16 * nt, kk, acc[m], lane);
    const int col = 16 * nt + r;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * m + 4 * q + j;
        const float a = acc[m][j] + s.b2[col];
        const uint16_t h = f2bf(gelu(a));
        part[m][j] += bf2f(h) * s.w3[col];
        if (STASH && st.row0 + row < st.n_rows) {
          st.a2[(st.row0 + row) * kH + col] = a;
          st.h2[(st.row0 + row) * kH + col] = h;
        }
      }
  }
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) d[m][j] = sum16(part[m][j]) + s.b3;
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
    const float d = mlp_rows<false>(s, X[w], lane, u32x4_t{0u, 0u, 0u, 0u});
    if (in) delta[row] = d;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
}

// ---------------------------------------------------------------- training

// Forward over the batch with every activation stashed, the loss terms and
// dL/dDelta = 2 (Delta - r) / n.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void sa_train_fwd_kernel(MlpDev M, const float *feat, const float *target,
                                                                  int64_t n, TrainBufs T) {
  __shared__ MlpLds s;
  __shared__ WaveBufs wbuf[WAVES];
  const int tid = threadIdx.x, lane = lane_id(), w = tid / 64;
  load_weights(M, s, tid, 64 * WAVES);
  __syncthreads();
  WaveBufs &wb = wbuf[w];
  const int64_t n_blocks = (n + kRows - 1) / kRows;
  for (int64_t blk = (int64_t)blockIdx.x * WAVES + w; blk < n_blocks; blk += (int64_t)gridDim.x * WAVES) {
    const int64_t row = blk * kRows + lane;
    float f[kF];
#pragma unroll
    for (int i = 0; i < kF; ++i) f[i] = row < n ? feat[row * kF + i] : 0.0f;
    put_row(s, wb, lane, f);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    if (row < n)
      for (int i = 0; i < kK1; ++i) T.x[row * kK1 + i] = wb.X[lane * kLdX + i];
    float d[4][4];
    forward_block<true>(s, wb, lane, d, FwdStash{T.a1, T.a2, T.h1, T.h2, blk * kRows, n});
    const int r = lane & 15, q = lane >> 4;
    if (r == 0) {
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t rr = blk * kRows + 16 * m + 4 * q + j;
          if (rr < n) {
            const float e = d[m][j] - target[rr];
            T.delta[rr] = d[m][j];
            T.gdelta[rr] = 2.0f * e / (float)n;
            T.sq[rr] = e * e;
          }
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  }
}

// Pairwise ranking loss, one workgroup per group of `group` consecutive rows
// (one kernel instance's configurations).  z = ln score (feature 22, raw) +
// Delta is the corrected key; every ordered pair (i, j) with y_i < y_j (y the
// measured log runtime) costs softplus(z_i - z_j), and the loss is the mean
// over pairs within each group, averaged over the groups.  dL/dz_i =
// (sum over j after i of sigma(z_i - z_j) - sum over j before i of
// sigma(z_j - z_i)) / (groups x pairs of the group); dL/dDelta = dL/dz.
// Overwrites the squared-error terms the forward kernel left.
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
    T.sq[g0 + i] = l * w;
  }
}

// Per row: dA2 = (dDelta w3) * GELU'(a2), dH1 = dA2 W2 (MFMA), dA1 = dH1 *
// GELU'(a1); dA2, dA1 stored bf16 for the weight-gradient contractions.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void sa_train_bwd_rows_kernel(MlpDev M, int64_t n, TrainBufs T) {
  __shared__ uint16_t W2t[kH * kLdH];  // W2 transposed: W2t[k][n] = W2[n][k]
  __shared__ float w3[kH];
  __shared__ uint16_t G2[WAVES][kRows * kLdH];
  const int tid = threadIdx.x, lane = lane_id(), w = tid / 64;
  for (int i = tid; i < kH * kH; i += 64 * WAVES) {
    const int nn = i / kH, kk = i % kH;
    W2t[kk * kLdH + nn] = M.W2[i];
  }
  for (int i = tid; i < kH; i += 64 * WAVES) w3[i] = bf2f(M.w3[i]);
  __syncthreads();
  uint16_t *g2 = G2[w];
  const int r = lane & 15, q = lane >> 4;
  const int64_t n_blocks = (n + kRows - 1) / kRows;
  for (int64_t blk = (int64_t)blockIdx.x * WAVES + w; blk < n_blocks; blk += (int64_t)gridDim.x * WAVES) {
    const int64_t row = blk * kRows + lane;
    const float gd = row < n ? T.gdelta[row] : 0.0f;
    for (int c = 0; c < kH; ++c) {
      const float a2 = row < n ? T.a2[row * kH + c] : 0.0f;
      const uint16_t g = f2bf(gd * w3[c] * gelu_grad(a2));
      g2[lane * kLdH + c] = g;
      if (row < n) T.ga2[row * kH + c] = g;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    for (int nt = 0; nt < kH / 16; ++nt) {
      v4f acc[4] = {};
      for (int kk = 0; kk < kH; kk += 16)
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[m] = mfma_tile(g2, kLdH, 16 * m, W2t, kLdH, 16 * nt, kk, acc[m], lane);
      const int col = 16 * nt + r;
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t rr = blk * kRows + 16 * m + 4 * q + j;
          if (rr < n) T.ga1[rr * kH + col] = f2bf(acc[m][j] * gelu_grad(T.a1[rr * kH + col]));
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  }
}

// Weight gradients, one workgroup per slab of kSlab rows: the slab's
// contributions to dW2 = dA2^T H1, dW1 = dA1^T X (MFMA over the rows) and to
// the bias / output-layer sums, written as fp32 partials part[slab][...].
constexpr int kSlab = 64;  // one 64-row chunk per workgroup: a 4,096-row step spreads over 64 workgroups
constexpr int kLdT = 64 + 4;  // transposed 64-row chunk, padded

__global__ __launch_bounds__(kMlpThreads) void sa_train_wgrad_kernel(int64_t n, TrainBufs T) {
  __shared__ uint16_t gA2t[kH * kLdT];  // [n][rows of chunk]
  __shared__ uint16_t gA1t[kH * kLdT];
  __shared__ uint16_t H1t[kH * kLdT];   // [k][rows]
  __shared__ uint16_t Xt[kK1 * kLdT];
  const int tid = threadIdx.x, lane = lane_id(), w = tid / 64;
  const int64_t slab = blockIdx.x;
  const int64_t r0 = slab * kSlab;
  float *part = T.part + slab * kPartStride;
  // each wave owns output tiles: dW2 has 64 tiles (8 x 8), dW1 16 (8 x 2)
  v4f accW2[16] = {};
  v4f accW1[4] = {};
  float sums_b1 = 0.f, sums_b2 = 0.f, sums_w3 = 0.f, sum_b3 = 0.f, sum_sq = 0.f;  // thread tid < 128 owns column tid
  for (int64_t c0 = r0; c0 < r0 + kSlab; c0 += 64) {
    __syncthreads();
    for (int i = tid; i < 64 * kH; i += kMlpThreads) {
      const int rr = i / kH, cc = i % kH;
      const int64_t row = c0 + rr;
      const bool in = row < n;
      gA2t[cc * kLdT + rr] = in ? T.ga2[row * kH + cc] : 0;
      gA1t[cc * kLdT + rr] = in ? T.ga1[row * kH + cc] : 0;
      H1t[cc * kLdT + rr] = in ? T.h1[row * kH + cc] : 0;
    }
    for (int i = tid; i < 64 * kK1; i += kMlpThreads) {
      const int rr = i / kK1, cc = i % kK1;
      const int64_t row = c0 + rr;
      Xt[cc * kLdT + rr] = row < n ? T.x[row * kK1 + cc] : 0;
    }
    __syncthreads();
    // dW2[nn][kk] += sum_rows gA2[row][nn] H1[row][kk]: A = gA2t ([nn][rows]), Bt = H1t ([kk][rows])
    for (int t = 0; t < 16; ++t) {
      const int tile = w * 16 + t, mt = tile / 8, nt = tile % 8;
#pragma unroll
      for (int kk = 0; kk < 64; kk += 16) accW2[t] = mfma_tile(gA2t, kLdT, 16 * mt, H1t, kLdT, 16 * nt, kk, accW2[t], lane);
    }
    for (int t = 0; t < 4; ++t) {
      const int tile = w * 4 + t, mt = tile / 2, nt = tile % 2;
#pragma unroll
      for (int kk = 0; kk < 64; kk += 16) accW1[t] = mfma_tile(gA1t, kLdT, 16 * mt, Xt, kLdT, 16 * nt, kk, accW1[t], lane);
    }
    if (tid < kH) {
      for (int rr = 0; rr < 64; ++rr) {
        const int64_t row = c0 + rr;
        if (row >= n) break;
        sums_b1 += bf2f(gA1t[tid * kLdT + rr]);
        sums_b2 += bf2f(gA2t[tid * kLdT + rr]);
        sums_w3 += bf2f(T.h2[row * kH + tid]) * T.gdelta[row];
        if (tid == 0) {
          sum_b3 += T.gdelta[row];
          sum_sq += T.sq[row];
        }
      }
    }
  }
  const int r = lane & 15, q = lane >> 4;
  for (int t = 0; t < 16; ++t) {
    const int tile = w * 16 + t, mt = tile / 8, nt = tile % 8;
#pragma unroll
    for (int j = 0; j < 4; ++j) part[kPartW2 + (16 * mt + 4 * q + j) * kH + 16 * nt + r] = accW2[t][j];
  }
  for (int t = 0; t < 4; ++t) {
    const int tile = w * 4 + t, mt = tile / 2, nt = tile % 2;
#pragma unroll
    for (int j = 0; j < 4; ++j) part[kPartW1 + (16 * mt + 4 * q + j) * kK1 + 16 * nt + r] = accW1[t][j];
  }
  if (tid < kH) {
    part[kPartB1 + tid] = sums_b1;
    part[kPartB2 + tid] = sums_b2;
    part[kPartW3 + tid] = sums_w3;
  }
  if (tid == 0) {
    part[kPartB3] = sum_b3;
    part[kPartLoss] = sum_sq;
  }
  // untouched tail of the partial row
  for (int64_t i = kPartLoss + 1 + tid; i < kPartStride; i += kMlpThreads) part[i] = 0.0f;
}

// Sum the slabs' partials (fixed order: deterministic), then Adam on the fp32
// master weights and the bf16 shadow.  One thread per parameter.
__global__ void sa_train_adam_kernel(TrainState S, MlpDev Mw, const float *part, int64_t n_slabs, AdamArgs h,
                                     float *grad_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kPartStride) return;
  float g = 0.0f;
  for (int64_t s = 0; s < n_slabs; ++s) g += part[s * kPartStride + i];
  if (grad_out) grad_out[i] = i == kPartLoss ? g * h.inv_n : g;
  if (i >= kPartUsed) return;
  const float m = h.beta1 * S.m[i] + (1.0f - h.beta1) * g;
  const float v = h.beta2 * S.v[i] + (1.0f - h.beta2) * g * g;
  S.m[i] = m;
  S.v[i] = v;
  const float mh = m / h.bc1, vh = v / h.bc2;
  const float p = S.master[i] - h.lr * mh / (sqrtf(vh) + h.eps);
  S.master[i] = p;
  uint16_t *W1 = (uint16_t *)Mw.W1, *W2 = (uint16_t *)Mw.W2, *w3 = (uint16_t *)Mw.w3;
  float *b1 = (float *)Mw.b1, *b2 = (float *)Mw.b2, *b3 = (float *)Mw.b3;
  if (i < kPartW1 + kH * kK1 && i >= kPartW1) {
    const int64_t j = i - kPartW1;
    W1[j] = (j % kK1) < kF ? f2bf(p) : 0;  // padding inputs stay zero
    if ((j % kK1) >= kF) S.master[i] = 0.0f;
  } else if (i >= kPartW2 && i < kPartW2 + kH * kH) {
    W2[i - kPartW2] = f2bf(p);
  } else if (i >= kPartW3 && i < kPartW3 + kH) {
    w3[i - kPartW3] = f2bf(p);
  } else if (i >= kPartB1 && i < kPartB1 + kH) {
    b1[i - kPartB1] = p;
  } else if (i >= kPartB2 && i < kPartB2 + kH) {
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

int64_t train_slabs(int64_t n) { return (n + kSlab - 1) / kSlab; }

hipError_t launch_train_step(const MlpDev &M, TrainState S, const float *feat, const float *target, int64_t n,
                             TrainBufs T, AdamArgs h, float *grad_out, int32_t group, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  // Batches of up to 1,024 row blocks run one wave per workgroup, so that
  // their few row blocks spread over as many compute units; larger ones
  // share each workgroup's staged weights among four waves.
  const int64_t n_blocks = (n + kRows - 1) / kRows;
  const bool narrow = n_blocks <= 1024;
  int64_t grid = narrow ? n_blocks : (n_blocks + kMlpWaves - 1) / kMlpWaves;
  if (grid > 4096) grid = 4096;
  if (narrow)
    hipLaunchKernelGGL(sa_train_fwd_kernel<1>, dim3((uint32_t)grid), dim3(64), 0, stream, M, feat, target, n, T);
  else
    hipLaunchKernelGGL(sa_train_fwd_kernel<kMlpWaves>, dim3((uint32_t)grid), dim3(kMlpThreads), 0, stream, M, feat,
                       target, n, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (group > 0) {
    const int64_t groups = n / group;
    hipLaunchKernelGGL(sa_train_rank_kernel, dim3((uint32_t)groups), dim3(256), (size_t)(2 * group) * sizeof(float),
                       stream, feat, target, group, 1.0f / (float)groups, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (narrow)
    hipLaunchKernelGGL(sa_train_bwd_rows_kernel<1>, dim3((uint32_t)grid), dim3(64), 0, stream, M, n, T);
  else
    hipLaunchKernelGGL(sa_train_bwd_rows_kernel<kMlpWaves>, dim3((uint32_t)grid), dim3(kMlpThreads), 0, stream, M, n,
                       T);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t slabs = train_slabs(n);
  hipLaunchKernelGGL(sa_train_wgrad_kernel, dim3((uint32_t)slabs), dim3(kMlpThreads), 0, stream, n, T);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(sa_train_adam_kernel, dim3((uint32_t)((kPartStride + 255) / 256)), dim3(256), 0, stream, S, M,
                     T.part, slabs, h, grad_out);
  return hipGetLastError();
}

}  // namespace sa
