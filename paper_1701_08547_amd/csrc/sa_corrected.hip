// Fused corrected scoring pass on gfx950: per evaluation the occupancy and
// score of the static model (Eqs. 1-6), its 24 features, the learned
// correction Delta (BF16 MFMA), the corrected key z = ln(score) + Delta, and
// per-variant top-k selection on z, in one kernel.
//
// Work decomposition as the tile path of the plain pass (wave-tiles of
// `tile` evaluations, pieces per overlapped segment, fragments merged by
// sa_merge_kernel), with a persistent grid: each workgroup of sixteen waves
// (one per CU: four per SIMD, at most 128 registers each) stages the
// network's weights and the GELU pieces in LDS once, and its waves stride
// over the wave-tiles independently.  A wave evaluates 64 configurations at a
// time (one per lane), writes their normalised inputs to its LDS block and
// runs the forward pass on them; its top-k candidates wait in a 256-key LDS
// buffer.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa_corrected.h"
#include "sa_dev.h"
#include "sa_mlp_dev.h"

namespace sa {
namespace {

constexpr int kCorrWaves = 16;
constexpr int kCorrRT = 2;  // row tiles per pass of the network
constexpr int kCorrCap = 256;  // candidate keys per wave: k <= 64 plus one batch of 64, with room to spare
constexpr int32_t kCorrTileMax = 8192;

template <bool HAS_GRID>
__global__ __launch_bounds__(64 * kCorrWaves) void sa_corrected_kernel(EvalLaunch L, MlpDev M) {
  extern __shared__ __align__(16) uint8_t dyn_lds[];
  __shared__ float tab_rcap[kMaxWB + 1];
  __shared__ uint32_t tab_mwb[kMaxWB + 2];
  __shared__ uint8_t tab_blim[kMaxWB + 2];
  __shared__ MlpLdsT s;
  __shared__ WaveLdsT<kCorrCap> wl[kCorrWaves];
  __shared__ __align__(16) uint16_t X[kCorrWaves][64 * kLdXin];

  const KArch &A = L.arch;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int w = tid / 64;
  build_tables(L, dyn_lds, tab_rcap, tab_mwb, tab_blim, tid, 64 * kCorrWaves);
  load_weights_t(M, s, tid, 64 * kCorrWaves);
  __syncthreads();
  const Tables tb{dyn_lds, tab_rcap};
  const uint8_t *tab_wsimd = dyn_lds + L.tab_wsimd_off;
  const int64_t *seg = L.cfg.seg;
  const int64_t n_evals = L.n_evals;
  const int k = L.k;
  const bool topk = k > 0;
  uint16_t *Xw = X[w];

  Selector sel;
  sel.buf = wl[w].cand;
  for (int64_t wt = (int64_t)blockIdx.x * kCorrWaves + w; wt < L.n_tiles; wt += (int64_t)gridDim.x * kCorrWaves) {
    const int64_t t0 = wt * L.tile;
    const int64_t t1 = (t0 + L.tile < n_evals) ? t0 + L.tile : n_evals;
    int64_t v = find_segment(seg, L.n_var, n_evals, t0, lane);
    int64_t e = t0;
    for (; v < L.n_var && e < t1; ++v) {
      const int64_t s0 = uniform64(clamp_off(seg[v], n_evals));
      const int64_t s1 = uniform64(clamp_off(seg[v + 1], n_evals));
      int64_t pe = s1 > e ? s1 : e;
      pe = pe < t1 ? pe : t1;
      if (pe <= e) continue;

      Piece pc;
      setup_piece<Mode::Model>(L, pc, wl[w], v, s0, lane);
      float f[kMF];
      variant_features(f, L.var.n_fp[v], L.var.n_int[v], L.var.n_ld[v], L.var.n_st[v], L.var.n_br[v],
                       L.var.n_bar[v], L.var.n_reg ? L.var.n_reg[v] : 0, L.var.lds[v], L.var.div[v]);
      // inputs 0..7 are the variant's: one packed slice for the whole piece
      uint32_t xv0[4];
      pack_inputs<4>(s, f, 0, xv0);
      const u32x4_t xv = {xv0[0], xv0[1], xv0[2], xv0[3]};
      sel.count = 0;
      sel.theta = kThetaInit;

      for (int64_t base = e; base < pe; base += 64) {
        if (topk) make_room<kCorrCap>(sel, 64, k, lane);
        const int64_t row = base + lane;
        const bool in = row < pe;
        const int32_t T = in ? L.cfg.block[row] : 1;
        const int32_t U = in ? L.cfg.unroll[row] : 1;
        const int32_t R = in ? L.cfg.regs[row] : 0;
        const int32_t G = (HAS_GRID && in) ? L.cfg.grid[row] : 1;
        const Terms t = eval_terms<HAS_GRID>(A, tb, tab_wsimd, tab_mwb, tab_blim, pc, T, U, R, G, in);
        if (L.occ && in) L.occ[row] = t.W;
        const bool legal = t.B > 0;
        config_features(f, T, U, R, G, HAS_GRID, A.n_cu, t.WB, t.gw, t.gr, t.gs, t.B, t.W, t.Ed, t.F, t.sc);
        put_x_cfg(s, Xw, lane, f);
        wave_lds_sync();
        const float delta = mlp_rows<true, kCorrRT>(s, Xw, lane, xv);
        wave_lds_sync();
        const float z = legal ? f[22] + delta : __builtin_huge_valf();
        if (L.score && in) L.score[row] = z;
        if (topk) {
          const uint32_t kk = order_key(z);
          const bool cand[1] = {legal && (z < __builtin_huge_valf()) && kk <= sel.theta};
          const uint64_t key[1] = {((uint64_t)kk << 32) | (uint32_t)(row - s0)};
          offer<1, kCorrCap>(sel, cand, key);
        }
      }

      if (topk) {
        const uint64_t mine = select_k<kCorrCap>(sel, k, lane);
        if (e == s0 && pe == s1) {
          write_final(mine, k, lane, v, L.topk_idx, L.topk_val, nullptr, s0);
        } else {
          const int64_t slot = 2 * wt + (e == t0 ? 0 : 1);
          if (lane < k) L.frag[slot * k + lane] = mine;
        }
      }
      e = pe;
    }
  }
}

int device_cus() {
  static thread_local int dev_cached = -1, cus = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (dev != dev_cached) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 1;
    cus = c;
    dev_cached = dev;
  }
  return cus;
}

// Workgroups of sa_corrected_kernel<G> one CU holds with `dyn` bytes of
// dynamic LDS.
template <bool G>
int resident_blocks(size_t dyn) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sa_corrected_kernel<G>, 64 * kCorrWaves, dyn) != hipSuccess ||
      nb < 1)
    nb = 1;
  return nb;
}

template <bool G>
hipError_t launch_corrected_one(const EvalLaunch &L, const MlpDev &M, hipStream_t stream) {
  const size_t dyn = (size_t)L.dyn_lds_bytes;
  int64_t grid = (int64_t)resident_blocks<G>(dyn) * device_cus();
  const int64_t need = (L.n_tiles + kCorrWaves - 1) / kCorrWaves;
  if (grid > need) grid = need;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((sa_corrected_kernel<G>), dim3((uint32_t)grid), dim3(64 * kCorrWaves), dyn, stream, L, M);
  return hipGetLastError();
}

}  // namespace

int32_t corrected_tile(int64_t n_evals, int32_t dyn_lds_bytes, bool has_grid) {
  const size_t dyn = (size_t)dyn_lds_bytes;
  const int64_t waves =
      (int64_t)(has_grid ? resident_blocks<true>(dyn) : resident_blocks<false>(dyn)) * device_cus() * kCorrWaves;
  // evaluations of the most loaded wave when the tiles are dealt round-robin
  auto most = [&](int64_t tile) { return (((n_evals + tile - 1) / tile + waves - 1) / waves) * tile; };
  const int64_t base = most(kTileMin);
  int32_t best = kTileMin;
  for (int32_t t = 2 * kTileMin; t <= kCorrTileMax; t *= 2)
    if (most(t) <= base) best = t;
  return best;
}

hipError_t launch_corrected(const EvalLaunch &L, const MlpDev &M, bool has_grid, hipStream_t stream) {
  if (L.n_tiles == 0) return hipSuccess;
  return has_grid ? launch_corrected_one<true>(L, M, stream) : launch_corrected_one<false>(L, M, stream);
}

}  // namespace sa
