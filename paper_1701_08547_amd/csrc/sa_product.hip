// Scoring over search spaces that are full products of value lists.
//
// When every variant's space is the same product block x unroll x registers
// [x grid] (the autotuner's space of Sec. III-C: each tuning parameter takes
// each of its values), no configuration rows need to exist: evaluation e of
// variant v = e / S has local index i = e - v S, and its values follow from
// i's mixed-radix digits (grid fastest, block slowest).  The pass is then
// bound by the arithmetic, not by reading 16 bytes of rows per evaluation.
// Results are those of sa_score on the materialised rows.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa.h"
#include "sa_dev.h"

namespace sa_detail {
sa_status fail(sa_status st, const char *fmt, ...);
bool aligned(const void *p, size_t a);
int64_t ceil_div(int64_t a, int64_t b);
sa_status check_arch(const sa_arch *a);
sa::KArch to_karch(const sa_arch *a);
int32_t pick_tile(int64_t n_evals);
void set_lds_layout(sa::EvalLaunch &L);
size_t frag_bytes(int64_t n_evals, int32_t tile, int32_t k);
sa_status check_variants(const sa_variants *v, int64_t n_var);
sa_status hip_fail(hipError_t e, const char *what);
}  // namespace sa_detail

namespace sa {
namespace {

constexpr int kItems = 4;  // evaluations per lane per chunk

struct KProduct {
  int32_t n[4];       // values of block, unroll, registers, grid (1 without a grid column)
  uint32_t magic[3];  // ceil(2^32 / n) for grid, registers, unroll; 0 when n = 1
  int32_t size;       // n[0] n[1] n[2] n[3]
  int32_t vals[4][SA_PRODUCT_MAX_VALUES];
};

// floor(x / n) for x < 2^24 and 2 <= n <= 256 from m = ceil(2^32 / n): with
// m n = 2^32 + r (0 <= r < n) and x = q n + t, x m / 2^32 = q + t / n +
// x r / (n 2^32) < q + (n - 1) / n + 1 / n.  m = 0 stands for n = 1.
__device__ __forceinline__ uint32_t div_small(uint32_t x, uint32_t m) { return m ? __umulhi(x, m) : x; }

__global__ __launch_bounds__(kBlockThreads) void sa_seg_fill_kernel(int64_t *seg, int64_t n_var, int64_t S) {
  for (int64_t v = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x; v <= n_var; v += (int64_t)gridDim.x * kBlockThreads)
    seg[v] = v * S;
}

template <bool HAS_GRID, bool TOPK>
__global__ __launch_bounds__(kBlockThreads) void sa_product_kernel(EvalLaunch L, KProduct P) {
  extern __shared__ __align__(16) uint8_t dyn_lds[];
  __shared__ float tab_rcap[kMaxWB + 1];
  __shared__ uint32_t tab_mwb[kMaxWB + 2];
  __shared__ uint8_t tab_blim[kMaxWB + 2];
  __shared__ WaveLds wl[kWavesPerBlock];
  __shared__ int32_t pv[4][SA_PRODUCT_MAX_VALUES];

  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int w = tid / kWaveSize;
  for (int i = tid; i < 4 * SA_PRODUCT_MAX_VALUES; i += kBlockThreads)
    pv[i / SA_PRODUCT_MAX_VALUES][i % SA_PRODUCT_MAX_VALUES] = P.vals[i / SA_PRODUCT_MAX_VALUES][i % SA_PRODUCT_MAX_VALUES];
  build_tables(L, dyn_lds, tab_rcap, tab_mwb, tab_blim, tid, kBlockThreads);  // ends with a barrier

  const int64_t wt = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wt >= L.n_tiles) return;
  const KArch &A = L.arch;
  const Tables tb{dyn_lds, tab_rcap};
  const int64_t S = P.size;
  const int64_t t0 = wt * L.tile;
  const int64_t t1 = (t0 + L.tile < L.n_evals) ? t0 + L.tile : L.n_evals;
  const int32_t nG = P.n[3], nR = P.n[2], nU = P.n[1];

  Selector sel;
  sel.buf = wl[w].cand;
  sel.count = 0;
  sel.theta = kThetaInit;
  int64_t e = t0;
  for (int64_t v = t0 / S; v < L.n_var && e < t1; ++v) {
    const int64_t s0 = v * S, s1 = s0 + S;
    const int64_t pe = s1 < t1 ? s1 : t1;
    Piece pc;
    setup_piece<Mode::Model>(L, pc, wl[w], v, s0, lane);
    if constexpr (TOPK) {
      sel.count = 0;
      sel.theta = kThetaInit;
    }
    for (int64_t base = e; base < pe; base += 64 * kItems) {
      if constexpr (TOPK) make_room(sel, 64 * kItems, L.k, lane);
      bool cand[kItems];
      uint64_t key[kItems];
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        const int64_t row = base + 64 * i + lane;
        const bool in = row < pe;
        // local index below S <= 2^24 for every row in the segment
        const uint32_t li = in ? (uint32_t)(row - s0) : 0u;
        const uint32_t q1 = div_small(li, P.magic[0]);
        const uint32_t q2 = div_small(q1, P.magic[1]);
        const uint32_t iT = div_small(q2, P.magic[2]);
        const int32_t T = pv[0][iT];
        const int32_t U = pv[1][q2 - iT * (uint32_t)nU];
        const int32_t R = pv[2][q1 - q2 * (uint32_t)nR];
        const int32_t G = HAS_GRID ? pv[3][li - q1 * (uint32_t)nG] : 1;
        int32_t W;
        float sc;
        eval_cfg<HAS_GRID>(A, tb, pc, T, U, R, G, in, L.need_score, W, sc);
        if (L.occ && in) L.occ[row] = W;
        if (L.score && in) L.score[row] = sc;
        // model scores are +0 .. +inf: the key is the bit pattern with the
        // sign bit set, and +inf's key lies above every threshold
        const uint32_t kk = __float_as_uint(sc) | 0x80000000u;
        cand[i] = kk <= sel.theta;
        key[i] = ((uint64_t)kk << 32) | li;
      }
      if constexpr (TOPK) offer<kItems>(sel, cand, key);
    }
    if constexpr (TOPK) {
      const uint64_t mine = select_k(sel, L.k, lane);
      if (e == s0 && pe == s1) {
        write_final(mine, L.k, lane, v, L.topk_idx, L.topk_val, nullptr, s0);
      } else {
        const int64_t slot = 2 * wt + (e == t0 ? 0 : 1);
        if (lane < L.k) L.frag[slot * L.k + lane] = mine;
      }
    }
    e = pe;
  }
}

template <bool G, bool K>
hipError_t launch_one(const EvalLaunch &L, const KProduct &P, hipStream_t s) {
  const int64_t blocks = (L.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL((sa_product_kernel<G, K>), dim3((uint32_t)blocks), dim3(kBlockThreads), (size_t)L.dyn_lds_bytes,
                     s, L, P);
  return hipGetLastError();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace sa

using namespace sa_detail;

extern "C" {

size_t sa_product_workspace_bytes(int64_t n_variants, int64_t space_size, int32_t k) {
  if (n_variants <= 0 || space_size <= 0 || k <= 0) return 0;
  if (k > SA_K_MAX) k = SA_K_MAX;
  return sa::align256(frag_bytes(n_variants * space_size, sa::kTileMin, k)) + sa::align256((size_t)(n_variants + 1) * 8);
}

sa_status sa_score_product(const sa_arch *arch, const sa_variants *variants, int64_t n_variants,
                           const sa_product *space, float *score, int32_t *occ_waves, int32_t k, int32_t *topk_idx,
                           float *topk_val, void *workspace, size_t workspace_bytes, void *stream) {
  sa_status st;
  if ((st = check_arch(arch)) != SA_OK) return st;
  if (n_variants < 0) return fail(SA_ERR_ARG, "negative n_variants");
  if ((st = check_variants(variants, n_variants)) != SA_OK) return st;
  if (!space) return fail(SA_ERR_ARG, "space is NULL");
  const int32_t counts[4] = {space->n_block, space->n_unroll, space->n_regs, space->n_grid};
  const int32_t *lists[4] = {space->block, space->unroll, space->regs, space->grid};
  int64_t S = 1;
  for (int d = 0; d < 4; ++d) {
    const int32_t lo = d == 3 ? 0 : 1;
    if (counts[d] < lo || counts[d] > SA_PRODUCT_MAX_VALUES)
      return fail(SA_ERR_ARG, "value count %d of dimension %d outside [%d, %d]", counts[d], d, lo,
                  SA_PRODUCT_MAX_VALUES);
    if (counts[d] > 0 && !lists[d]) return fail(SA_ERR_ARG, "value list of dimension %d is NULL", d);
    S *= counts[d] > 0 ? counts[d] : 1;
  }
  if (S > SA_PRODUCT_MAX_SIZE) return fail(SA_ERR_ARG, "space of %lld configurations exceeds %d", (long long)S,
                                           SA_PRODUCT_MAX_SIZE);
  const bool topk = topk_idx || topk_val;
  if (topk && (k < 1 || k > SA_K_MAX)) return fail(SA_ERR_ARG, "k = %d outside [1, %d]", k, SA_K_MAX);
  if (!topk && !score && !occ_waves) return fail(SA_ERR_ARG, "no output requested");
  const void *outs[] = {score, occ_waves, topk_idx, topk_val};
  for (const void *p : outs)
    if (p && !aligned(p, 4)) return fail(SA_ERR_ALIGN, "output not 4-byte aligned");
  if (n_variants == 0) return SA_OK;

  sa::KProduct P{};
  for (int d = 0; d < 4; ++d) {
    const int32_t n = counts[d] > 0 ? counts[d] : 1;
    P.n[d] = n;
    for (int i = 0; i < counts[d]; ++i) P.vals[d][i] = lists[d][i];
    if (counts[d] == 0) P.vals[d][0] = 1;
  }
  P.magic[0] = P.n[3] > 1 ? (uint32_t)((((uint64_t)1 << 32) + P.n[3] - 1) / P.n[3]) : 0u;
  P.magic[1] = P.n[2] > 1 ? (uint32_t)((((uint64_t)1 << 32) + P.n[2] - 1) / P.n[2]) : 0u;
  P.magic[2] = P.n[1] > 1 ? (uint32_t)((((uint64_t)1 << 32) + P.n[1] - 1) / P.n[1]) : 0u;
  P.size = (int32_t)S;

  sa::EvalLaunch L{};
  L.arch = to_karch(arch);
  L.var = {variants->n_fp, variants->n_int, variants->n_ld, variants->n_st, variants->n_br,
           variants->n_bar, variants->n_reg, variants->lds_bytes, variants->div};
  L.n_var = n_variants;
  L.n_evals = n_variants * S;
  L.occ = occ_waves;
  L.score = score;
  L.topk_idx = topk_idx;
  L.topk_val = topk_val;
  L.k = topk ? k : 0;
  L.tile = pick_tile(L.n_evals);
  L.n_tiles = ceil_div(L.n_evals, L.tile);
  L.need_score = (score || topk) ? 1 : 0;
  set_lds_layout(L);
  hipStream_t s = (hipStream_t)stream;
  int64_t *seg = nullptr;
  if (topk) {
    const size_t fb = sa::align256(frag_bytes(L.n_evals, L.tile, L.k));
    const size_t need = fb + sa::align256((size_t)(n_variants + 1) * 8);
    if (!workspace) return fail(SA_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", need);
    if (!aligned(workspace, 256)) return fail(SA_ERR_ALIGN, "workspace not 256-byte aligned");
    if (workspace_bytes < need) return fail(SA_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace_bytes, need);
    L.frag = (uint64_t *)workspace;
    seg = (int64_t *)((uint8_t *)workspace + fb);
    L.cfg.seg = seg;
    int64_t blocks = (n_variants + 1 + sa::kBlockThreads - 1) / sa::kBlockThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(sa::sa_seg_fill_kernel, dim3((uint32_t)blocks), dim3(sa::kBlockThreads), 0, s, seg, n_variants, S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "sa_seg_fill_kernel launch");
  }
  const bool grid = counts[3] > 0;
  hipError_t e = grid ? (topk ? sa::launch_one<true, true>(L, P, s) : sa::launch_one<true, false>(L, P, s))
                      : (topk ? sa::launch_one<false, true>(L, P, s) : sa::launch_one<false, false>(L, P, s));
  if (e != hipSuccess) return hip_fail(e, "sa_product_kernel launch");
  if (topk) {
    e = sa::launch_merge(L, s);
    if (e != hipSuccess) return hip_fail(e, "sa_merge_kernel launch");
  }
  return SA_OK;
}

}  // extern "C"
