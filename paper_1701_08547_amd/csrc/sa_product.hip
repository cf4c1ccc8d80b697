// Scoring over search spaces that are full products of value lists.
//
// When every variant's space is the same product block x unroll x registers
// [x grid] (the autotuner's space of Sec. III-C: each tuning parameter takes
// each of its values), no configuration rows need to exist: evaluation e of
// variant v = e / S has local index i = e - v S, and its values follow from
// i's mixed-radix digits (grid fastest, block slowest).  The pass is then
// bound by the arithmetic, not by reading 16 bytes of rows per evaluation.
// Results are those of sa_score on the materialised rows.  The evaluation
// kernel is the tile path's (Mode::Product): only where a chunk's values come
// from differs.
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
void set_lds_layout(sa::EvalLaunch &L);
size_t frag_bytes(int64_t n_evals, int32_t tile, int32_t k);
sa_status check_variants(const sa_variants *v, int64_t n_var);
sa_status hip_fail(hipError_t e, const char *what);
int32_t tile_override();
}  // namespace sa_detail

namespace sa {
namespace {

__global__ __launch_bounds__(kBlockThreads) void sa_seg_fill_kernel(int64_t *seg, int64_t n_var, int64_t S) {
  for (int64_t v = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x; v <= n_var; v += (int64_t)gridDim.x * kBlockThreads)
    seg[v] = v * S;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Wave-tiles of a product pass: the smallest power-of-two tile (from 1,024)
// that needs no more than 16 wave-tiles per compute unit (four resident
// waves per SIMD): smaller tiles multiply the per-piece selection and merge
// work, larger ones leave SIMDs idle (measured on 1,000 x 16,384: 1,024 ->
// 92 us, 2,048 -> 73, 4,096 -> 65, 8,192 -> 71, 16,384 -> 96).
int32_t product_tile(int64_t n_evals, int32_t n_cu) {
  if (sa_detail::tile_override() > 0) return sa_detail::tile_override();
  const int64_t max_tiles = 16 * (int64_t)(n_cu > 0 ? n_cu : 1);
  int32_t t = kTileMin;
  while (t < kTileMax && (n_evals + t - 1) / t > max_tiles) t *= 2;
  return t;
}

}  // namespace
}  // namespace sa

using namespace sa_detail;

extern "C" {

size_t sa_product_workspace_bytes(int64_t n_variants, int64_t space_size, int32_t k) {
  if (n_variants <= 0 || space_size <= 0 || k <= 0) return 0;
  if (k > SA_K_MAX) k = SA_K_MAX;
  return sa::align256(frag_bytes(n_variants * space_size, sa::kTileMin, k)) +
         sa::align256((size_t)(n_variants + 1) * 8);
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
    if (counts[d] < lo || counts[d] > SA_PRODUCT_MAX_VALUES || counts[d] > sa::kProductMaxValues)
      return fail(SA_ERR_ARG, "value count %d of dimension %d outside [%d, %d]", counts[d], d, lo,
                  SA_PRODUCT_MAX_VALUES);
    if (counts[d] > 0 && !lists[d]) return fail(SA_ERR_ARG, "value list of dimension %d is NULL", d);
    S *= counts[d] > 0 ? counts[d] : 1;
  }
  if (S > SA_PRODUCT_MAX_SIZE) return fail(SA_ERR_ARG, "space of %lld configurations exceeds %d", (long long)S,
                                           SA_PRODUCT_MAX_SIZE);
  if (n_variants == 0) return SA_OK;  // nothing to write (outputs of an empty batch may be NULL)
  const bool topk = topk_idx || topk_val;
  if (topk && (k < 1 || k > SA_K_MAX)) return fail(SA_ERR_ARG, "k = %d outside [1, %d]", k, SA_K_MAX);
  if (!topk && !score && !occ_waves) return fail(SA_ERR_ARG, "no output requested");
  const void *outs[] = {score, occ_waves, topk_idx, topk_val};
  for (const void *p : outs)
    if (p && !aligned(p, 4)) return fail(SA_ERR_ALIGN, "output not 4-byte aligned");

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
  L.tile = sa::product_tile(L.n_evals, L.arch.n_cu);
  L.n_tiles = ceil_div(L.n_evals, L.tile);
  L.need_score = (score || topk) ? 1 : 0;
  L.vec = (aligned(score, 16) && aligned(occ_waves, 16)) ? 1 : 0;  // NULL counts as aligned
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
  hipError_t e = sa::launch_product(L, P, counts[3] > 0, topk, s);
  if (e != hipSuccess) return hip_fail(e, "sa_eval_kernel (product) launch");
  if (topk) {
    e = sa::launch_merge(L, s);
    if (e != hipSuccess) return hip_fail(e, "sa_merge_kernel launch");
  }
  return SA_OK;
}

}  // extern "C"
