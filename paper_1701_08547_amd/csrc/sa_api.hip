// C ABI of the static autotuning model: argument validation, workspace
// sizing and kernel launches.  Every entry point validates before it
// enqueues anything and never allocates, synchronises or copies to the host.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <initializer_list>

#include "sa.h"
#include "sa_internal.h"
#include "sa_corrected.h"

namespace {
thread_local char g_err[512] = "";
thread_local int32_t g_tile = 0;
}  // namespace

namespace sa_detail {

sa_status fail(sa_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int32_t log2_exact(int64_t x) {
  int32_t s = 0;
  while ((int64_t)1 << s < x) ++s;
  return s;
}

sa_status check_arch(const sa_arch *a) {
  if (!a) return fail(SA_ERR_ARG, "arch is NULL");
#define SA_RANGE(f, lo, hi)                                                                          \
  if ((int64_t)a->f < (int64_t)(lo) || (int64_t)a->f > (int64_t)(hi))                                \
    return fail(SA_ERR_UNSUPPORTED, "arch." #f " = %lld outside [%lld, %lld]", (long long)a->f,        \
                (long long)(lo), (long long)(hi));
  SA_RANGE(n_cu, 1, 2048)
  SA_RANGE(wave_size, 2, 1024)
  SA_RANGE(max_threads_per_block, 1, 65536)
  SA_RANGE(max_waves_per_cu, 1, 64)
  SA_RANGE(max_blocks_per_cu, 1, 1 << 20)
  SA_RANGE(single_wave_exempt, 0, 1)
  SA_RANGE(simd_per_cu, 1, a->max_waves_per_cu)
  SA_RANGE(vgprs_per_simd_lane, 1, 65536)
  SA_RANGE(vgpr_granule, 1, 1024)
  SA_RANGE(max_vgprs_per_thread, 0, 65536)
  SA_RANGE(lds_per_cu, 1, 1 << 24)
  SA_RANGE(lds_granule, 1, 1 << 24)
  SA_RANGE(max_lds_per_block, 0, 1 << 24)
  SA_RANGE(w_sat, 1, 4096)
  SA_RANGE(max_unroll, 1, sa::kMaxUnroll)
  SA_RANGE(max_grid, 1, 1 << 18)
#undef SA_RANGE
  if (!pow2(a->wave_size)) return fail(SA_ERR_UNSUPPORTED, "wave_size %d is not a power of two", a->wave_size);
  if (!pow2(a->vgpr_granule)) return fail(SA_ERR_UNSUPPORTED, "vgpr_granule %d is not a power of two", a->vgpr_granule);
  if (!pow2(a->simd_per_cu)) return fail(SA_ERR_UNSUPPORTED, "simd_per_cu %d is not a power of two", a->simd_per_cu);
  if (a->max_threads_per_block % a->wave_size)
    return fail(SA_ERR_UNSUPPORTED, "max_threads_per_block %d is not a multiple of wave_size %d",
                a->max_threads_per_block, a->wave_size);
  if (a->max_vgprs_per_thread % a->vgpr_granule)
    return fail(SA_ERR_UNSUPPORTED, "max_vgprs_per_thread %d is not a multiple of vgpr_granule %d",
                a->max_vgprs_per_thread, a->vgpr_granule);
  const int64_t nw = ceil_div(a->max_threads_per_block, a->wave_size);
  const int64_t nr = ceil_div(a->max_vgprs_per_thread, a->vgpr_granule);
  if (nw > sa::kMaxWB) return fail(SA_ERR_UNSUPPORTED, "ceil(max_threads_per_block / wave_size) = %lld > %d", (long long)nw, sa::kMaxWB);
  if ((nr + 2) * (nw + 2) > sa::kTabBMax)
    return fail(SA_ERR_UNSUPPORTED, "occupancy table (%lld x %lld) exceeds %d entries", (long long)(nr + 2),
                (long long)(nw + 2), sa::kTabBMax);
  const float c[6] = {a->cpi_fp, a->cpi_int, a->cpi_mem, a->cpi_ctrl, a->cpi_sync, a->cpi_reg};
  for (float x : c)
    if (!(x >= 0.0f) || !isfinite(x)) return fail(SA_ERR_UNSUPPORTED, "cpi weights must be finite and >= 0");
  return SA_OK;
}

sa::KArch to_karch(const sa_arch *a) {
  sa::KArch k;
  k.n_cu = a->n_cu;
  k.ws = a->wave_size;
  k.max_threads = a->max_threads_per_block;
  k.max_waves = a->max_waves_per_cu;
  k.max_blocks = a->max_blocks_per_cu;
  k.exempt = a->single_wave_exempt;
  k.simd = a->simd_per_cu;
  k.vgprs = a->vgprs_per_simd_lane;
  k.vgpr_gran = a->vgpr_granule;
  k.max_vgprs = a->max_vgprs_per_thread;
  k.lds_cu = a->lds_per_cu;
  k.lds_gran = a->lds_granule;
  k.max_lds = a->max_lds_per_block;
  k.w_sat = a->w_sat;
  k.max_unroll = a->max_unroll;
  k.max_grid = a->max_grid;
  k.cfp = a->cpi_fp;
  k.cint = a->cpi_int;
  k.cmem = a->cpi_mem;
  k.cctrl = a->cpi_ctrl;
  k.csync = a->cpi_sync;
  k.creg = a->cpi_reg;
  k.nw = (int32_t)ceil_div(a->max_threads_per_block, a->wave_size);
  k.nr = (int32_t)ceil_div(a->max_vgprs_per_thread, a->vgpr_granule);
  k.ws_shift = log2_exact(a->wave_size);
  k.gran_shift = log2_exact(a->vgpr_granule);
  k.simd_shift = log2_exact(a->simd_per_cu);
  return k;
}

int32_t tile_override() { return g_tile; }

int32_t pick_tile(int64_t n_evals) {
  if (g_tile > 0) return g_tile;
  (void)n_evals;
  return sa::kTileDefault;
}

// Dynamic LDS of the evaluation kernel: occupancy table, then the per-granule
// wave counts, each rounded to 16 bytes.
void set_lds_layout(sa::EvalLaunch &L) {
  const int32_t tab = (L.arch.nr + 2) * (L.arch.nw + 2);
  L.tab_wsimd_off = (tab + 15) & ~15;
  L.dyn_lds_bytes = L.tab_wsimd_off + (((L.arch.nr + 2) + 15) & ~15);
}

bool all16(std::initializer_list<const void *> ps) {
  for (const void *p : ps)
    if (p && !aligned(p, 16)) return false;
  return true;
}

size_t frag_bytes(int64_t n_evals, int32_t tile, int32_t k) {
  const int64_t tiles = ceil_div(n_evals, tile);
  return (size_t)(2 * tiles * (int64_t)k * (int64_t)sizeof(uint64_t));
}

// Tile sa_score sizes its workspace for: the plain pass's, or for the
// corrected pass (~100x the work per evaluation) the smallest, which bounds
// the fragment slots of whatever tile its launch then picks.
int32_t score_tile(int64_t n_evals, bool corrected) {
  return corrected ? (g_tile > 0 ? g_tile : sa::kTileMin) : pick_tile(n_evals);
}

// Workspace bytes one sa_score call uses (its fragment slots).
size_t score_workspace_need(int64_t n_evals, int32_t k, bool corrected) {
  if (n_evals <= 0 || k <= 0) return 0;
  return frag_bytes(n_evals, score_tile(n_evals, corrected), k);
}

// Point the launch at its workspace: the fragment slots.
sa_status bind_workspace(sa::EvalLaunch &L, void *workspace, size_t workspace_bytes) {
  const size_t need = frag_bytes(L.n_evals, L.tile, L.k);
  if (need == 0) return SA_OK;
  if (!workspace) return fail(SA_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", need);
  if (!aligned(workspace, 256)) return fail(SA_ERR_ALIGN, "workspace not 256-byte aligned");
  if (workspace_bytes < need) return fail(SA_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace_bytes, need);
  L.frag = (uint64_t *)workspace;
  return SA_OK;
}

sa_status check_mlp(const sa_mlp *m);  // sa_mlp_api.hip
sa::MlpDev mlp_dev(const sa_mlp *m);

sa_status check_variants(const sa_variants *v, int64_t n_var) {
  if (!v) return fail(SA_ERR_ARG, "variants is NULL");
  if (n_var == 0) return SA_OK;
  const void *req[] = {v->n_fp, v->n_int, v->n_ld, v->n_st, v->n_br, v->n_bar, v->lds_bytes, v->div};
  for (const void *p : req) {
    if (!p) return fail(SA_ERR_ARG, "a required variant column is NULL");
    if (!aligned(p, 4)) return fail(SA_ERR_ALIGN, "variant column not 4-byte aligned");
  }
  if (v->n_reg && !aligned(v->n_reg, 4)) return fail(SA_ERR_ALIGN, "n_reg not 4-byte aligned");
  return SA_OK;
}

sa_status check_configs(const sa_configs *c, int64_t n_evals, bool need_cols) {
  if (!c) return fail(SA_ERR_ARG, "configs is NULL");
  if (!c->seg) return fail(SA_ERR_ARG, "configs.seg is NULL");
  if (!aligned(c->seg, 8)) return fail(SA_ERR_ALIGN, "configs.seg not 8-byte aligned");
  if (!need_cols || n_evals == 0) return SA_OK;
  const void *req[] = {c->block, c->unroll, c->regs};
  for (const void *p : req) {
    if (!p) return fail(SA_ERR_ARG, "a required configuration column is NULL");
    if (!aligned(p, 4)) return fail(SA_ERR_ALIGN, "configuration column not 4-byte aligned");
  }
  if (c->grid && !aligned(c->grid, 4)) return fail(SA_ERR_ALIGN, "configs.grid not 4-byte aligned");
  return SA_OK;
}

sa_status check_sizes(int64_t n_var, int64_t n_evals) {
  if (n_var < 0 || n_evals < 0) return fail(SA_ERR_ARG, "negative size (n_variants %lld, n_evals %lld)", (long long)n_var, (long long)n_evals);
  if (n_evals > 0 && n_var == 0) return fail(SA_ERR_ARG, "n_evals > 0 with no variants");
  return SA_OK;
}

sa_status hip_fail(hipError_t e, const char *what) {
  return fail(SA_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace sa_detail

using namespace sa_detail;

extern "C" {

const char *sa_status_string(sa_status s) {
  switch (s) {
    case SA_OK: return "SA_OK";
    case SA_ERR_ARG: return "SA_ERR_ARG";
    case SA_ERR_ALIGN: return "SA_ERR_ALIGN";
    case SA_ERR_NODEV: return "SA_ERR_NODEV";
    case SA_ERR_WORKSPACE: return "SA_ERR_WORKSPACE";
    case SA_ERR_HIP: return "SA_ERR_HIP";
    case SA_ERR_UNSUPPORTED: return "SA_ERR_UNSUPPORTED";
    default: return "SA_ERR_UNKNOWN";
  }
}

const char *sa_last_error(void) { return g_err; }

sa_status sa_arch_gfx950(sa_arch *out) {
  if (!out) return fail(SA_ERR_ARG, "out is NULL");
  out->n_cu = 256;
  out->wave_size = 64;
  out->max_threads_per_block = 1024;
  out->max_waves_per_cu = 32;
  out->max_blocks_per_cu = 16;
  out->single_wave_exempt = 1;
  out->simd_per_cu = 4;
  out->vgprs_per_simd_lane = 512;
  out->vgpr_granule = 8;
  out->max_vgprs_per_thread = 512;
  out->lds_per_cu = 163840;
  out->lds_granule = 1280;
  out->max_lds_per_block = 163840;
  out->w_sat = 32;
  out->max_unroll = 64;
  out->max_grid = 1 << 18;
  out->cpi_fp = 1.0f / 64.0f;
  out->cpi_int = 1.0f / 64.0f;
  out->cpi_mem = 1.0f / 16.0f;
  out->cpi_ctrl = 1.0f / 16.0f;
  out->cpi_sync = 1.0f / 16.0f;
  out->cpi_reg = 1.0f / 32.0f;
  return SA_OK;
}

sa_status sa_arch_default_gfx950(int device, sa_arch *out) {
  if (!out) return fail(SA_ERR_ARG, "out is NULL");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return fail(SA_ERR_NODEV, "no HIP device");
  if (device < 0 || device >= n) return fail(SA_ERR_ARG, "device %d outside [0, %d)", device, n);
  hipDeviceProp_t p;
  hipError_t e = hipGetDeviceProperties(&p, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  sa_arch_gfx950(out);
  if (p.multiProcessorCount > 0) out->n_cu = p.multiProcessorCount;
  if (p.warpSize > 0) out->wave_size = p.warpSize;
  if (p.maxThreadsPerBlock > 0) out->max_threads_per_block = p.maxThreadsPerBlock;
  if (p.maxSharedMemoryPerMultiProcessor > 0) out->lds_per_cu = (int32_t)p.maxSharedMemoryPerMultiProcessor;
  if (p.sharedMemPerBlock > 0) out->max_lds_per_block = (int32_t)p.sharedMemPerBlock;
  return SA_OK;
}

sa_status sa_arch_validate(const sa_arch *arch) { return check_arch(arch); }

size_t sa_workspace_bytes(int64_t n_variants, int64_t n_evals, int32_t k, int32_t flags) {
  (void)flags;
  (void)n_variants;
  if (k <= 0 || n_evals <= 0) return 0;
  if (k > SA_K_MAX) k = SA_K_MAX;
  return frag_bytes(n_evals, sa::kTileMin, k);
}

sa_status sa_set_tile(int32_t evals_per_wave) {
  if (evals_per_wave == 0) {
    g_tile = 0;
    return SA_OK;
  }
  if (evals_per_wave < sa::kTileMin || evals_per_wave > sa::kTileMax || evals_per_wave % (64 * sa::kItems) != 0)
    return fail(SA_ERR_ARG, "tile %d must be a multiple of %d in [%d, %d]", evals_per_wave, 64 * sa::kItems,
                sa::kTileMin, sa::kTileMax);
  g_tile = evals_per_wave;
  return SA_OK;
}

sa_status sa_occupancy(const sa_arch *arch, const sa_variants *variants, const sa_configs *configs,
                       int64_t n_variants, int64_t n_evals, int32_t *occ_waves, void *stream) {
  sa_status st;
  if ((st = check_arch(arch)) != SA_OK) return st;
  if ((st = check_sizes(n_variants, n_evals)) != SA_OK) return st;
  if ((st = check_variants(variants, n_variants)) != SA_OK) return st;
  if ((st = check_configs(configs, n_evals, true)) != SA_OK) return st;
  if (n_evals > 0 && !occ_waves) return fail(SA_ERR_ARG, "occ_waves is NULL");
  if (occ_waves && !aligned(occ_waves, 4)) return fail(SA_ERR_ALIGN, "occ_waves not 4-byte aligned");
  if (n_evals == 0) return SA_OK;
  sa::EvalLaunch L{};
  L.arch = to_karch(arch);
  L.var = {variants->n_fp, variants->n_int, variants->n_ld, variants->n_st, variants->n_br,
           variants->n_bar, variants->n_reg, variants->lds_bytes, variants->div};
  L.cfg = {configs->seg, configs->block, configs->unroll, configs->regs, configs->grid};
  L.n_var = n_variants;
  L.n_evals = n_evals;
  L.occ = occ_waves;
  L.tile = pick_tile(n_evals);
  L.n_tiles = ceil_div(n_evals, L.tile);
  L.need_score = 0;
  L.k = 0;
  L.vec = all16({configs->block, configs->unroll, configs->regs, configs->grid, occ_waves}) ? 1 : 0;
  set_lds_layout(L);
  hipError_t e = sa::launch_eval(L, sa::Mode::Model, configs->grid != nullptr, false, (hipStream_t)stream);
  return e == hipSuccess ? SA_OK : hip_fail(e, "sa_eval_kernel launch");
}

sa_status sa_score(const sa_arch *arch, const sa_variants *variants, const sa_configs *configs,
                   int64_t n_variants, int64_t n_evals, float *score, int32_t *occ_waves, int32_t k,
                   int32_t *topk_idx, float *topk_val, const sa_mlp *mlp, void *workspace,
                   size_t workspace_bytes, void *stream) {
  sa_status st;
  if ((st = check_arch(arch)) != SA_OK) return st;
  if ((st = check_sizes(n_variants, n_evals)) != SA_OK) return st;
  if ((st = check_variants(variants, n_variants)) != SA_OK) return st;
  if ((st = check_configs(configs, n_evals, true)) != SA_OK) return st;
  if (mlp && (st = check_mlp(mlp)) != SA_OK) return st;
  const bool topk = topk_idx || topk_val;
  if (topk && (k < 1 || k > SA_K_MAX)) return fail(SA_ERR_ARG, "k = %d outside [1, %d]", k, SA_K_MAX);
  if (!topk && !score && !occ_waves) return fail(SA_ERR_ARG, "no output requested");
  const void *outs[] = {score, occ_waves, topk_idx, topk_val};
  for (const void *p : outs)
    if (p && !aligned(p, 4)) return fail(SA_ERR_ALIGN, "output not 4-byte aligned");
  sa::EvalLaunch L{};
  L.arch = to_karch(arch);
  L.var = {variants->n_fp, variants->n_int, variants->n_ld, variants->n_st, variants->n_br,
           variants->n_bar, variants->n_reg, variants->lds_bytes, variants->div};
  L.cfg = {configs->seg, configs->block, configs->unroll, configs->regs, configs->grid};
  L.n_var = n_variants;
  L.n_evals = n_evals;
  L.occ = occ_waves;
  L.score = score;
  L.topk_idx = topk_idx;
  L.topk_val = topk_val;
  L.k = topk ? k : 0;
  L.need_score = (score || topk) ? 1 : 0;
  L.vec = all16({configs->block, configs->unroll, configs->regs, configs->grid, occ_waves, score}) ? 1 : 0;
  set_lds_layout(L);
  L.tile = (mlp && g_tile <= 0) ? sa::corrected_tile(n_evals, L.dyn_lds_bytes, configs->grid != nullptr)
                                : score_tile(n_evals, mlp != nullptr);
  L.n_tiles = ceil_div(n_evals, L.tile);
  if (topk && n_variants > 0) {
    if ((st = bind_workspace(L, workspace, workspace_bytes)) != SA_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  if (n_evals > 0) {
    hipError_t e = mlp ? sa::launch_corrected(L, mlp_dev(mlp), configs->grid != nullptr, s)
                       : sa::launch_eval(L, sa::Mode::Model, configs->grid != nullptr, topk, s);
    if (e != hipSuccess) return hip_fail(e, mlp ? "sa_corrected_kernel launch" : "sa_eval_kernel launch");
  }
  if (topk && n_variants > 0) {
    hipError_t e = sa::launch_merge(L, s);
    if (e != hipSuccess) return hip_fail(e, "sa_merge_kernel launch");
  }
  return SA_OK;
}

sa_status sa_suggest(const sa_arch *arch, const sa_variants *variants, int64_t n_variants, uint64_t *kept,
                     void *stream) {
  sa_status st;
  if ((st = check_arch(arch)) != SA_OK) return st;
  if (n_variants < 0) return fail(SA_ERR_ARG, "negative n_variants");
  if (n_variants == 0) return SA_OK;
  if ((st = check_variants(variants, n_variants)) != SA_OK) return st;
  if (!kept) return fail(SA_ERR_ARG, "kept is NULL");
  if (!aligned(kept, 8)) return fail(SA_ERR_ALIGN, "kept not 8-byte aligned");
  sa::EvalLaunch L{};
  L.arch = to_karch(arch);
  L.var = {variants->n_fp, variants->n_int, variants->n_ld, variants->n_st, variants->n_br,
           variants->n_bar, variants->n_reg, variants->lds_bytes, variants->div};
  L.n_var = n_variants;
  set_lds_layout(L);
  hipError_t e = sa::launch_suggest(L, kept, (hipStream_t)stream);
  return e == hipSuccess ? SA_OK : hip_fail(e, "sa_suggest_kernel launch");
}

sa_status sa_headroom(const sa_arch *arch, const int32_t *block, const int32_t *regs, int64_t n, int32_t *r_star,
                      int32_t *s_star, void *stream) {
  sa_status st;
  if ((st = check_arch(arch)) != SA_OK) return st;
  if (n < 0) return fail(SA_ERR_ARG, "negative n");
  if (n == 0) return SA_OK;
  if (!block) return fail(SA_ERR_ARG, "block is NULL");
  if (!r_star && !s_star) return fail(SA_ERR_ARG, "no output");
  const void *ps[] = {block, regs, r_star, s_star};
  for (const void *p : ps)
    if (p && !aligned(p, 4)) return fail(SA_ERR_ALIGN, "array not 4-byte aligned");
  sa::EvalLaunch L{};
  L.arch = to_karch(arch);
  set_lds_layout(L);
  hipError_t e = sa::launch_headroom(L, block, regs, n, r_star, s_star, (hipStream_t)stream);
  return e == hipSuccess ? SA_OK : hip_fail(e, "sa_headroom_kernel launch");
}

sa_status sa_score_suggested(const sa_arch *arch, const sa_variants *variants, const sa_configs *configs,
                             int64_t n_variants, int64_t n_evals, float *score, int32_t *occ_waves, int32_t k,
                             int32_t *topk_idx, float *topk_val, void *workspace, size_t workspace_bytes,
                             void *stream) {
  sa_status st;
  if ((st = check_arch(arch)) != SA_OK) return st;
  if ((st = check_sizes(n_variants, n_evals)) != SA_OK) return st;
  if ((st = check_variants(variants, n_variants)) != SA_OK) return st;
  if ((st = check_configs(configs, n_evals, true)) != SA_OK) return st;
  if (!topk_idx && !topk_val) return fail(SA_ERR_ARG, "no top-k output");
  if (k < 1 || k > SA_K_MAX) return fail(SA_ERR_ARG, "k = %d outside [1, %d]", k, SA_K_MAX);
  const void *outs[] = {score, occ_waves, topk_idx, topk_val};
  for (const void *p : outs)
    if (p && !aligned(p, 4)) return fail(SA_ERR_ALIGN, "output not 4-byte aligned");
  sa::EvalLaunch L{};
  L.arch = to_karch(arch);
  L.var = {variants->n_fp, variants->n_int, variants->n_ld, variants->n_st, variants->n_br,
           variants->n_bar, variants->n_reg, variants->lds_bytes, variants->div};
  L.cfg = {configs->seg, configs->block, configs->unroll, configs->regs, configs->grid};
  L.n_var = n_variants;
  L.n_evals = n_evals;
  L.occ = occ_waves;
  L.score = score;
  L.topk_idx = topk_idx;
  L.topk_val = topk_val;
  L.k = k;
  L.tile = pick_tile(n_evals);
  L.n_tiles = ceil_div(n_evals, L.tile);
  L.need_score = 1;
  L.vec = all16({configs->block, configs->unroll, configs->regs, configs->grid, occ_waves, score}) ? 1 : 0;
  set_lds_layout(L);
  if (n_variants > 0) {
    if ((st = bind_workspace(L, workspace, workspace_bytes)) != SA_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  if (n_evals > 0) {
    hipError_t e = sa::launch_eval(L, sa::Mode::Suggest, configs->grid != nullptr, true, s);
    if (e != hipSuccess) return hip_fail(e, "sa_eval_kernel launch");
  }
  if (n_variants > 0) {
    hipError_t e = sa::launch_merge(L, s);
    if (e != hipSuccess) return hip_fail(e, "sa_merge_kernel launch");
  }
  return SA_OK;
}

sa_status sa_topk(const float *keys, const int64_t *seg, int64_t n_variants, int64_t n_evals, int32_t k,
                  int32_t *idx, float *val, void *workspace, size_t workspace_bytes, void *stream) {
  sa_status st;
  if ((st = check_sizes(n_variants, n_evals)) != SA_OK) return st;
  if (k < 1 || k > SA_K_MAX) return fail(SA_ERR_ARG, "k = %d outside [1, %d]", k, SA_K_MAX);
  if (!seg) return fail(SA_ERR_ARG, "seg is NULL");
  if (!aligned(seg, 8)) return fail(SA_ERR_ALIGN, "seg not 8-byte aligned");
  if (n_evals > 0 && !keys) return fail(SA_ERR_ARG, "keys is NULL");
  if (keys && !aligned(keys, 4)) return fail(SA_ERR_ALIGN, "keys not 4-byte aligned");
  if (n_variants > 0 && !idx) return fail(SA_ERR_ARG, "idx is NULL");
  if ((idx && !aligned(idx, 4)) || (val && !aligned(val, 4))) return fail(SA_ERR_ALIGN, "output not 4-byte aligned");
  sa::EvalLaunch L{};
  L.cfg.seg = seg;
  L.keys = keys;
  L.n_var = n_variants;
  L.n_evals = n_evals;
  L.topk_idx = idx;
  L.topk_val = val;
  L.k = k;
  L.tile = pick_tile(n_evals);
  L.n_tiles = ceil_div(n_evals, L.tile);
  L.vec = all16({keys}) ? 1 : 0;
  if (n_variants > 0) {
    if ((st = bind_workspace(L, workspace, workspace_bytes)) != SA_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  if (n_evals > 0) {
    hipError_t e = sa::launch_eval(L, sa::Mode::Keys, false, true, s);
    if (e != hipSuccess) return hip_fail(e, "sa_eval_kernel launch");
  }
  if (n_variants > 0) {
    hipError_t e = sa::launch_merge(L, s);
    if (e != hipSuccess) return hip_fail(e, "sa_merge_kernel launch");
  }
  return SA_OK;
}

}  // extern "C"
