// Plans for batches of uneven search spaces: a host-side decomposition of a
// CSR layout into workgroup items for the persistent kernel, the launch
// shape autotuner, and their C-ABI entry points.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "sa.h"
#include "sa_internal.h"

// Defined in sa_api.hip.
namespace sa_detail {
sa_status fail(sa_status st, const char *fmt, ...);
sa_status check_arch(const sa_arch *a);
sa::KArch to_karch(const sa_arch *a);
void set_lds_layout(sa::EvalLaunch &L);
bool all16(std::initializer_list<const void *> ps);
sa_status hip_fail(hipError_t e, const char *what);
}  // namespace sa_detail

using sa_detail::fail;
using sa_detail::hip_fail;

struct sa_plan {
  int64_t n_var = 0, n_evals = 0;
  int32_t k = 0;
  sa::PlanShape shape{};
  int64_t n_items = 0, n_splits = 0, n_slots = 0;
  void *dev = nullptr;
  sa::PlanDev pd{};
  int device = 0;
  int n_cu = 0;
};

namespace {

bool shape_ok(const sa::PlanShape &s) {
  const bool items = s.items == 1 || s.items == 2 || s.items == 4;
  const bool wpb = s.wpb == 4 || s.wpb == 8 || s.wpb == 16;
  return items && wpb && s.tile >= 256 && s.tile <= (1 << 20) && s.tile % 256 == 0;
}

// Host decomposition.  Segments longer than `tile` become kind-1 items of up
// to tile x wpb evaluations each (one part per wave); shorter ones are packed,
// whole, into kind-0 items of up to tile x wpb evaluations, spread over the
// waves by cumulative cost (evaluations + a fixed per-segment charge).
void decompose(const int64_t *seg, int64_t n_var, const sa::PlanShape &S, std::vector<sa::PlanItem> &items,
               std::vector<sa::PlanWave> &waves, std::vector<sa::PlanSplit> &splits, int64_t &n_slots) {
  const int64_t tile = S.tile, wpb = S.wpb, cap = tile * wpb;
  const int64_t kSegCharge = 256;
  n_slots = 0;
  int64_t i = 0;
  while (i < n_var) {
    const int64_t n_i = seg[i + 1] - seg[i];
    if (n_i > tile) {
      const int64_t m = (n_i + cap - 1) / cap;
      if (m > 1) splits.push_back(sa::PlanSplit{i, n_slots, m, 0});
      for (int64_t j = 0; j < m; ++j) {
        const int64_t a = seg[i] + n_i * j / m, b = seg[i] + n_i * (j + 1) / m;
        items.push_back(sa::PlanItem{1, m > 1 ? (int32_t)(n_slots + j) : -1, i});
        for (int64_t w = 0; w < wpb; ++w) {
          const int64_t e0 = a + (b - a) * w / wpb, e1 = a + (b - a) * (w + 1) / wpb;
          waves.push_back(sa::PlanWave{e0, e1, i, i + 1});
        }
      }
      if (m > 1) n_slots += m;
      ++i;
      continue;
    }
    int64_t j = i, total = 0, cost = 0;
    while (j < n_var) {
      const int64_t n_j = seg[j + 1] - seg[j];
      if (n_j > tile || total + n_j > cap) break;
      total += n_j;
      cost += n_j + kSegCharge;
      ++j;
    }
    items.push_back(sa::PlanItem{0, -1, i});
    int64_t acc = 0, v = i;
    for (int64_t w = 0; w < wpb; ++w) {
      const int64_t v0 = v;
      const int64_t goal = cost * (w + 1) / wpb;
      while (v < j && (w == wpb - 1 || acc + (seg[v + 1] - seg[v]) + kSegCharge / 2 <= goal)) {
        acc += seg[v + 1] - seg[v] + kSegCharge;
        ++v;
      }
      waves.push_back(sa::PlanWave{0, 0, v0, v});
    }
    i = j;
  }
}

sa_status plan_launch(const sa_plan *plan, sa::EvalLaunch &L, sa::Mode mode, bool has_grid, bool topk, void *workspace,
                      size_t workspace_bytes, hipStream_t stream) {
  L.k = topk ? plan->k : 0;
  if (topk) {
    const size_t need = (size_t)plan->n_slots * (size_t)plan->k * sizeof(uint64_t);
    if (need > 0) {
      if (!workspace) return fail(SA_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", need);
      if ((uintptr_t)workspace % 256) return fail(SA_ERR_ALIGN, "workspace not 256-byte aligned");
      if (workspace_bytes < need) return fail(SA_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace_bytes, need);
    }
    L.frag = (uint64_t *)workspace;
  }
  hipError_t e = sa::launch_plan(L, plan->pd, plan->shape, mode, has_grid, topk, plan->n_cu, stream);
  if (e != hipSuccess) return hip_fail(e, "sa_plan_kernel launch");
  if (topk && plan->n_splits > 0) {
    e = sa::launch_split_merge(L, plan->pd, stream);
    if (e != hipSuccess) return hip_fail(e, "sa_split_merge_kernel launch");
  }
  return SA_OK;
}

}  // namespace

extern "C" {

sa_status sa_plan_layout(const int64_t *seg_host, int64_t n_variants, int64_t n_evals, const sa_plan_shape *shape,
                         int64_t *n_items, int64_t *n_splits, int64_t *n_slots, int64_t *items, int64_t *waves,
                         int64_t *splits) {
  if (n_variants < 0 || n_evals < 0 || !seg_host) return fail(SA_ERR_ARG, "bad sizes or NULL seg_host");
  if (seg_host[0] != 0 || seg_host[n_variants] != n_evals)
    return fail(SA_ERR_ARG, "seg[0] must be 0 and seg[n_variants] must equal n_evals");
  for (int64_t v = 0; v < n_variants; ++v)
    if (seg_host[v + 1] < seg_host[v]) return fail(SA_ERR_ARG, "seg decreases at variant %lld", (long long)v);
  sa::PlanShape S{4096, 4, 4};
  if (shape) S = sa::PlanShape{shape->tile, shape->items_per_lane, shape->waves_per_block};
  if (!shape_ok(S)) return fail(SA_ERR_ARG, "plan shape outside the supported set");
  std::vector<sa::PlanItem> it;
  std::vector<sa::PlanWave> wv;
  std::vector<sa::PlanSplit> sp;
  int64_t slots = 0;
  decompose(seg_host, n_variants, S, it, wv, sp, slots);
  if (n_items) *n_items = (int64_t)it.size();
  if (n_splits) *n_splits = (int64_t)sp.size();
  if (n_slots) *n_slots = slots;
  if (items)
    for (size_t i = 0; i < it.size(); ++i) {
      items[3 * i] = it[i].kind;
      items[3 * i + 1] = it[i].slot;
      items[3 * i + 2] = it[i].v;
    }
  if (waves)
    for (size_t i = 0; i < wv.size(); ++i) {
      waves[4 * i] = wv[i].e0;
      waves[4 * i + 1] = wv[i].e1;
      waves[4 * i + 2] = wv[i].v0;
      waves[4 * i + 3] = wv[i].v1;
    }
  if (splits)
    for (size_t i = 0; i < sp.size(); ++i) {
      splits[3 * i] = sp[i].v;
      splits[3 * i + 1] = sp[i].first_slot;
      splits[3 * i + 2] = sp[i].n_slots;
    }
  return SA_OK;
}

sa_status sa_plan_create(const int64_t *seg_host, int64_t n_variants, int64_t n_evals, int32_t k,
                         const sa_plan_shape *shape, sa_plan **out) {
  if (!out) return fail(SA_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n_variants < 0 || n_evals < 0) return fail(SA_ERR_ARG, "negative size");
  if (!seg_host) return fail(SA_ERR_ARG, "seg_host is NULL");
  if (k < 0 || k > SA_K_MAX) return fail(SA_ERR_ARG, "k = %d outside [0, %d]", k, SA_K_MAX);
  if (n_variants > INT32_MAX) return fail(SA_ERR_UNSUPPORTED, "more than 2^31 variants");
  if (seg_host[0] != 0 || seg_host[n_variants] != n_evals)
    return fail(SA_ERR_ARG, "seg[0] must be 0 and seg[n_variants] must equal n_evals");
  for (int64_t v = 0; v < n_variants; ++v)
    if (seg_host[v + 1] < seg_host[v]) return fail(SA_ERR_ARG, "seg decreases at variant %lld", (long long)v);
  sa::PlanShape S{4096, 4, 4};
  if (shape) S = sa::PlanShape{shape->tile, shape->items_per_lane, shape->waves_per_block};
  if (!shape_ok(S))
    return fail(SA_ERR_ARG, "plan shape (tile %d, items %d, waves %d) outside {256k} x {1,2,4} x {4,8,16}", S.tile,
                S.items, S.wpb);
  int dev = 0, n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev == 0) return fail(SA_ERR_NODEV, "no HIP device");
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");

  std::vector<sa::PlanItem> items;
  std::vector<sa::PlanWave> waves;
  std::vector<sa::PlanSplit> splits;
  int64_t n_slots = 0;
  decompose(seg_host, n_variants, S, items, waves, splits, n_slots);

  const size_t bi = items.size() * sizeof(sa::PlanItem), bw = waves.size() * sizeof(sa::PlanWave),
               bs = splits.size() * sizeof(sa::PlanSplit);
  const size_t oi = 0, ow = (bi + 255) / 256 * 256, os = ow + (bw + 255) / 256 * 256;
  const size_t total = os + bs + 256;
  sa_plan *p = new sa_plan();
  p->n_var = n_variants;
  p->n_evals = n_evals;
  p->k = k;
  p->shape = S;
  p->n_items = (int64_t)items.size();
  p->n_splits = (int64_t)splits.size();
  p->n_slots = n_slots;
  p->device = dev;
  p->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
  e = hipMalloc(&p->dev, total);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipMalloc (plan)");
  }
  char *base = (char *)p->dev;
  if ((e = hipMemcpy(base + oi, items.data(), bi, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(base + ow, waves.data(), bw, hipMemcpyHostToDevice)) != hipSuccess ||
      (bs && (e = hipMemcpy(base + os, splits.data(), bs, hipMemcpyHostToDevice)) != hipSuccess)) {
    (void)hipFree(p->dev);
    delete p;
    return hip_fail(e, "hipMemcpy (plan)");
  }
  p->pd.items = (const sa::PlanItem *)(base + oi);
  p->pd.waves = (const sa::PlanWave *)(base + ow);
  p->pd.splits = (const sa::PlanSplit *)(base + os);
  p->pd.n_items = p->n_items;
  p->pd.n_splits = p->n_splits;
  *out = p;
  return SA_OK;
}

sa_status sa_plan_destroy(sa_plan *plan) {
  if (!plan) return SA_OK;
  hipError_t e = plan->dev ? hipFree(plan->dev) : hipSuccess;
  delete plan;
  return e == hipSuccess ? SA_OK : hip_fail(e, "hipFree (plan)");
}

sa_status sa_plan_info(const sa_plan *plan, sa_plan_shape *shape, int64_t *n_items, int64_t *n_splits,
                       size_t *workspace_bytes) {
  if (!plan) return fail(SA_ERR_ARG, "plan is NULL");
  if (shape) *shape = sa_plan_shape{plan->shape.tile, plan->shape.items, plan->shape.wpb};
  if (n_items) *n_items = plan->n_items;
  if (n_splits) *n_splits = plan->n_splits;
  if (workspace_bytes) *workspace_bytes = (size_t)plan->n_slots * (size_t)plan->k * sizeof(uint64_t);
  return SA_OK;
}

sa_status sa_plan_score(const sa_plan *plan, const sa_arch *arch, const sa_variants *variants,
                        const sa_configs *configs, float *score, int32_t *occ_waves, int32_t *topk_idx,
                        float *topk_val, void *workspace, size_t workspace_bytes, void *stream) {
  if (!plan) return fail(SA_ERR_ARG, "plan is NULL");
  sa_status st;
  if ((st = sa_detail::check_arch(arch)) != SA_OK) return st;
  if (!variants || !configs || !configs->seg) return fail(SA_ERR_ARG, "variants / configs / seg is NULL");
  if (plan->n_evals > 0 && (!configs->block || !configs->unroll || !configs->regs))
    return fail(SA_ERR_ARG, "a required configuration column is NULL");
  if (plan->n_var > 0 && (!variants->n_fp || !variants->n_int || !variants->n_ld || !variants->n_st ||
                          !variants->n_br || !variants->n_bar || !variants->lds_bytes || !variants->div))
    return fail(SA_ERR_ARG, "a required variant column is NULL");
  const bool topk = topk_idx || topk_val;
  if (topk && plan->k < 1) return fail(SA_ERR_ARG, "the plan was made with k = 0");
  if (!topk && !score && !occ_waves) return fail(SA_ERR_ARG, "no output requested");
  sa::EvalLaunch L{};
  L.arch = sa_detail::to_karch(arch);
  L.var = {variants->n_fp, variants->n_int, variants->n_ld, variants->n_st, variants->n_br,
           variants->n_bar, variants->n_reg, variants->lds_bytes, variants->div};
  L.cfg = {configs->seg, configs->block, configs->unroll, configs->regs, configs->grid};
  L.n_var = plan->n_var;
  L.n_evals = plan->n_evals;
  L.occ = occ_waves;
  L.score = score;
  L.topk_idx = topk_idx;
  L.topk_val = topk_val;
  L.tile = plan->shape.tile;
  L.need_score = (score || topk) ? 1 : 0;
  L.vec = sa_detail::all16({configs->block, configs->unroll, configs->regs, configs->grid, occ_waves, score}) ? 1 : 0;
  sa_detail::set_lds_layout(L);
  return plan_launch(plan, L, sa::Mode::Model, configs->grid != nullptr, topk, workspace, workspace_bytes,
                     (hipStream_t)stream);
}

sa_status sa_plan_topk(const sa_plan *plan, const float *keys, const int64_t *seg, int32_t *idx, float *val,
                       void *workspace, size_t workspace_bytes, void *stream) {
  if (!plan) return fail(SA_ERR_ARG, "plan is NULL");
  if (plan->k < 1) return fail(SA_ERR_ARG, "the plan was made with k = 0");
  if (!seg || (plan->n_evals > 0 && !keys) || (plan->n_var > 0 && !idx)) return fail(SA_ERR_ARG, "NULL argument");
  sa::EvalLaunch L{};
  L.cfg.seg = seg;
  L.keys = keys;
  L.n_var = plan->n_var;
  L.n_evals = plan->n_evals;
  L.topk_idx = idx;
  L.topk_val = val;
  L.tile = plan->shape.tile;
  L.vec = sa_detail::all16({keys}) ? 1 : 0;
  return plan_launch(plan, L, sa::Mode::Keys, false, true, workspace, workspace_bytes, (hipStream_t)stream);
}

size_t sa_plan_autotune_workspace_bytes(int64_t n_variants, int64_t n_evals, int32_t k) {
  // kind-1 items of the smallest candidate shape bound the fragment slots
  if (k <= 0 || n_evals <= 0) return 0;
  (void)n_variants;
  const int64_t smallest = 1024 * 4;
  return (size_t)((n_evals + smallest - 1) / smallest + n_variants + 1) * (size_t)k * sizeof(uint64_t);
}

sa_status sa_plan_autotune(const int64_t *seg_host, int64_t n_variants, int64_t n_evals, int32_t k,
                           const sa_arch *arch, const sa_variants *variants, const sa_configs *configs, float *score,
                           int32_t *occ_waves, int32_t *topk_idx, float *topk_val, void *workspace,
                           size_t workspace_bytes, void *stream, int32_t reps, sa_plan_shape *best, float *best_ms) {
  if (!best) return fail(SA_ERR_ARG, "best is NULL");
  if (reps < 1) reps = 3;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(SA_ERR_HIP, "hipEventCreate");
  const int32_t tiles[] = {1024, 2048, 4096, 8192};
  const int32_t items[] = {1, 2, 4};
  const int32_t wpbs[] = {4, 8, 16};
  float best_t = 3.0e38f;
  sa_status result = SA_ERR_UNSUPPORTED;
  for (int32_t t : tiles)
    for (int32_t it : items)
      for (int32_t w : wpbs) {
        sa_plan_shape sh{t, it, w};
        sa_plan *p = nullptr;
        sa_status st = sa_plan_create(seg_host, n_variants, n_evals, k, &sh, &p);
        if (st != SA_OK) {
          result = st;
          goto done;
        }
        size_t need = 0;
        sa_plan_info(p, nullptr, nullptr, nullptr, &need);
        if (need > workspace_bytes && (topk_idx || topk_val)) {
          sa_plan_destroy(p);
          continue;
        }
        st = sa_plan_score(p, arch, variants, configs, score, occ_waves, topk_idx, topk_val, workspace,
                           workspace_bytes, stream);  // warm-up
        std::vector<float> ts;
        for (int r = 0; st == SA_OK && r < reps; ++r) {
          (void)hipEventRecord(e0, s);
          st = sa_plan_score(p, arch, variants, configs, score, occ_waves, topk_idx, topk_val, workspace,
                             workspace_bytes, stream);
          (void)hipEventRecord(e1, s);
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          ts.push_back(ms);
        }
        sa_plan_destroy(p);
        if (st != SA_OK) {
          result = st;
          goto done;
        }
        std::sort(ts.begin(), ts.end());
        const float med = ts[ts.size() / 2];
        if (med < best_t) {
          best_t = med;
          *best = sh;
          result = SA_OK;
        }
      }
done:
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_ms) *best_ms = best_t;
  return result;
}

}  // extern "C"
