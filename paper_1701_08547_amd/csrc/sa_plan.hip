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

// A plan owns no device memory: its decomposition lives here, on the host,
// and sa_plan_bind copies it into a caller-provided device table.
struct sa_plan {
  int64_t n_var = 0, n_evals = 0;
  int32_t k = 0;
  sa::PlanShape shape{};
  int64_t n_items = 0, n_splits = 0, n_slots = 0;
  std::vector<sa::PlanItem> items;
  std::vector<sa::PlanWave> waves;
  std::vector<sa::PlanSplit> splits;
  sa::PlanDev pd{};  // pointers into the bound table (null until bound)
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

// Items in descending order of their longest wave part (evaluations plus the
// per-segment charge), the order the kernel's workgroups take them from its
// queue: the long items start first and the last ones taken are short, so
// the workgroups finish close together (greedy list scheduling of the
// longest first).  Slots and splits name items by slot, not by position, so
// the order is free.
void order_items(const int64_t *seg, const sa::PlanShape &S, std::vector<sa::PlanItem> &items,
                 std::vector<sa::PlanWave> &waves) {
  const int64_t kSegCharge = 256, wpb = S.wpb, n = (int64_t)items.size();
  std::vector<int64_t> cost(n), order(n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = 0;
    for (int64_t w = 0; w < wpb; ++w) {
      const sa::PlanWave &pw = waves[i * wpb + w];
      const int64_t cw = items[i].kind == 0 ? seg[pw.v1] - seg[pw.v0] + kSegCharge * (pw.v1 - pw.v0)
                                            : pw.e1 - pw.e0 + kSegCharge;
      c = std::max(c, cw);
    }
    cost[i] = c;
    order[i] = i;
  }
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cost[a] > cost[b]; });
  std::vector<sa::PlanItem> it(n);
  std::vector<sa::PlanWave> wv(waves.size());
  for (int64_t j = 0; j < n; ++j) {
    it[j] = items[order[j]];
    for (int64_t w = 0; w < wpb; ++w) wv[j * wpb + w] = waves[order[j] * wpb + w];
  }
  items.swap(it);
  waves.swap(wv);
}

// Byte offsets of the three arrays and the item queue inside the device
// table.
struct TableLayout {
  size_t items, waves, splits, queue, total;
};

TableLayout table_layout(const sa_plan *p) {
  const size_t bi = p->items.size() * sizeof(sa::PlanItem), bw = p->waves.size() * sizeof(sa::PlanWave),
               bs = p->splits.size() * sizeof(sa::PlanSplit);
  TableLayout t;
  t.items = 0;
  t.waves = (bi + 255) / 256 * 256;
  t.splits = t.waves + (bw + 255) / 256 * 256;
  t.queue = t.splits + (bs + 255) / 256 * 256;
  t.total = t.queue + 256;
  return t;
}

size_t fragment_bytes(const sa_plan *p) { return (size_t)p->n_slots * (size_t)p->k * sizeof(uint64_t); }

sa_status plan_launch(const sa_plan *plan, sa::EvalLaunch &L, sa::Mode mode, bool has_grid, bool topk, void *workspace,
                      size_t workspace_bytes, hipStream_t stream) {
  if (!plan->pd.items && plan->n_items > 0)
    return fail(SA_ERR_ARG, "the plan has no device table: call sa_plan_bind first");
  L.k = topk ? plan->k : 0;
  if (topk) {
    const size_t need = fragment_bytes(plan);
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
  order_items(seg_host, S, it, wv);
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
  sa_plan *p = new sa_plan();
  decompose(seg_host, n_variants, S, p->items, p->waves, p->splits, p->n_slots);
  order_items(seg_host, S, p->items, p->waves);
  if ((int64_t)p->items.size() > (int64_t)INT32_MAX) {
    delete p;
    return fail(SA_ERR_UNSUPPORTED, "more than 2^31 workgroup items");
  }
  p->n_var = n_variants;
  p->n_evals = n_evals;
  p->k = k;
  p->shape = S;
  p->n_items = (int64_t)p->items.size();
  p->n_splits = (int64_t)p->splits.size();
  *out = p;
  return SA_OK;
}

size_t sa_plan_device_bytes(const sa_plan *plan) { return plan ? table_layout(plan).total : 0; }

sa_status sa_plan_bind(sa_plan *plan, void *table, size_t table_bytes, void *stream) {
  if (!plan) return fail(SA_ERR_ARG, "plan is NULL");
  if (!table) return fail(SA_ERR_ARG, "table is NULL");
  if ((uintptr_t)table % 256) return fail(SA_ERR_ALIGN, "table not 256-byte aligned");
  const TableLayout t = table_layout(plan);
  if (table_bytes < t.total) return fail(SA_ERR_WORKSPACE, "table %zu bytes < %zu needed", table_bytes, t.total);
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return hip_fail(e, "hipDeviceGetAttribute");
  char *base = (char *)table;
  hipStream_t s = (hipStream_t)stream;
  const size_t bi = plan->items.size() * sizeof(sa::PlanItem), bw = plan->waves.size() * sizeof(sa::PlanWave),
               bs = plan->splits.size() * sizeof(sa::PlanSplit);
  if ((bi && (e = hipMemcpyAsync(base + t.items, plan->items.data(), bi, hipMemcpyHostToDevice, s)) != hipSuccess) ||
      (bw && (e = hipMemcpyAsync(base + t.waves, plan->waves.data(), bw, hipMemcpyHostToDevice, s)) != hipSuccess) ||
      (bs && (e = hipMemcpyAsync(base + t.splits, plan->splits.data(), bs, hipMemcpyHostToDevice, s)) != hipSuccess))
    return hip_fail(e, "hipMemcpyAsync (plan table)");
  static const uint32_t kQueueZero[1] = {0u};
  if ((e = hipMemcpyAsync(base + t.queue, kQueueZero, sizeof(kQueueZero), hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "hipMemcpyAsync (plan queue)");
  plan->n_cu = n_cu > 0 ? n_cu : 1;
  plan->pd.items = (const sa::PlanItem *)(base + t.items);
  plan->pd.waves = (const sa::PlanWave *)(base + t.waves);
  plan->pd.splits = (const sa::PlanSplit *)(base + t.splits);
  plan->pd.n_items = plan->n_items;
  plan->pd.n_splits = plan->n_splits;
  plan->pd.queue = (uint32_t *)(base + t.queue);
  return SA_OK;
}

sa_status sa_plan_destroy(sa_plan *plan) {
  delete plan;
  return SA_OK;
}

sa_status sa_plan_info(const sa_plan *plan, sa_plan_shape *shape, int64_t *n_items, int64_t *n_splits,
                       size_t *workspace_bytes) {
  if (!plan) return fail(SA_ERR_ARG, "plan is NULL");
  if (shape) *shape = sa_plan_shape{plan->shape.tile, plan->shape.items, plan->shape.wpb};
  if (n_items) *n_items = plan->n_items;
  if (n_splits) *n_splits = plan->n_splits;
  if (workspace_bytes) *workspace_bytes = fragment_bytes(plan);
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

}  // extern "C"

namespace {

const int32_t kTuneTiles[] = {1024, 2048, 4096, 8192};
const int32_t kTuneItems[] = {1, 2, 4};
const int32_t kTuneWaves[] = {4, 8, 16};

// Largest fragment area and largest device table over the autotuner's
// shapes (each 256-byte aligned): the workspace holds both, fragments first.
sa_status tune_sizes(const int64_t *seg_host, int64_t n_variants, int64_t n_evals, int32_t k, size_t *frag,
                     size_t *table) {
  *frag = *table = 0;
  for (int32_t t : kTuneTiles)
    for (int32_t it : kTuneItems)
      for (int32_t w : kTuneWaves) {
        sa_plan_shape sh{t, it, w};
        sa_plan *p = nullptr;
        sa_status st = sa_plan_create(seg_host, n_variants, n_evals, k, &sh, &p);
        if (st != SA_OK) return st;
        *frag = std::max(*frag, (fragment_bytes(p) + 255) / 256 * 256);
        *table = std::max(*table, table_layout(p).total);
        sa_plan_destroy(p);
      }
  return SA_OK;
}

}  // namespace

extern "C" {

size_t sa_plan_autotune_workspace_bytes(const int64_t *seg_host, int64_t n_variants, int64_t n_evals, int32_t k) {
  size_t frag = 0, table = 0;
  if (tune_sizes(seg_host, n_variants, n_evals, k, &frag, &table) != SA_OK) return 0;
  return frag + table;
}

sa_status sa_plan_autotune(const int64_t *seg_host, int64_t n_variants, int64_t n_evals, int32_t k,
                           const sa_arch *arch, const sa_variants *variants, const sa_configs *configs, float *score,
                           int32_t *occ_waves, int32_t *topk_idx, float *topk_val, void *workspace,
                           size_t workspace_bytes, void *stream, int32_t reps, sa_plan_shape *best, float *best_ms) {
  if (!best) return fail(SA_ERR_ARG, "best is NULL");
  if (reps < 1) reps = 3;
  size_t frag_bytes = 0, table_bytes = 0;
  sa_status st0 = tune_sizes(seg_host, n_variants, n_evals, k, &frag_bytes, &table_bytes);
  if (st0 != SA_OK) return st0;
  if (!workspace) return fail(SA_ERR_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)workspace % 256) return fail(SA_ERR_ALIGN, "workspace not 256-byte aligned");
  if (workspace_bytes < frag_bytes + table_bytes)
    return fail(SA_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", workspace_bytes, frag_bytes + table_bytes);
  void *table = (char *)workspace + frag_bytes;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(SA_ERR_HIP, "hipEventCreate");
  float best_t = 3.0e38f;
  sa_status result = SA_ERR_UNSUPPORTED;
  for (int32_t t : kTuneTiles)
    for (int32_t it : kTuneItems)
      for (int32_t w : kTuneWaves) {
        sa_plan_shape sh{t, it, w};
        sa_plan *p = nullptr;
        sa_status st = sa_plan_create(seg_host, n_variants, n_evals, k, &sh, &p);
        if (st == SA_OK) st = sa_plan_bind(p, table, table_bytes, stream);
        if (st != SA_OK) {
          sa_plan_destroy(p);
          result = st;
          goto done;
        }
        st = sa_plan_score(p, arch, variants, configs, score, occ_waves, topk_idx, topk_val, workspace,
                           frag_bytes, stream);  // warm-up
        std::vector<float> ts;
        for (int r = 0; st == SA_OK && r < reps; ++r) {
          (void)hipEventRecord(e0, s);
          st = sa_plan_score(p, arch, variants, configs, score, occ_waves, topk_idx, topk_val, workspace,
                             frag_bytes, stream);
          (void)hipEventRecord(e1, s);
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          ts.push_back(ms);
        }
        // the table's upload and every launch reading it have finished
        // before the plan (the upload's host source) goes away
        (void)hipStreamSynchronize(s);
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
