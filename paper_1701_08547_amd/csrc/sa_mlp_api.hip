// C ABI of the learned correction: features, inference and training steps.
#include <hip/hip_runtime.h>
#include <math.h>

#include <initializer_list>

#include "sa.h"
#include "sa_internal.h"
#include "sa_train.h"

namespace sa_detail {
sa_status fail(sa_status st, const char *fmt, ...);
sa_status check_arch(const sa_arch *a);
sa::KArch to_karch(const sa_arch *a);
sa_status hip_fail(hipError_t e, const char *what);

bool a4(const void *p) { return ((uintptr_t)p % 4) == 0; }

sa_status check_mlp(const sa_mlp *m) {
  if (!m) return fail(SA_ERR_ARG, "mlp is NULL");
  const void *ps[] = {m->W1, m->W2, m->w3, m->b1, m->b2, m->b3, m->feat_mean, m->feat_inv_std};
  for (const void *p : ps)
    if (!p) return fail(SA_ERR_ARG, "a pointer of mlp is NULL");
  if (((uintptr_t)m->W1 % 8) || ((uintptr_t)m->W2 % 8) || ((uintptr_t)m->w3 % 2))
    return fail(SA_ERR_ALIGN, "mlp weights must be 8-byte aligned");
  return SA_OK;
}

sa::MlpDev mlp_dev(const sa_mlp *m) {
  return sa::MlpDev{m->W1, m->W2, m->w3, m->b1, m->b2, m->b3, m->feat_mean, m->feat_inv_std};
}

}  // namespace sa_detail

using sa_detail::a4;
using sa_detail::check_mlp;
using sa_detail::fail;
using sa_detail::hip_fail;
using sa_detail::mlp_dev;

static_assert(sa::kPartUsed == SA_MLP_PARAMS, "parameter layout");
static_assert(sa::kPartStride == SA_MLP_FLAT, "flat layout");

namespace {

// Workspace carve-up of one training step of n rows: Delta, dL/dDelta and
// the per-row loss terms (pairwise loss), then the workgroups' gradient
// partials.
struct TrainLayout {
  size_t off[4];
  size_t total;
};

TrainLayout train_layout(int64_t n) {
  const size_t sizes[4] = {(size_t)n * 4, (size_t)n * 4, (size_t)n * 4,
                           (size_t)sa::train_partials(n) * (size_t)sa::kPartStride * 4};
  TrainLayout L{};
  size_t o = 0;
  for (int i = 0; i < 4; ++i) {
    L.off[i] = o;
    o += (sizes[i] + 255) / 256 * 256;
  }
  L.total = o;
  return L;
}

}  // namespace

extern "C" {

sa_status sa_features(const sa_arch *arch, const sa_variants *variants, const sa_configs *configs,
                      int64_t n_variants, int64_t n_evals, float *feat, void *stream) {
  sa_status st;
  if ((st = sa_detail::check_arch(arch)) != SA_OK) return st;
  if (n_variants < 0 || n_evals < 0) return fail(SA_ERR_ARG, "negative size");
  if (n_evals > 0 && n_variants == 0) return fail(SA_ERR_ARG, "n_evals > 0 with no variants");
  if (n_evals == 0) return SA_OK;
  if (!variants || !configs || !configs->seg || !configs->block || !configs->unroll || !configs->regs || !feat)
    return fail(SA_ERR_ARG, "NULL argument");
  if (!variants->n_fp || !variants->n_int || !variants->n_ld || !variants->n_st || !variants->n_br ||
      !variants->n_bar || !variants->lds_bytes || !variants->div)
    return fail(SA_ERR_ARG, "a required variant column is NULL");
  if (!a4(feat)) return fail(SA_ERR_ALIGN, "feat not 4-byte aligned");
  sa::EvalLaunch L{};
  L.arch = sa_detail::to_karch(arch);
  L.var = {variants->n_fp, variants->n_int, variants->n_ld, variants->n_st, variants->n_br,
           variants->n_bar, variants->n_reg, variants->lds_bytes, variants->div};
  L.cfg = {configs->seg, configs->block, configs->unroll, configs->regs, configs->grid};
  L.n_var = n_variants;
  L.n_evals = n_evals;
  hipError_t e = sa::launch_features(L, feat, (hipStream_t)stream);
  return e == hipSuccess ? SA_OK : hip_fail(e, "sa_features_kernel launch");
}

sa_status sa_surrogate_fwd(const sa_mlp *mlp, const float *feat, int64_t n, float *delta, void *stream) {
  sa_status st;
  if ((st = check_mlp(mlp)) != SA_OK) return st;
  if (n < 0) return fail(SA_ERR_ARG, "negative n");
  if (n == 0) return SA_OK;
  if (!feat || !delta) return fail(SA_ERR_ARG, "NULL argument");
  if (!a4(feat) || !a4(delta)) return fail(SA_ERR_ALIGN, "feat / delta not 4-byte aligned");
  hipError_t e = sa::launch_mlp_fwd(mlp_dev(mlp), feat, n, delta, (hipStream_t)stream);
  return e == hipSuccess ? SA_OK : hip_fail(e, "sa_mlp_fwd_kernel launch");
}

size_t sa_surrogate_train_workspace_bytes(int64_t n) {
  if (n <= 0) return 0;
  return train_layout(n).total;
}

}  // extern "C"

namespace {

sa_status train_step(const sa_mlp *mlp, float *master, float *adam_m, float *adam_v, int64_t step,
                     int64_t *step_counter, float lr, const float *feat, const float *target, int64_t n,
                     float *grad_out, int32_t group, void *workspace, size_t workspace_bytes, void *stream) {
  sa_status st;
  if ((st = check_mlp(mlp)) != SA_OK) return st;
  if (!master || !adam_m || !adam_v || !feat || !target) return fail(SA_ERR_ARG, "NULL argument");
  if (n < 1 || n > (1 << 20)) return fail(SA_ERR_ARG, "n = %lld outside [1, 2^20]", (long long)n);
  if (step_counter) {
    if (step != 0) return fail(SA_ERR_ARG, "step must be 0 when a step counter is given");
    if ((uintptr_t)step_counter % 8) return fail(SA_ERR_ALIGN, "step_counter not 8-byte aligned");
  } else if (step < 1) {
    return fail(SA_ERR_ARG, "step must be >= 1");
  }
  if (!(lr > 0.0f) || !isfinite(lr)) return fail(SA_ERR_ARG, "lr must be finite and > 0");
  const TrainLayout TL = train_layout(n);
  if (!workspace) return fail(SA_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", TL.total);
  if ((uintptr_t)workspace % 256) return fail(SA_ERR_ALIGN, "workspace not 256-byte aligned");
  if (workspace_bytes < TL.total) return fail(SA_ERR_WORKSPACE, "workspace %zu < %zu bytes", workspace_bytes, TL.total);
  char *w = (char *)workspace;
  sa::TrainBufs T;
  T.delta = (float *)(w + TL.off[0]);
  T.gdelta = (float *)(w + TL.off[1]);
  T.loss = (float *)(w + TL.off[2]);
  T.part = (float *)(w + TL.off[3]);
  sa::AdamArgs h;
  h.lr = lr;
  h.beta1 = 0.9f;
  h.beta2 = 0.999f;
  h.eps = 1e-8f;
  h.beta1_d = 0.9;
  h.beta2_d = 0.999;
  h.bc1 = step > 0 ? (float)(1.0 - pow(h.beta1_d, (double)step)) : 1.0f;
  h.bc2 = step > 0 ? (float)(1.0 - pow(h.beta2_d, (double)step)) : 1.0f;
  h.step_counter = step_counter;
  // the ranking loss's per-row terms already carry its normalisation
  h.inv_n = group > 0 ? 1.0f : 1.0f / (float)n;
  hipError_t e = sa::launch_train_step(mlp_dev(mlp), sa::TrainState{master, adam_m, adam_v}, feat, target, n, T, h,
                                       grad_out, group, (hipStream_t)stream);
  return e == hipSuccess ? SA_OK : hip_fail(e, "training kernels launch");
}

}  // namespace

extern "C" {

sa_status sa_surrogate_train_step(const sa_mlp *mlp, float *master, float *adam_m, float *adam_v, int64_t step,
                                  int64_t *step_counter, float lr, const float *feat, const float *target, int64_t n,
                                  float *grad_out, void *workspace, size_t workspace_bytes, void *stream) {
  return train_step(mlp, master, adam_m, adam_v, step, step_counter, lr, feat, target, n, grad_out, 0, workspace,
                    workspace_bytes, stream);
}

sa_status sa_surrogate_train_step_pairwise(const sa_mlp *mlp, float *master, float *adam_m, float *adam_v,
                                           int64_t step, int64_t *step_counter, float lr, const float *feat,
                                           const float *log_time, int64_t n, int32_t group, float *grad_out,
                                           void *workspace, size_t workspace_bytes, void *stream) {
  if (group < 2 || group > SA_RANK_GROUP_MAX) return fail(SA_ERR_ARG, "group %d outside [2, %d]", group, SA_RANK_GROUP_MAX);
  if (n % group != 0) return fail(SA_ERR_ARG, "n = %lld is not a multiple of group %d", (long long)n, group);
  return train_step(mlp, master, adam_m, adam_v, step, step_counter, lr, feat, log_time, n, grad_out, group,
                    workspace, workspace_bytes, stream);
}

}  // extern "C"
