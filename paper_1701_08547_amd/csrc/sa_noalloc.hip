// sa_score for callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation): the same pass with
// its fragment slots in a fixed device array of this library instead of a
// caller workspace.
//
// The array is a file-scope device variable; each GPU the library runs on
// holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol): the first call on a device, with that device current, asks HIP for
// the copy's device address, and every later call on that device uses the
// address kept for it.  The fragment slots need no initialisation (each is
// written before it is read within one call), so nothing is cleared.  All
// calls on one GPU share its copy: calls that overlap in time on one GPU
// (different streams, or different host threads without ordering) race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sa.h"
#include "sa_internal.h"

namespace sa_detail {
sa_status fail(sa_status st, const char *fmt, ...);
sa_status hip_fail(hipError_t e, const char *what);
size_t score_workspace_need(int64_t n_evals, int32_t k, bool corrected);
}  // namespace sa_detail

static __device__ __align__(256) uint8_t scratch[SA_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices];
std::mutex g_mu;

// Device address of the current device's copy of `scratch`.
sa_status scratch_ptr(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return sa_detail::hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return sa_detail::fail(SA_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return sa_detail::hip_fail(e, "hipGetSymbolAddress (scratch)");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return SA_OK;
}

}  // namespace

extern "C" {

sa_status sa_score_noalloc(const sa_arch *arch, const sa_variants *variants, const sa_configs *configs,
                           int64_t n_variants, int64_t n_evals, float *score, int32_t *occ_waves, int32_t k,
                           int32_t *topk_idx, float *topk_val, const sa_mlp *mlp, void *stream) {
  const bool topk = topk_idx || topk_val;
  void *ws = nullptr;
  if (topk && n_variants > 0 && n_evals > 0 && k >= 1 && k <= SA_K_MAX) {
    const size_t need = sa_detail::score_workspace_need(n_evals, k, mlp != nullptr);
    if (need > (size_t)SA_NOALLOC_SCRATCH_BYTES)
      return sa_detail::fail(SA_ERR_WORKSPACE,
                             "%lld evaluations with k = %d need %zu bytes of fragment slots; the allocation-free "
                             "entry point holds %zu",
                             (long long)n_evals, k, need, (size_t)SA_NOALLOC_SCRATCH_BYTES);
    const sa_status st = scratch_ptr(&ws);
    if (st != SA_OK) return st;
  }
  return sa_score(arch, variants, configs, n_variants, n_evals, score, occ_waves, k, topk_idx, topk_val, mlp, ws,
                  ws ? (size_t)SA_NOALLOC_SCRATCH_BYTES : 0, stream);
}

}  // extern "C"
