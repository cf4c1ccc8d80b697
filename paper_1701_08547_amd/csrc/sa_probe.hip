// Residency probe: how many workgroups of a given block size, register
// count and LDS size one compute unit actually holds at once.
//
// The occupancy bound of Sec. III-A (Eqs. 1-5) rests on per-device limits
// (Table I: warps and blocks per multiprocessor, register file and its
// allocation unit, shared memory per multiprocessor).  For CDNA4 those
// limits come from public documentation; this probe measures them.  Each
// workgroup of a probe kernel spins for a fixed real time and records the
// hardware slot it ran on (XCC, shader engine, array and CU ids) with its
// start and end time; on the host, the largest number of intervals that
// overlap on one CU is the number of workgroups the CU held at once.  The
// probe kernels force their register count with a clobber of the highest
// register they must own, so the code object declares exactly that many
// (checked on the build's assembly).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa_runtime.h"

namespace sa_rt_detail {
int32_t fail(int32_t code, const char *msg);
}

namespace {

// s_getreg immediates: register id | offset << 6 | (bits - 1) << 11.
constexpr int kHwRegHwId = 4 | (0 << 6) | (31 << 11);
constexpr int kHwRegXccId = 20 | (0 << 6) | (31 << 11);

// Claim registers up to v(R - 1) (and the whole AGPR file for R = 512): the
// register allocator must then reserve at least R unified registers.
template <int R>
__device__ __forceinline__ void claim_registers() {
  static_assert(R == 16 || R == 24 || R == 64 || R == 72 || R == 80 || R == 96 || R == 128 || R == 168 ||
                    R == 256 || R == 512,
                "unsupported register count");
  if constexpr (R == 16) asm volatile("" ::: "v15");
  if constexpr (R == 24) asm volatile("" ::: "v23");
  if constexpr (R == 64) asm volatile("" ::: "v63");
  if constexpr (R == 72) asm volatile("" ::: "v71");
  if constexpr (R == 80) asm volatile("" ::: "v79");
  if constexpr (R == 96) asm volatile("" ::: "v95");
  if constexpr (R == 128) asm volatile("" ::: "v127");
  if constexpr (R == 168) asm volatile("" ::: "v167");
  if constexpr (R == 256) asm volatile("" ::: "v255");
  if constexpr (R == 512) asm volatile("" ::: "v255", "a255");
}

// One record per workgroup: start and end (the constant-rate real-time counter),
// the HW_ID and XCC_ID hardware registers of its first wave.
template <int LB, int R>
__global__ __launch_bounds__(LB) void sa_residency_kernel(int64_t *records, uint64_t spin_ticks) {
  const uint64_t t0 = wall_clock64();
  claim_registers<R>();
  while (wall_clock64() - t0 < spin_ticks) {
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t t1 = wall_clock64();
    const uint32_t hw = (uint32_t)__builtin_amdgcn_s_getreg(kHwRegHwId);
    const uint32_t xcc = (uint32_t)__builtin_amdgcn_s_getreg(kHwRegXccId);
    int64_t *r = records + 4 * (int64_t)blockIdx.x;
    r[0] = (int64_t)t0;
    r[1] = (int64_t)t1;
    r[2] = (int64_t)hw;
    r[3] = (int64_t)xcc;
  }
}

using ProbeFn = void (*)(int64_t *, uint64_t);

struct ProbeEntry {
  int32_t lb, vgprs;
  ProbeFn fn;
};

#define SA_PROBE(LB, R) {LB, R, sa_residency_kernel<LB, R>}
const ProbeEntry kProbes[] = {
    SA_PROBE(64, 16),   SA_PROBE(64, 24),   SA_PROBE(64, 64),   SA_PROBE(64, 72),   SA_PROBE(64, 80),
    SA_PROBE(64, 128),  SA_PROBE(64, 256),  SA_PROBE(64, 512),  SA_PROBE(128, 16),  SA_PROBE(128, 64),
    SA_PROBE(128, 256), SA_PROBE(192, 16),  SA_PROBE(192, 96),  SA_PROBE(192, 168), SA_PROBE(256, 64),
    SA_PROBE(256, 128), SA_PROBE(320, 16),  SA_PROBE(320, 96),  SA_PROBE(320, 168), SA_PROBE(384, 16),
    SA_PROBE(384, 128), SA_PROBE(448, 16),  SA_PROBE(512, 80),  SA_PROBE(576, 16),  SA_PROBE(640, 16),
    SA_PROBE(768, 16),  SA_PROBE(960, 16),  SA_PROBE(1024, 64), SA_PROBE(1024, 128),
};
#undef SA_PROBE

const ProbeEntry *find_probe(int32_t block, int32_t vgprs) {
  const int32_t lb = (block + 63) / 64 * 64;
  for (const ProbeEntry &p : kProbes)
    if (p.lb == lb && p.vgprs == vgprs) return &p;
  return nullptr;
}

}  // namespace

extern "C" {

int32_t sa_rt_residency(int32_t block, int32_t vgprs, int32_t lds_bytes, int32_t n_blocks, int32_t spin_us,
                        int64_t *records, int32_t *api_blocks_per_cu, void *stream) {
  using sa_rt_detail::fail;
  const ProbeEntry *p = block >= 1 ? find_probe(block, vgprs) : nullptr;
  if (!p) return fail(-1, "no probe kernel for this (block, vgprs) pair");
  if (n_blocks < 1 || n_blocks > (1 << 20)) return fail(-1, "n_blocks outside [1, 2^20]");
  if (spin_us < 1 || spin_us > 100000) return fail(-1, "spin_us outside [1, 100000]");
  if (!records) return fail(-1, "records is NULL");
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(-5, "hipGetDevice");
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return fail(-5, "hipDeviceGetAttribute");
  if (lds_bytes < 0 || lds_bytes > max_lds) return fail(-1, "lds_bytes outside [0, the device's per-block limit]");
  if (api_blocks_per_cu) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, p->fn, block, (size_t)lds_bytes) != hipSuccess)
      return fail(-5, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    *api_blocks_per_cu = nb;
  }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return fail(-5, "hipDeviceGetAttribute (wall clock rate)");
  const uint64_t ticks = (uint64_t)spin_us * (uint64_t)khz / 1000u;
  hipLaunchKernelGGL(p->fn, dim3((uint32_t)n_blocks), dim3((uint32_t)block), (size_t)lds_bytes, (hipStream_t)stream,
                     records, ticks);
  if (hipGetLastError() != hipSuccess) return fail(-5, "residency probe launch");
  return 0;
}

}  // extern "C"
