// Issue cost of the instruction categories of Eq. 6 on the current device.
//
// Table II of the paper gives, per NVIDIA architecture, the instructions per
// cycle per multiprocessor of each functional-unit class; the static score
// weights a kernel's instruction counts by their inverses.  These
// microbenchmarks measure the same quantity on this device: every compute
// unit runs 32 waves (8 four-wave workgroups) whose instruction stream is
// dominated by one category, and the cost is CU-cycles per thread-
// instruction, elapsed cycles x CUs / thread-instructions issued.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "sa_runtime.h"

namespace sa_rt_detail {
int32_t fail(int32_t code, const char *msg);
}

namespace {

constexpr int kThreads = 256;
constexpr int kBlocksPerCu = 8;
constexpr int kBufFloats = 4096;  // 16 KiB, cache resident

// Thread-instructions of the measured category per loop iteration, and
// iterations per launch (about a millisecond each).
constexpr int kPerIter[6] = {64, 64, 16, 1, 16, 64};
constexpr int kIters[6] = {1024, 1024, 1024, 65536, 512, 1024};

template <int CAT>
__global__ __launch_bounds__(kThreads) void rt_cpi_kernel(const float *buf, int iters, float *sink) {
  const int tid = threadIdx.x;
  if constexpr (CAT == SA_CPI_FP) {
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (float)(tid + j);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = fmaf(a[j], 0.999f, 0.001f);
    }
    float t = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) t += a[j];
    if (t == -1.0f) sink[tid] = t;
  } else if constexpr (CAT == SA_CPI_INT || CAT == SA_CPI_REG) {
    uint32_t a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (uint32_t)(tid * 8 + j);
    const uint32_t k = (uint32_t)blockIdx.x | 1u;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if constexpr (CAT == SA_CPI_INT)
            asm volatile("v_add_u32_e32 %0, %1, %0" : "+v"(a[j]) : "v"(k));
          else
            asm volatile("v_mov_b32_e32 %0, %1" : "=v"(a[j]) : "v"(a[(j + 1) & 7]));
        }
    }
    uint32_t t = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) t ^= a[j];
    if (t == 0xFFFFFFFFu) sink[tid] = (float)t;
  } else if constexpr (CAT == SA_CPI_MEM) {
    const float *p = buf + (tid & 63);
    float a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int j = 0; j < 16; ++j) a[j & 3] += p[(((i & 3) * 16 + j) * 64) & (kBufFloats - 1)];
    }
    const float t = (a[0] + a[1]) + (a[2] + a[3]);
    if (t == -1.0f) sink[tid] = t;
  } else if constexpr (CAT == SA_CPI_CTRL) {
    // one uniform loop branch per iteration, nothing else but its counter
    for (int i = 0; i < iters; ++i) asm volatile("" ::: "memory");
  } else {  // SA_CPI_SYNC
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int j = 0; j < 16; ++j) __syncthreads();
    }
  }
}

hipError_t launch_cpi(int32_t cat, int grid, const float *buf, float *sink, hipStream_t s) {
  const int it = kIters[cat];
  switch (cat) {
    case SA_CPI_FP: hipLaunchKernelGGL(rt_cpi_kernel<SA_CPI_FP>, dim3(grid), dim3(kThreads), 0, s, buf, it, sink); break;
    case SA_CPI_INT: hipLaunchKernelGGL(rt_cpi_kernel<SA_CPI_INT>, dim3(grid), dim3(kThreads), 0, s, buf, it, sink); break;
    case SA_CPI_MEM: hipLaunchKernelGGL(rt_cpi_kernel<SA_CPI_MEM>, dim3(grid), dim3(kThreads), 0, s, buf, it, sink); break;
    case SA_CPI_CTRL: hipLaunchKernelGGL(rt_cpi_kernel<SA_CPI_CTRL>, dim3(grid), dim3(kThreads), 0, s, buf, it, sink); break;
    case SA_CPI_SYNC: hipLaunchKernelGGL(rt_cpi_kernel<SA_CPI_SYNC>, dim3(grid), dim3(kThreads), 0, s, buf, it, sink); break;
    default: hipLaunchKernelGGL(rt_cpi_kernel<SA_CPI_REG>, dim3(grid), dim3(kThreads), 0, s, buf, it, sink); break;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" int32_t sa_rt_cpi(int32_t category, int32_t reps, float *buf, float *cpi_out, float *ms_out, void *stream) {
  using sa_rt_detail::fail;
  if (category < 0 || category > 5) return fail(-1, "category outside [0, 5]");
  if (reps < 1 || reps > 64) return fail(-1, "reps outside [1, 64]");
  if (!buf || !cpi_out) return fail(-1, "NULL argument");
  int dev = 0, n_cu = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev) != hipSuccess || n_cu < 1 || khz < 1)
    return fail(-5, "device query failed");
  hipStream_t s = (hipStream_t)stream;
  const int grid = n_cu * kBlocksPerCu;
  float *sink = buf + kBufFloats;  // written only if a result were impossible
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(-5, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(-5, "hipEventCreate failed");
  }
  int32_t status = 0;
  std::vector<float> t;
  if (launch_cpi(category, grid, buf, sink, s) != hipSuccess) status = fail(-5, "launch failed");  // warm-up
  for (int r = 0; r < reps && status == 0; ++r) {
    float ms = 0.0f;
    if (hipEventRecord(e0, s) != hipSuccess || launch_cpi(category, grid, buf, sink, s) != hipSuccess ||
        hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      status = fail(-5, "timed launch failed");
    else
      t.push_back(ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status) return status;
  std::sort(t.begin(), t.end());
  const double ms = t[t.size() / 2];
  const double cycles = ms * (double)khz;  // kHz x ms
  const double thread_instr = (double)grid * kThreads * kIters[category] * kPerIter[category];
  *cpi_out = (float)(cycles * n_cu / thread_instr);
  if (ms_out) *ms_out = (float)ms;
  return 0;
}
