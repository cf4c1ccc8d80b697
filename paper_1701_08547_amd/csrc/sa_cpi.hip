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

// Memory ceiling of the plain scoring pass: the same bytes per evaluation
// (four 4-byte configuration columns read, two 4-byte result columns
// written) with none of the model's arithmetic, so that a pass's HBM rate
// can be set against what a pure stream of its traffic reaches here.
namespace {

constexpr int kStreamThreads = 256;
typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

template <int ITEMS, bool NT>
__global__ __launch_bounds__(kStreamThreads) void rt_stream_kernel(const v4i *c0, const v4i *c1, const v4i *c2,
                                                                    const v4i *c3, v4i *o0, v4i *o1, int64_t n4) {
  const int64_t step = (int64_t)gridDim.x * kStreamThreads * ITEMS;
  for (int64_t base = (int64_t)blockIdx.x * kStreamThreads * ITEMS + threadIdx.x; base < n4; base += step) {
    v4i a[ITEMS], b[ITEMS], c[ITEMS], d[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int64_t i = base + (int64_t)j * kStreamThreads;
      if (i < n4) {
        a[j] = c0[i];
        b[j] = c1[i];
        c[j] = c2[i];
        d[j] = c3[i];
      }
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int64_t i = base + (int64_t)j * kStreamThreads;
      if (i < n4) {
        // wrapping sum: add as unsigned
        const v4i s = __builtin_bit_cast(v4i, __builtin_bit_cast(v4u, a[j]) + __builtin_bit_cast(v4u, b[j]));
        const v4i x = c[j] ^ d[j];
        if constexpr (NT) {
          __builtin_nontemporal_store(s, o0 + i);
          __builtin_nontemporal_store(x, o1 + i);
        } else {
          o0[i] = s;
          o1[i] = x;
        }
      }
    }
  }
}

template <bool NT>
hipError_t launch_stream_nt(int32_t items, dim3 g, const v4i *const *in, v4i *o0, v4i *o1, int64_t n4,
                            hipStream_t s) {
  const dim3 b(kStreamThreads);
  switch (items) {
    case 1: hipLaunchKernelGGL((rt_stream_kernel<1, NT>), g, b, 0, s, in[0], in[1], in[2], in[3], o0, o1, n4); break;
    case 2: hipLaunchKernelGGL((rt_stream_kernel<2, NT>), g, b, 0, s, in[0], in[1], in[2], in[3], o0, o1, n4); break;
    default: hipLaunchKernelGGL((rt_stream_kernel<4, NT>), g, b, 0, s, in[0], in[1], in[2], in[3], o0, o1, n4); break;
  }
  return hipGetLastError();
}

hipError_t launch_stream(int32_t items, bool nt, int64_t grid, const v4i *const *in, v4i *o0, v4i *o1, int64_t n4,
                         hipStream_t s) {
  const dim3 g((uint32_t)grid);
  return nt ? launch_stream_nt<true>(items, g, in, o0, o1, n4, s) : launch_stream_nt<false>(items, g, in, o0, o1, n4, s);
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

extern "C" int32_t sa_rt_stream(int64_t n, const int32_t *c0, const int32_t *c1, const int32_t *c2,
                                const int32_t *c3, int32_t *o0, int32_t *o1, int32_t items, int32_t blocks_per_cu,
                                int32_t nontemporal, int32_t reps, float *ms_out, void *stream) {
  using sa_rt_detail::fail;
  if (n < 4 || n % 4 != 0) return fail(-1, "n must be a positive multiple of 4");
  if (items != 1 && items != 2 && items != 4) return fail(-1, "items must be 1, 2 or 4");
  if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(-1, "blocks_per_cu outside [0, 64]");
  if (nontemporal != 0 && nontemporal != 1) return fail(-1, "nontemporal must be 0 or 1");
  if (reps < 1 || reps > 64) return fail(-1, "reps outside [1, 64]");
  const void *ptrs[] = {c0, c1, c2, c3, o0, o1};
  for (const void *p : ptrs) {
    if (!p) return fail(-1, "NULL column");
    if (!aligned16(p)) return fail(-1, "column not 16-byte aligned");
  }
  if (!ms_out) return fail(-1, "ms_out is NULL");
  const int64_t n4 = n / 4;
  const int64_t per_block = (int64_t)kStreamThreads * items;
  int64_t grid = (n4 + per_block - 1) / per_block;
  if (blocks_per_cu > 0) {
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
      return fail(-5, "device query failed");
    grid = std::min<int64_t>(grid, (int64_t)n_cu * blocks_per_cu);
  }
  if (grid > 0x7FFFFFFF) return fail(-1, "n too large for one launch");
  const v4i *in[4] = {(const v4i *)c0, (const v4i *)c1, (const v4i *)c2, (const v4i *)c3};
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(-5, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(-5, "hipEventCreate failed");
  }
  // one warm-up launch, then `reps` launches back to back between two events
  int32_t status = 0;
  if (launch_stream(items, nontemporal != 0, grid, in, (v4i *)o0, (v4i *)o1, n4, s) != hipSuccess) status = fail(-5, "launch failed");
  if (status == 0 && hipEventRecord(e0, s) != hipSuccess) status = fail(-5, "hipEventRecord failed");
  for (int r = 0; r < reps && status == 0; ++r)
    if (launch_stream(items, nontemporal != 0, grid, in, (v4i *)o0, (v4i *)o1, n4, s) != hipSuccess) status = fail(-5, "launch failed");
  float ms = 0.0f;
  if (status == 0 && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                      hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    status = fail(-5, "timing failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status) return status;
  *ms_out = ms / (float)reps;
  return 0;
}
