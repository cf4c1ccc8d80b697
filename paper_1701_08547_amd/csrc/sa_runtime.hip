// Parametric kernel families whose measured runtimes train the learned
// correction, and the native timing harness that measures them.
//
// Each family is one kernel template over the unroll factor U (1..8); the
// block size T is a launch parameter and the grid G follows from the
// problem size by the family's launch rule.  Every kernel has exactly the
// loops listed in sa_runtime.h (a main loop whose body holds U unrolled
// steps, plus the reduction's tree loop), so that static instruction counts
// read from the compiled code object scale with the trip counts computed on
// the host.
//
// Timing follows the paper's experimental protocol (Sec. IV-A): one warm-up
// launch, then repeated timed launches of which a fixed order statistic is
// kept (the fifth smallest of ten).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "sa_runtime.h"

namespace {

constexpr int kLcmUnroll = 840;  // lcm(1..8): matvec sizes are multiples of it

// y += A x, A column-major N x N (thread i reads row i: coalesced), split
// over the columns: block (bx, by) covers rows bx T .. bx T + T - 1 and the
// 840 columns of chunk by; each thread adds its partial dot product with one
// atomic.  840 = lcm(1..8), so every U divides a chunk; N is a multiple of
// 840.
template <int U>
__global__ void rt_matvec(const float *__restrict__ A, const float *__restrict__ x, float *__restrict__ y, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int j0 = blockIdx.y * kLcmUnroll;
  float acc = 0.0f;
#pragma unroll 1
  for (int j = j0; j < j0 + kLcmUnroll; j += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) acc += A[(size_t)(j + u) * N + i] * x[j + u];
  }
  atomicAdd(&y[i], acc);
}

// One out-of-place 5-point sweep over the interior of an n x n grid: a unit
// is U consecutive interior points of a row; grid-stride over units (32-bit
// indices: n <= 32768).
template <int U>
__global__ void rt_stencil(const float *__restrict__ in, float *__restrict__ out, int n, int units) {
  const int per_row = (n - 2 + U - 1) / U;
  const int stride = gridDim.x * blockDim.x;
#pragma unroll 1
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < units; w += stride) {
    const int row = 1 + w / per_row;
    const int col0 = 1 + (w % per_row) * U;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = col0 + u;
      if (c < n - 1) {
        const int p = row * n + c;
        out[p] = 0.25f * (in[p - 1] + in[p + 1] + in[p - n] + in[p + n]) - in[p];
      }
    }
  }
}

// Sum of n values (n < 2^30): grid-stride accumulation of U elements per
// step, a tree reduction in LDS, one atomic add per block.
template <int U>
__global__ void rt_reduce(const float *__restrict__ in, float *__restrict__ out, int n) {
  __shared__ float buf[1024];
  const int tid = threadIdx.x, T = blockDim.x;
  float acc = 0.0f;
  const int stride = gridDim.x * T * U;
#pragma unroll 1
  for (int b = blockIdx.x * T * U + tid; b < n; b += stride) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = b + u * T;
      if (i < n) acc += in[i];
    }
  }
  buf[tid] = acc;
  __syncthreads();
  const int h = T > 1 ? 1 << (32 - __clz(T - 1)) : 1;  // T rounded up to a power of two
#pragma unroll 1
  for (int s = h >> 1; s > 0; s >>= 1) {
    if (tid < s && tid + s < T) buf[tid] += buf[tid + s];
    __syncthreads();
  }
  if (tid == 0) atomicAdd(out, buf[0]);
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Blocks a grid-stride family launches: enough for the work, at most
// 2048 threads' worth per compute unit.
int64_t stride_grid(int64_t work_units, int32_t T, int32_t n_cu) {
  const int64_t cap = (int64_t)n_cu * (2048 / T > 0 ? 2048 / T : 1);
  const int64_t need = ceil_div(work_units, T);
  return std::max<int64_t>(1, std::min(need, cap));
}

hipError_t launch(int32_t family, int64_t n, int32_t T, int32_t U, int64_t G, const float *a, const float *b,
                  float *c, hipStream_t s) {
  // matvec: G = row blocks x column chunks, launched as a 2-D grid
  const dim3 grid = family == SA_RT_MATVEC ? dim3((uint32_t)ceil_div(n, T), (uint32_t)(n / kLcmUnroll))
                                           : dim3((uint32_t)G);
  const dim3 block((uint32_t)T);
#define SA_RT_CASE(UU)                                                                                   \
  case UU:                                                                                               \
    if (family == SA_RT_MATVEC)                                                                          \
      hipLaunchKernelGGL(rt_matvec<UU>, grid, block, 0, s, a, b, c, (int)n);                             \
    else if (family == SA_RT_STENCIL)                                                                    \
      hipLaunchKernelGGL(rt_stencil<UU>, grid, block, 0, s, a, c, (int)n,                                \
                         (int)((n - 2) * ceil_div(n - 2, UU)));                                          \
    else                                                                                                 \
      hipLaunchKernelGGL(rt_reduce<UU>, grid, block, 0, s, a, c, (int)n);                                \
    break;
  switch (U) {
    SA_RT_CASE(1) SA_RT_CASE(2) SA_RT_CASE(3) SA_RT_CASE(4)
    SA_RT_CASE(5) SA_RT_CASE(6) SA_RT_CASE(7) SA_RT_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef SA_RT_CASE
  return hipGetLastError();
}

thread_local char g_rt_err[256] = "";

int32_t rt_fail(int32_t code, const char *msg) {
  snprintf(g_rt_err, sizeof g_rt_err, "%s", msg);
  return code;
}

}  // namespace

// shared with the instruction-cost microbenchmarks (sa_cpi.hip)
namespace sa_rt_detail {
int32_t fail(int32_t code, const char *msg) { return rt_fail(code, msg); }
}  // namespace sa_rt_detail

extern "C" {

const char *sa_rt_last_error(void) { return g_rt_err; }

int64_t sa_rt_grid(int32_t family, int64_t n, int32_t T, int32_t U, int32_t n_cu) {
  if (T < 1 || T > 1024 || U < 1 || U > 8 || n_cu < 1) return -1;
  switch (family) {
    case SA_RT_MATVEC:
      if (n < 1 || n % kLcmUnroll || n > 65520) return -1;
      return ceil_div(n, T) * (n / kLcmUnroll);
    case SA_RT_STENCIL:
      if (n < 3 || n > 32768) return -1;
      return stride_grid((n - 2) * ceil_div(n - 2, U), T, n_cu);
    case SA_RT_REDUCE:
      if (n < 1 || n >= (1 << 30)) return -1;
      return stride_grid(ceil_div(n, U), T, n_cu);
    default:
      return -1;
  }
}

int64_t sa_rt_trips(int32_t family, int64_t n, int32_t T, int32_t U, int64_t G, int32_t loop) {
  if (T < 1 || U < 1 || G < 1) return -1;
  switch (family) {
    case SA_RT_MATVEC:
      return loop == 0 ? kLcmUnroll / U : -1;
    case SA_RT_STENCIL:
      return loop == 0 ? ceil_div((n - 2) * ceil_div(n - 2, U), G * T) : -1;
    case SA_RT_REDUCE: {
      if (loop == 0) return ceil_div(n, G * T * (int64_t)U);
      if (loop == 1) {
        int h = 1, steps = 0;
        while (h < T) h <<= 1;
        for (int s = h >> 1; s > 0; s >>= 1) ++steps;
        return steps;
      }
      return -1;
    }
    default:
      return -1;
  }
}

size_t sa_rt_buffer_floats(int32_t family, int64_t n, int32_t which) {
  if (n < 1) return 0;
  switch (family) {
    case SA_RT_MATVEC: return which == 0 ? (size_t)(n * n) : (size_t)n;
    case SA_RT_STENCIL: return which == 1 ? 0 : (size_t)(n * n);
    case SA_RT_REDUCE: return which == 0 ? (size_t)n : (which == 2 ? 1 : 0);
    default: return 0;
  }
}

int32_t sa_rt_measure(int32_t family, int64_t n, const float *a, const float *b, float *c, const int32_t *T,
                      const int32_t *U, int32_t n_cfg, int32_t n_cu, int32_t warmup, int32_t reps, int32_t keep,
                      float *ms_out, void *stream) {
  if (!T || !U || !ms_out || n_cfg < 0) return rt_fail(-1, "NULL argument or negative count");
  if (reps < 1 || reps > 64 || keep < 1 || keep > reps || warmup < 0) return rt_fail(-1, "bad repetition counts");
  if (!a || !c || (family == SA_RT_MATVEC && !b)) return rt_fail(-1, "missing buffer");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t ev[2 * 64];
  for (int i = 0; i < 2 * reps; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
      return rt_fail(-5, "hipEventCreate failed");
    }
  int32_t status = 0;
  std::vector<float> t(reps);
  for (int32_t ci = 0; ci < n_cfg && status == 0; ++ci) {
    const int64_t G = sa_rt_grid(family, n, T[ci], U[ci], n_cu);
    if (G < 1) {
      status = rt_fail(-1, "configuration outside the family's domain");
      break;
    }
    for (int w = 0; w < warmup && status == 0; ++w)
      if (launch(family, n, T[ci], U[ci], G, a, b, c, s) != hipSuccess) status = rt_fail(-5, "launch failed");
    for (int r = 0; r < reps && status == 0; ++r) {
      if (hipEventRecord(ev[2 * r], s) != hipSuccess ||
          launch(family, n, T[ci], U[ci], G, a, b, c, s) != hipSuccess ||
          hipEventRecord(ev[2 * r + 1], s) != hipSuccess)
        status = rt_fail(-5, "launch or event record failed");
    }
    if (status) break;
    if (hipEventSynchronize(ev[2 * reps - 1]) != hipSuccess) {
      status = rt_fail(-5, "hipEventSynchronize failed");
      break;
    }
    for (int r = 0; r < reps && status == 0; ++r)
      if (hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]) != hipSuccess)
        status = rt_fail(-5, "hipEventElapsedTime failed");
    if (status) break;
    std::sort(t.begin(), t.end());
    ms_out[ci] = t[keep - 1];
  }
  for (int i = 0; i < 2 * reps; ++i) (void)hipEventDestroy(ev[i]);
  return status;
}

}  // extern "C"
