// Device-side configuration rows for streamed batches too large to
// materialise (100,000 variants, ~1.3e10 evaluations): every column value of
// evaluation e is drawn from a counter-based generator, SplitMix64 (Steele,
// Lea and Flood, OOPSLA 2014) read at position 4 e + c for column c, so any
// row can be recomputed independently (the CPU replica in the workload module
// does the same).  The generator draws random numbers only: no part of the
// model is computed here.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa_workload.h"

namespace {

// Output of SplitMix64 at position k of the sequence seeded with `seed`: the
// state after k + 1 steps (seed + (k + 1) * golden gamma), finalised.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Value index in [0, n): the high 32 bits times n, high word.
__device__ __forceinline__ uint32_t pick(uint64_t u, uint32_t n) {
  return (uint32_t)(((u >> 32) * (uint64_t)n) >> 32);
}

__global__ __launch_bounds__(256) void sa_gen_configs_kernel(uint64_t seed, int64_t e0, int64_t n, int32_t n_cu,
                                                             int32_t *T, int32_t *U, int32_t *R, int32_t *G) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint64_t e = (uint64_t)(e0 + i);
    T[i] = 64 * (int32_t)(pick(splitmix64_at(seed, 4 * e + 0), 16) + 1);
    U[i] = (int32_t)pick(splitmix64_at(seed, 4 * e + 1), 8) + 1;
    R[i] = 16 * (int32_t)(pick(splitmix64_at(seed, 4 * e + 2), 32) + 1);
    if (G) G[i] = n_cu << pick(splitmix64_at(seed, 4 * e + 3), 4);
  }
}

}  // namespace

extern "C" int32_t sa_gen_configs(uint64_t seed, int64_t e0, int64_t n, int32_t n_cu, int32_t *block, int32_t *unroll,
                                  int32_t *regs, int32_t *grid, void *stream) {
  if (n < 0 || e0 < 0 || n_cu < 1 || n_cu > 2048) return -1;
  if (n == 0) return 0;
  if (!block || !unroll || !regs) return -1;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(sa_gen_configs_kernel, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, seed, e0, n,
                     n_cu, block, unroll, regs, grid);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}
