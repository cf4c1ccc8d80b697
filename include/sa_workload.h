/*
 * Synthetic configuration rows generated on the device, for batches whose
 * rows are too many to materialise at once (the 100,000-variant streamed
 * configuration): rows are produced chunk by chunk right before they are
 * scored.  This is input generation only; it computes nothing of the model.
 */
#ifndef SA_WORKLOAD_H
#define SA_WORKLOAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Rows e0 .. e0 + n - 1 of a synthetic batch into block / unroll / regs /
 * grid (int32[n] device arrays; grid nullable).  Column c of evaluation e is
 * drawn from u = SplitMix64 output number 4 e + c of the sequence seeded with
 * `seed` (state seed + (4 e + c + 1) * 0x9E3779B97F4A7C15, then the standard
 * finaliser), index i = floor((u >> 32) * n_values / 2^32):
 *   block = 64 (i + 1), i < 16;   unroll = i + 1, i < 8;
 *   regs = 16 (i + 1), i < 32;    grid = n_cu * 2^i, i < 4.
 * Asynchronous on `stream`.  Returns 0, -1 for bad arguments (n < 0,
 * e0 < 0, n_cu outside [1, 2048], a required pointer NULL), -5 if the launch
 * fails.
 */
int32_t sa_gen_configs(uint64_t seed, int64_t e0, int64_t n, int32_t n_cu, int32_t *block, int32_t *unroll,
                       int32_t *regs, int32_t *grid, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SA_WORKLOAD_H */
