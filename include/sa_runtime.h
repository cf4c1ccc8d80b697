/*
 * Measured-runtime dataset for the learned correction of the static model:
 * three parametric kernel families compiled for gfx950, and a native timing
 * harness.
 *
 * The paper tunes kernels by running every candidate configuration and
 * timing it (Sec. IV-A: one warm-up, ten timed runs, a fixed order statistic
 * kept); its static model exists to avoid that cost.  This library produces
 * such measurements for its own kernels so that a model correction can be
 * trained and assessed on real runtimes: configurations are the paper's
 * tuning parameters block size T (threads per block) and unroll factor U
 * (Sec. III-C, Table III), with the grid following from the problem size.
 *
 * Families (float32 data, problem size n):
 *   SA_RT_MATVEC   y += A x, A column-major n x n, n a multiple of 840, at
 *                  most 65,520; block (bx, by) covers T rows and the 840
 *                  columns of chunk by, one thread per row, one atomic add
 *                  per thread; main loop of 840 / U steps, U multiply-adds
 *                  each; G = ceil(n / T) * (n / 840).
 *   SA_RT_STENCIL  one out-of-place 5-point sweep over the interior of an
 *                  n x n grid, 3 <= n <= 32,768; a work unit is U consecutive points
 *                  of a row; grid-stride main loop.
 *   SA_RT_REDUCE   sum of n < 2^30 values; grid-stride main loop adding U values
 *                  per step, then a tree reduction in LDS (second loop) and
 *                  one atomic add per block.
 * Grid-stride families launch G = min(ceil(units / T), n_cu * max(1, 2048 / T))
 * blocks, units = the family's work units.
 *
 * Every function is synchronous on the host unless it takes a stream;
 * errors: -1 argument, -5 HIP runtime (message: sa_rt_last_error).
 */
#ifndef SA_RUNTIME_H
#define SA_RUNTIME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SA_RT_MATVEC = 0, SA_RT_STENCIL = 1, SA_RT_REDUCE = 2 };

/* Message of the last failing call on this thread. */
const char *sa_rt_last_error(void);

/* Blocks launched for (family, n, T, U) on a device of n_cu compute units;
 * -1 outside the family's domain (T in [1, 1024], U in [1, 8]). */
int64_t sa_rt_grid(int32_t family, int64_t n, int32_t T, int32_t U, int32_t n_cu);

/* Iterations each thread makes of loop `loop` (0 = main loop, 1 = the
 * reduction's tree loop) at grid G; an upper bound for threads at the
 * edges.  -1 for a loop the family does not have. */
int64_t sa_rt_trips(int32_t family, int64_t n, int32_t T, int32_t U, int64_t G, int32_t loop);

/* Floats of device buffer `which` (0 = a, 1 = b, 2 = c) the family needs at
 * size n: matvec A / x / y, stencil in / - / out, reduce in / - / out. */
size_t sa_rt_buffer_floats(int32_t family, int64_t n, int32_t which);

/* Time n_cfg configurations (T[i], U[i]) of one instance on `stream`:
 * per configuration `warmup` untimed launches, then `reps` (<= 64) launches
 * each bracketed by HIP events; ms_out[i] = the keep-th smallest duration
 * (milliseconds).  a, b, c: device buffers of sa_rt_buffer_floats floats,
 * caller-owned (inputs are read, outputs overwritten).  Blocks until the
 * timings are read. */
int32_t sa_rt_measure(int32_t family, int64_t n, const float *a, const float *b, float *c, const int32_t *T,
                      const int32_t *U, int32_t n_cfg, int32_t n_cu, int32_t warmup, int32_t reps, int32_t keep,
                      float *ms_out, void *stream);

/* Issue cost of one instruction category of Eq. 6 on the current device,
 * the counterpart of Table II (instructions per cycle per multiprocessor):
 * a microbenchmark whose instruction stream is one category runs 32 waves
 * (eight 256-thread workgroups) on every compute unit; cpi_out = elapsed
 * cycles (peak clock) x compute units / thread-instructions of the category,
 * i.e. CU-cycles per thread-instruction, from the median of `reps` (1..64)
 * timed launches after one warm-up.  Categories:
 *   SA_CPI_FP    v_fma_f32, eight independent chains
 *   SA_CPI_INT   v_add_u32, eight independent chains
 *   SA_CPI_MEM   global dword loads from a 16 KiB cache-resident buffer
 *   SA_CPI_CTRL  a uniform loop branch (with its scalar counter)
 *   SA_CPI_SYNC  workgroup barriers of four-wave workgroups
 *   SA_CPI_REG   v_mov_b32
 * buf: device buffer of at least 4,096 + 256 floats (read by SA_CPI_MEM; the
 * tail is written only on an impossible result, which keeps the work live).
 * ms_out (nullable): median launch time.  Synchronous. */
enum { SA_CPI_FP = 0, SA_CPI_INT = 1, SA_CPI_MEM = 2, SA_CPI_CTRL = 3, SA_CPI_SYNC = 4, SA_CPI_REG = 5 };
int32_t sa_rt_cpi(int32_t category, int32_t reps, float *buf, float *cpi_out, float *ms_out, void *stream);

/* Memory ceiling of a scoring pass (the bytes it must move, Sec. III's
 * per-configuration evaluation of Eqs. 1-6 reads one configuration row and
 * writes its results): a stream of n elements of four int32 input columns
 * c0..c3 and two int32 output columns, o0 = c0 + c1 and o1 = c2 ^ c3 element
 * by element (wrapping), i.e. 24 bytes per element with no other work.
 * Columns: device buffers of n int32, 16-byte aligned, caller-owned; n a
 * positive multiple of 4.  Launch shape: 256-thread workgroups, each lane
 * moving `items` (1, 2 or 4) 16-byte vectors per column per iteration;
 * blocks_per_cu = 0 covers the columns in one pass of workgroups,
 * 1..64 runs that many workgroups per compute unit over a grid-stride loop;
 * nontemporal = 1 writes the outputs with non-temporal stores (0: ordinary
 * stores).  One warm-up launch, then `reps` (1..64) launches back to back between two
 * HIP events on `stream`; ms_out = their mean duration (milliseconds).
 * Synchronous.  Returns 0, -1 on an invalid argument (nothing launched) or
 * -5 on a HIP failure; sa_rt_last_error() holds the message. */
int32_t sa_rt_stream(int64_t n, const int32_t *c0, const int32_t *c1, const int32_t *c2, const int32_t *c3,
                     int32_t *o0, int32_t *o1, int32_t items, int32_t blocks_per_cu, int32_t nontemporal,
                     int32_t reps, float *ms_out, void *stream);

/* Residency probe for the device limits behind the occupancy bound (Sec.
 * III-A, Eqs. 1-5; the per-multiprocessor limits of Table I): launches
 * n_blocks workgroups of `block` threads of a probe kernel that owns exactly
 * `vgprs` unified registers per lane (the code object declares that count)
 * with `lds_bytes` of dynamic LDS; each workgroup spins for spin_us
 * microseconds of real time and writes records[4 b .. 4 b + 3] = {start,
 * end (device real-time counter ticks), HW_ID, XCC_ID hardware registers of
 * its first wave}.  The number of workgroups one compute unit holds at once
 * is the largest number of overlapping [start, end) intervals among the
 * records of that unit.  api_blocks_per_cu (nullable) receives HIP's own
 * answer, hipOccupancyMaxActiveBlocksPerMultiprocessor, for the same
 * kernel, block size and LDS.  Supported (block rounded up to a multiple of
 * 64, vgprs): (64: 16, 24, 64, 72, 80, 128, 256, 512), (128: 16, 64, 256),
 * (192: 16, 96, 168), (256: 64, 128), (320: 16, 96, 168), (384: 16, 128),
 * (448: 16), (512: 80), (576: 16), (640: 16), (768: 16), (960: 16),
 * (1024: 64, 128).
 * lds_bytes in [0, the device's per-block LDS limit]; n_blocks in [1, 2^20];
 * spin_us in [1, 100000]; records: device int64[4 n_blocks], caller-owned.
 * Asynchronous on `stream` (the records are valid once it completes).
 * Returns 0, -1 for an argument outside these sets (nothing launched) or -5
 * on a HIP failure. */
int32_t sa_rt_residency(int32_t block, int32_t vgprs, int32_t lds_bytes, int32_t n_blocks, int32_t spin_us,
                        int64_t *records, int32_t *api_blocks_per_cu, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SA_RUNTIME_H */
