/*
 * sa.h -- C ABI of the MI355X (gfx950) static autotuning model.
 *
 * The library evaluates the static performance model of Lim, Norris and
 * Malony, "Autotuning GPU Kernels via Static and Predictive Analysis"
 * (arXiv:1701.08547) over batches of (kernel variant, launch configuration)
 * pairs, on the GPU:
 *
 *   occupancy  Sec. III-A, Eqs. 1-5: the active blocks B* per compute unit are
 *              the minimum of the wave-slot, register-file and shared-memory
 *              (LDS) bounds; the active waves are W* = B* x W_B (Eq. 2).
 *   score      Sec. III-B, Eq. 6: the instruction-mix cost
 *              c_f O_fl + c_m O_mem + c_b O_ctrl + c_r O_reg, weighted by
 *              branch divergence (Sec. II-A) and by a latency-hiding and
 *              grid-tail factor (occupancy is not to be used alone, Eq. 2
 *              discussion).
 *   selection  Sec. II-C / III-C: per variant, the k configurations with the
 *              smallest predicted cost (the autotuner keeps the fastest).
 *
 * Conventions for every entry point:
 *   - Pointers named in the argument structs and arrays are DEVICE pointers
 *     (hipMalloc'd or torch CUDA tensors), owned by the caller; the library
 *     never allocates, frees or retains them.  `sa_arch`, `sa_variants`,
 *     `sa_configs` themselves are host structs read during the call.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     asynchronously on it; results are valid after the stream synchronises.
 *     No entry point synchronises, allocates or copies to the host, so calls
 *     can be captured into a HIP graph.
 *   - Argument errors (NULL required pointer, negative sizes, misalignment,
 *     k outside [1, 64], too small a workspace, an unsupported descriptor)
 *     return a negative status before anything is enqueued;
 *     `sa_last_error()` then holds a message (per calling thread).
 *   - Element values are never errors: an out-of-range configuration or
 *     variant is "illegal" (occupancy 0, score +inf, never selected); see
 *     `sa_configs` and `sa_variants`.  Segment offsets that are not
 *     non-decreasing, or whose last entry differs from n_evals, give
 *     unspecified results but every memory access stays in bounds.
 *   - Layouts are structure-of-arrays; all int32/float arrays must be 4-byte
 *     aligned, int64 arrays 8-byte aligned, the workspace 256-byte aligned.
 */
#ifndef SA_H_
#define SA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sa_status;
#define SA_OK 0
#define SA_ERR_ARG (-1)         /* bad argument value or NULL required pointer */
#define SA_ERR_ALIGN (-2)       /* pointer not aligned as required            */
#define SA_ERR_NODEV (-3)       /* no HIP device visible                      */
#define SA_ERR_WORKSPACE (-4)   /* workspace missing or smaller than needed   */
#define SA_ERR_HIP (-5)         /* a HIP runtime call failed                  */
#define SA_ERR_UNSUPPORTED (-6) /* descriptor or option outside what is built */

#define SA_K_MAX 64

/*
 * Target descriptor (the paper's Table I limits and Table II weights).
 * One descriptor describes both the paper's NVIDIA parts (one register pool
 * per SM) and CDNA parts (`simd_per_cu` register-file partitions).
 *
 * Occupancy of a launch with T threads, R registers per thread and S bytes of
 * LDS per block (W_B = ceil(T / wave_size) waves per block):
 *   P = simd_per_cu partitions; a block of W_B waves is admitted by
 *   partitions with w free wave places each:
 *     f(w) = floor(P w / W_B)                 when W_B <= P (one wave per
 *                                             partition: the places pool),
 *     f(w) = floor(P (w - c) / W_B) + 1       when W_B > P and w >= c,
 *            c = ceil(W_B / P) (every partition needs c free places and the
 *            waves go round-robin), 0 when w < c;
 *   with P = 1 both are the pooled floor(w / W_B).
 *   G_W = min(B_lim, f(max_waves_per_cu / P))                (Eq. 3)
 *         B_lim = max_blocks_per_cu, unlimited when W_B = 1 and
 *         single_wave_exempt != 0
 *   G_R = f(w_v),                                            (Eq. 4, plain reading)
 *         w_v = min(max_waves_per_cu / P,
 *                   floor(vgprs_per_simd_lane / roundup(R, vgpr_granule)));
 *         unlimited when R = 0
 *   G_S = floor(lds_per_cu / roundup(S, lds_granule)),       (Eq. 5, floor)
 *         unlimited when S = 0
 *   B*  = min(G_W, G_R, G_S)                                 (Eq. 1)
 *   W*  = B* x W_B                                           (Eq. 2)
 * A launch is illegal (W* = 0) when T outside [1, max_threads_per_block],
 * R outside [0, max_vgprs_per_thread] or S outside [0, max_lds_per_block].
 *
 * Supported ranges (sa_arch_validate): wave_size a power of two in [2, 1024];
 * max_threads_per_block in [1, 65536], a multiple of wave_size, with
 * max_threads_per_block / wave_size <= 64; max_waves_per_cu in [1, 64];
 * simd_per_cu a power of two in [1, max_waves_per_cu]; max_blocks_per_cu >= 1; vgpr_granule
 * a power of two dividing max_vgprs_per_thread, with
 * (max_vgprs_per_thread / vgpr_granule + 2) x
 * (max_threads_per_block / wave_size + 2) <= 16384;
 * vgprs_per_simd_lane in [1, 65536]; lds_per_cu in [1, 2^24]; lds_granule
 * >= 1; max_lds_per_block in [0, 2^24]; n_cu in [1, 2048]; w_sat in
 * [1, 4096]; max_unroll in [1, 64]; max_grid in [1, 2^18]; every cpi_*
 * finite and >= 0.
 */
typedef struct sa_arch {
  int32_t n_cu;                  /* compute units (mp)                         */
  int32_t wave_size;             /* T_W                                        */
  int32_t max_threads_per_block; /* T_B                                        */
  int32_t max_waves_per_cu;      /* W_mp                                       */
  int32_t max_blocks_per_cu;     /* B_mp                                       */
  int32_t single_wave_exempt;    /* != 0: one-wave blocks not counted by B_mp  */
  int32_t simd_per_cu;           /* register-file partitions per CU            */
  int32_t vgprs_per_simd_lane;   /* registers per lane in one partition        */
  int32_t vgpr_granule;          /* register allocation unit (per thread)      */
  int32_t max_vgprs_per_thread;  /* R_T                                        */
  int32_t lds_per_cu;            /* LDS pool per CU, bytes                     */
  int32_t lds_granule;           /* LDS allocation unit, bytes                 */
  int32_t max_lds_per_block;     /* S_B, bytes                                 */
  int32_t w_sat;                 /* waves x unroll that hide latency           */
  int32_t max_unroll;            /* largest legal unroll factor U              */
  int32_t max_grid;              /* largest legal grid G (blocks)              */
  float cpi_fp;                  /* c_f for floating-point ops                 */
  float cpi_int;                 /* c_f for integer ops (FLOPS group)          */
  float cpi_mem;                 /* c_m for loads + stores                     */
  float cpi_ctrl;                /* c_b for branches                           */
  float cpi_sync;                /* c_b for barriers, per wave of the block    */
  float cpi_reg;                 /* c_r for register moves                     */
} sa_arch;

/*
 * Per-variant instruction mix (Sec. III-B), structure of arrays of length
 * n_variants, device pointers.  Counts are per thread.  A variant is valid
 * when every count is in [0, 2^24), n_bar in [0, 2^14] and div in [0, 1]; an
 * invalid variant makes all of its configurations illegal.
 */
typedef struct sa_variants {
  const int32_t *n_fp;      /* floating-point ops                   -> O_fl   */
  const int32_t *n_int;     /* integer ops                          -> O_fl   */
  const int32_t *n_ld;      /* loads                                -> O_mem  */
  const int32_t *n_st;      /* stores                               -> O_mem  */
  const int32_t *n_br;      /* branches                             -> O_ctrl */
  const int32_t *n_bar;     /* barriers                             -> O_ctrl */
  const int32_t *n_reg;     /* register moves (NULL = all zero)     -> O_reg  */
  const int32_t *lds_bytes; /* S: LDS bytes per block                         */
  const float *div;         /* d: divergent fraction of the instruction stream */
} sa_variants;

/*
 * Launch configurations, CSR by variant, device pointers.  `seg` has
 * n_variants + 1 non-decreasing offsets with seg[0] = 0 and
 * seg[n_variants] = n_evals; variant v owns evaluations [seg[v], seg[v+1]).
 * A configuration is legal when 1 <= unroll <= max_unroll, 1 <= grid <=
 * max_grid (when present) and its (block, regs, lds) launch is legal.
 */
typedef struct sa_configs {
  const int64_t *seg;    /* n_variants + 1                                     */
  const int32_t *block;  /* T: threads per block                              */
  const int32_t *unroll; /* U: unroll factor                                  */
  const int32_t *regs;   /* R: registers per thread                           */
  const int32_t *grid;   /* G: blocks in the grid (NULL = no grid dimension)  */
} sa_configs;

/*
 * Learned correction: a 24 -> 128 -> 128 -> 1 perceptron (GELU, bfloat16
 * weights and activations, fp32 accumulation on MFMA) that predicts, from
 * 24 static features of one (variant, configuration), the residual Delta of
 * the log-runtime the plain score misses; the corrected key is
 * ln(score) + Delta.  The paper motivates learned models over static
 * features (Sec. V, Sec. VII) without specifying one.
 *
 * Features (binary32, in this order): ln(1+n_fp), ln(1+n_int), ln(1+n_ld),
 * ln(1+n_st), ln(1+n_br), n_bar/4, ln(1+n_reg), S/65536, d, log2(T)/10,
 * (U-1)/7, R/512, log2(G/n_cu)/3 (0 without grid), W_B/16, min(G_W,32)/32,
 * min(G_R,32)/32, min(G_S,32)/32, Bstar/32, Wstar/32, ln(1+intensity), ln E',
 * 1/F, ln score, [intensity > 4]; intensity = n_fp / max(1, n_ld + n_st).
 * The network input is bf16((f - feat_mean) * feat_inv_std), padded with
 * eight zeros; h1 = bf16(GELU(W1 x + b1)), h2 = bf16(GELU(W2 h1 + b2)),
 * Delta = w3 . h2 + b3, GELU(a) = a/2 (1 + erf(a / sqrt 2)).
 */
typedef struct sa_mlp {
  const uint16_t *W1;         /* bf16 [128][32]; columns 24..31 must be zero */
  const uint16_t *W2;         /* bf16 [128][128]                              */
  const uint16_t *w3;         /* bf16 [128]                                   */
  const float *b1, *b2, *b3;  /* [128], [128], [1]                            */
  const float *feat_mean;     /* [24]                                         */
  const float *feat_inv_std;  /* [24]                                         */
} sa_mlp;

/* Flat fp32 parameter vector used by training (master weights, Adam
 * moments, gradients): W1 [128][32] | b1 | W2 [128][128] | b2 | w3 | b3,
 * then one slot holding the mean squared error, padded. */
#define SA_MLP_PARAMS 20865
#define SA_MLP_FLAT 20992

/* Human-readable name of a status code (static storage). */
const char *sa_status_string(sa_status status);

/* Message describing the last error returned on the calling thread. */
const char *sa_last_error(void);

/* CDNA4 / MI355X constants without any device query (n_cu = 256): wave 64,
 * 32 wave slots over 4 SIMDs, 512 unified VGPR/AGPR per SIMD lane (granule
 * 8), 160 KiB LDS per CU (granule 1,280 B), 16 multi-wave blocks per CU
 * (one-wave blocks exempt), w_sat 32, U <= 64, G <= 2^18, CPI 2^-6 (fp,
 * int), 2^-4 (memory, branch, barrier), 2^-5 (register moves).  The
 * occupancy constants are the ones sa_rt_residency measures on the device.
 * Fills *out; SA_ERR_ARG if out is NULL. */
sa_status sa_arch_gfx950(sa_arch *out);

/* The same, with n_cu, wave size, thread and LDS limits read from HIP device
 * `device` (hipGetDeviceProperties).  SA_ERR_NODEV without a device. */
sa_status sa_arch_default_gfx950(int device, sa_arch *out);

/* SA_OK when the descriptor is inside the supported ranges listed above. */
sa_status sa_arch_validate(const sa_arch *arch);

/* Bytes of workspace sa_score / sa_topk need for this problem size (an upper
 * bound over every tile size the library may pick).  0 when k <= 0 or
 * n_evals == 0.  `flags` is reserved (pass 0). */
size_t sa_workspace_bytes(int64_t n_variants, int64_t n_evals, int32_t k, int32_t flags);

/*
 * Occupancy only (Eqs. 1-5).  occ_waves[e] = W* of evaluation e (0 when
 * illegal), int32[n_evals].  No workspace.
 */
sa_status sa_occupancy(const sa_arch *arch, const sa_variants *variants, const sa_configs *configs,
                       int64_t n_variants, int64_t n_evals, int32_t *occ_waves, void *stream);

/*
 * Occupancy, score and per-variant top-k in one pass over the batch.
 *   score     float[n_evals] or NULL: predicted cost (+inf when illegal), the
 *             binary32 sequence
 *               P  = ((c_fp n_fp + c_int n_int) + c_mem (n_ld + n_st)) + c_reg n_reg
 *               E  = (P + (c_ctrl n_br) / U) + c_sync (n_bar W_B)
 *               E' = E (1 + d)
 *               x  = W* U;  F = max(w_sat, x) / x              (no grid)
 *                           F = (rounds cap max(w_sat, x)) / (G x),
 *                               cap = n_cu B*, rounds = ceil(G / cap)
 *               score = E' F
 *             each step rounded to nearest even, no fused multiply-add.
 *   occ_waves int32[n_evals] or NULL: W*.
 *   topk_idx  int32[n_variants * k] or NULL: for variant v, row v holds the
 *             local indices (0 .. seg[v+1]-seg[v]-1) of its k legal
 *             configurations with the smallest (score, local index), in that
 *             order; -1 past the number of legal configurations.
 *   topk_val  float[n_variants * k] or NULL: the matching scores (+inf pad).
 *   k         1 .. 64 when topk_idx or topk_val is given, else ignored.
 *   mlp       NULL for the plain model.  Non-NULL selects the fused
 *             corrected pass (the learned correction applied inside the
 *             scoring kernel): score[e] receives the corrected key
 *             z = ln(score) + Delta (Delta = the network of sa_surrogate_fwd
 *             on the 24 features of sa_features, +inf when illegal) and the
 *             top-k ranks by z with the same tie rule.  W1 and W2 must be
 *             8-byte aligned and w3 2-byte aligned (SA_ERR_ALIGN otherwise;
 *             16-byte aligned W1 and W2 are staged a whole 16 bytes at a
 *             time, others element by element, to the same result); every
 *             pointer is required.
 *   workspace device buffer of sa_workspace_bytes(...) bytes (may be NULL
 *             when no top-k is asked for).  Contents need no initialisation.
 *             Segments that span several wave-tiles leave per-tile partial
 *             results there, combined by a second kernel on the same stream.
 * Calls that share a workspace must be ordered on one stream.
 */
sa_status sa_score(const sa_arch *arch, const sa_variants *variants, const sa_configs *configs,
                   int64_t n_variants, int64_t n_evals, float *score, int32_t *occ_waves, int32_t k,
                   int32_t *topk_idx, float *topk_val, const sa_mlp *mlp, void *workspace,
                   size_t workspace_bytes, void *stream);

/*
 * sa_score for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same pass, arguments and results as sa_score, without the workspace.  Its
 * fragment slots live in a fixed array of SA_NOALLOC_SCRATCH_BYTES bytes of
 * device memory that the library holds on each GPU it runs on until the
 * process ends; the call allocates nothing.  A problem whose slots exceed
 * that array (sa_workspace_bytes-style need for the tile the pass uses: 16 k
 * bytes per 1,024 evaluations for the corrected pass, per 8,192 for the plain
 * one) returns SA_ERR_WORKSPACE before any launch.  Every call on one GPU
 * shares its array: calls that overlap in time on one GPU race (order them on
 * one stream).  Errors as sa_score.
 */
#define SA_NOALLOC_SCRATCH_BYTES (4 << 20)
sa_status sa_score_noalloc(const sa_arch *arch, const sa_variants *variants, const sa_configs *configs,
                           int64_t n_variants, int64_t n_evals, float *score, int32_t *occ_waves, int32_t k,
                           int32_t *topk_idx, float *topk_val, const sa_mlp *mlp, void *stream);

/*
 * Segmented top-k over given keys: for each segment [seg[v], seg[v+1]) of
 * keys (float[n_evals]) the k smallest finite-or-negative-infinite keys
 * (NaN and +inf are excluded), ties by smaller local index; idx
 * int32[n_variants * k] (-1 pad), val float[n_variants * k] or NULL (+inf
 * pad).  Workspace as for sa_score.
 */
sa_status sa_topk(const float *keys, const int64_t *seg, int64_t n_variants, int64_t n_evals, int32_t k,
                  int32_t *idx, float *val, void *workspace, size_t workspace_bytes, void *stream);

/*
 * The paper's search-space reduction (Sec. III-C; pruning rates Sec. IV-C):
 * T* = the block sizes, multiples of the wave size up to the thread limit,
 * at which occupancy (Eqs. 1-5) is full when registers and LDS do not limit;
 * a kernel whose intensity n_fp / max(1, n_ld + n_st) exceeds 4 keeps the
 * upper half of T* (by thread count), any other the lower half; an odd-length
 * T* drops its median.  kept uint64[n_variants] (8-byte aligned): bit j set
 * when T = wave_size * (j + 1) is kept.  Asynchronous on `stream`.
 */
sa_status sa_suggest(const sa_arch *arch, const sa_variants *variants, int64_t n_variants, uint64_t *kept,
                     void *stream);

/*
 * Search spaces that are full products (the autotuner's space of Sec. III-C,
 * every tuning parameter taking each of its values): every variant is scored
 * over the same S = n_block x n_unroll x n_regs x max(1, n_grid)
 * configurations, and no configuration rows are stored.  Local index
 * i = ((iT n_unroll + iU) n_regs + iR) max(1, n_grid) + iG (block slowest,
 * grid fastest) stands for (block[iT], unroll[iU], regs[iR], grid[iG]); evaluation
 * e = v S + i.  n_grid = 0: no grid dimension.  Value lists are host arrays,
 * read during the call (each count at most SA_PRODUCT_MAX_VALUES, S at most
 * SA_PRODUCT_MAX_SIZE).
 */
#define SA_PRODUCT_MAX_VALUES 64
#define SA_PRODUCT_MAX_SIZE (1 << 24)
typedef struct {
  int32_t n_block, n_unroll, n_regs, n_grid;
  const int32_t *block, *unroll, *regs, *grid;
} sa_product;

/* Workspace of sa_score_product with top-k output (bytes; 256-byte aligned
 * device memory): fragment slots plus the implicit segment offsets. */
size_t sa_product_workspace_bytes(int64_t n_variants, int64_t space_size, int32_t k);

/* sa_score over the materialised product, without the rows: the same
 * occupancy, score and top-k results (bit for bit) with score / occ_waves
 * indexed by e = v S + i (n_variants * S entries) and top-k indices local.
 * Errors as sa_score; an empty or oversized value list is SA_ERR_ARG; with
 * n_variants = 0 the call only checks the descriptor and the space.
 * Asynchronous on `stream`; contents of the workspace need no
 * initialisation. */
sa_status sa_score_product(const sa_arch *arch, const sa_variants *variants, int64_t n_variants,
                           const sa_product *space, float *score, int32_t *occ_waves, int32_t k, int32_t *topk_idx,
                           float *topk_val, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Headroom at full occupancy (Sec. III-C; the R* and S* columns of Table VII):
 * for the block size T = block[i] of each row, the largest register count per
 * thread and the largest LDS per workgroup at which occupancy (Eqs. 1-5) is
 * still full, the other resource not limiting.  r_star[i] = max(0, largest
 * such register count - regs[i]) (regs NULL: 0 registers in use);
 * s_star[i] = the largest such LDS size in bytes (at most the per-workgroup
 * limit).  Both are 0 when T cannot reach full occupancy, when T lies outside
 * [1, max_threads_per_block], or when regs[i] lies outside
 * [0, max_vgprs_per_thread].  block, regs, r_star, s_star: int32[n], 4-byte
 * aligned device arrays; either output may be NULL, not both.  Asynchronous
 * on `stream`.
 */
sa_status sa_headroom(const sa_arch *arch, const int32_t *block, const int32_t *regs, int64_t n, int32_t *r_star,
                      int32_t *s_star, void *stream);

/* sa_score's pass with the top-k restricted to the reduced space: only
 * evaluations whose block size is kept by sa_suggest's rule compete; the
 * optional occupancy and score outputs cover every evaluation.  k in
 * [1, SA_K_MAX]; at least one of topk_idx / topk_val.  Workspace as for
 * sa_score. */
sa_status sa_score_suggested(const sa_arch *arch, const sa_variants *variants, const sa_configs *configs,
                             int64_t n_variants, int64_t n_evals, float *score, int32_t *occ_waves, int32_t k,
                             int32_t *topk_idx, float *topk_val, void *workspace, size_t workspace_bytes,
                             void *stream);

/* The 24 features of every evaluation, feat float[n_evals][24] (features of
 * illegal evaluations are unspecified).  Asynchronous on `stream`. */
sa_status sa_features(const sa_arch *arch, const sa_variants *variants, const sa_configs *configs,
                      int64_t n_variants, int64_t n_evals, float *feat, void *stream);

/* Delta for n rows of features (float[n][24]); delta float[n]. */
sa_status sa_surrogate_fwd(const sa_mlp *mlp, const float *feat, int64_t n, float *delta, void *stream);

/* One training step on a batch of n rows: forward (the same arithmetic as
 * sa_surrogate_fwd, so Delta equals the served one), mean squared error
 * against target float[n], backward (dL/dh1 and the weight gradients dW1,
 * dW2 on the matrix cores, bf16 operands, fp32 sums; each workgroup's sums
 * added in a fixed order), and Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8,
 * bias correction for step t) on master / adam_m / adam_v
 * (float[SA_MLP_FLAT] each); the bf16 shadow weights and the biases named by
 * `mlp` are rewritten from the master.  t is `step` (>= 1) when step_counter
 * is NULL; otherwise `step` must be 0 and t is read from the device counter
 * *step_counter (int64, 8-byte aligned, caller-owned) after the step advances
 * it by one, so that steps replayed from a captured HIP graph each use their
 * own t.  grad_out (float[SA_MLP_FLAT], nullable) receives the summed
 * gradients and, at index SA_MLP_PARAMS, the batch loss.  n in [1, 2^20].
 * Workspace: sa_surrogate_train_workspace_bytes(n) bytes, 256-byte aligned. */
size_t sa_surrogate_train_workspace_bytes(int64_t n);
sa_status sa_surrogate_train_step(const sa_mlp *mlp, float *master, float *adam_m, float *adam_v, int64_t step,
                                  int64_t *step_counter, float lr, const float *feat, const float *target, int64_t n,
                                  float *grad_out, void *workspace, size_t workspace_bytes, void *stream);

/* The same step with a pairwise ranking loss instead of squared error (the
 * correction's purpose is the order of configurations, Sec. III-C): rows come
 * in groups of `group` consecutive rows (one kernel instance's
 * configurations; n a multiple of group, group in [2, SA_RANK_GROUP_MAX]).
 * With z = feat[.][22] (ln score, as computed by sa_features) + Delta, every
 * ordered pair (i, j) of a group with log_time[i] < log_time[j] costs
 * softplus(z_i - z_j) = ln(1 + e^(z_i - z_j)); the loss is the mean over each
 * group's pairs, averaged over the groups (a group of equal times adds 0).
 * grad_out's loss entry is that loss.  step / step_counter as above. */
#define SA_RANK_GROUP_MAX 1024
sa_status sa_surrogate_train_step_pairwise(const sa_mlp *mlp, float *master, float *adam_m, float *adam_v,
                                           int64_t step, int64_t *step_counter, float lr, const float *feat,
                                           const float *log_time, int64_t n, int32_t group, float *grad_out,
                                           void *workspace, size_t workspace_bytes, void *stream);

/* Tile size (evaluations per wave) the next sa_score / sa_occupancy /
 * sa_topk / sa_score_product calls on this thread use; 0 restores the
 * library's choice.  Must
 * be a multiple of 256 in [1024, 65536]. */
sa_status sa_set_tile(int32_t evals_per_wave);

/*
 * Plans: batches of uneven search spaces (segments of very different
 * lengths) scored by one persistent kernel launch.
 *
 * A plan is a host object made once per CSR layout from a HOST copy of the
 * segment offsets.  Segments longer than `tile` are cut into workgroup items
 * of up to tile x waves_per_block evaluations, whose chunks the item's waves
 * take in turn (adjacent addresses across the workgroup) and whose per-wave
 * top-k meet in LDS; shorter segments are packed whole into items and spread
 * over the waves.  A segment longer than one item leaves one
 * k-key fragment per item in the workspace, combined by a second small
 * kernel only when such segments exist.  Shape: tile a multiple of 256 in
 * [256, 2^20]; items_per_lane 1, 2 or 4 (consecutive evaluations per lane per
 * load: 4-, 8- or 16-byte accesses); waves_per_block 4, 8 or 16.
 *
 * sa_plan_create validates the offsets (seg[0] = 0, non-decreasing,
 * seg[n_variants] = n_evals) and decomposes them on the host; it makes no HIP
 * call.  The decomposition reaches the device through sa_plan_bind, which
 * copies it into a caller-owned table of sa_plan_device_bytes(plan) bytes
 * (the library allocates no device memory).  sa_plan_score / sa_plan_topk are
 * asynchronous, allocation-free and capturable, like sa_score / sa_topk; they
 * return SA_ERR_ARG for a plan that was never bound, and `seg` passed to them
 * must hold the same offsets on the device.
 */
typedef struct sa_plan sa_plan;
typedef struct sa_plan_shape {
  int32_t tile;            /* evaluations per wave of an item (its share)     */
  int32_t items_per_lane;  /* 1, 2, 4                                         */
  int32_t waves_per_block; /* 4, 8, 16                                        */
} sa_plan_shape;

sa_status sa_plan_create(const int64_t *seg_host, int64_t n_variants, int64_t n_evals, int32_t k,
                         const sa_plan_shape *shape /* NULL = 4096, 4, 4 */, sa_plan **out);
/* Frees the host object only (never the bound table, which the caller owns). */
sa_status sa_plan_destroy(sa_plan *plan);
/* Bytes of the device table of a plan (0 for a NULL plan); a multiple of 256.
 * The table holds the workgroup items (longest first), their wave parts, the
 * split records and a 256-byte item queue: with more items than the launch
 * has workgroups, the workgroups take the rest from a ticket counter there.
 * Each launch leaves the counter at zero, so launches of one plan (replays
 * of captured graphs included) must run in stream order, not concurrently. */
size_t sa_plan_device_bytes(const sa_plan *plan);
/* Copies the plan's decomposition into `table` (device memory, 256-byte
 * aligned, at least sa_plan_device_bytes(plan) bytes, caller-owned) and
 * zeroes its item queue, with hipMemcpyAsync on `stream`, and records `table` and the current device's
 * compute-unit count in the plan.  The copy reads the plan's host memory when
 * `stream` reaches it: keep the plan alive until then, and keep `table`
 * alive and unmodified while launches of the plan are pending.  Rebinding
 * to another table is allowed.  A set-up call: not for graph capture (the
 * copy's source is pageable host memory).  SA_ERR_ARG (NULL), SA_ERR_ALIGN,
 * SA_ERR_WORKSPACE (too small), SA_ERR_HIP. */
sa_status sa_plan_bind(sa_plan *plan, void *table, size_t table_bytes, void *stream);
/* The plan's decomposition computed on the host only (no device needed):
 * counts, and when the arrays are non-NULL, items (n_items x {kind, slot,
 * v}), waves (n_items x waves_per_block x {e0, e1, v0, v1}) and splits
 * (n_splits x {v, first_slot, n_slots}).  Validates like sa_plan_create. */
sa_status sa_plan_layout(const int64_t *seg_host, int64_t n_variants, int64_t n_evals, const sa_plan_shape *shape,
                         int64_t *n_items, int64_t *n_splits, int64_t *n_slots, int64_t *items, int64_t *waves,
                         int64_t *splits);
/* Shape, item and split counts, and the workspace bytes the plan needs. */
sa_status sa_plan_info(const sa_plan *plan, sa_plan_shape *shape, int64_t *n_items, int64_t *n_splits,
                       size_t *workspace_bytes);
/* sa_score over a plan: same outputs and conventions; k is the plan's. */
sa_status sa_plan_score(const sa_plan *plan, const sa_arch *arch, const sa_variants *variants,
                        const sa_configs *configs, float *score, int32_t *occ_waves, int32_t *topk_idx,
                        float *topk_val, void *workspace, size_t workspace_bytes, void *stream);
/* sa_topk over a plan. */
sa_status sa_plan_topk(const sa_plan *plan, const float *keys, const int64_t *seg, int32_t *idx, float *val,
                       void *workspace, size_t workspace_bytes, void *stream);

/*
 * Launch-shape autotuner: times sa_plan_score for every shape in
 * {1024, 2048, 4096, 8192} x {1, 2, 4} x {4, 8, 16} on the caller's buffers
 * (outputs are overwritten), `reps` timed runs each after one warm-up, on
 * `stream`, and returns the fastest shape and its median milliseconds.
 * Synchronises; creates, binds and destroys plans (host objects) inside.
 * The workspace (256-byte aligned) must hold
 * sa_plan_autotune_workspace_bytes(...) bytes: the largest fragment area of
 * the candidate shapes followed by their largest device table (0 when the
 * offsets are invalid).
 */
size_t sa_plan_autotune_workspace_bytes(const int64_t *seg_host, int64_t n_variants, int64_t n_evals, int32_t k);
sa_status sa_plan_autotune(const int64_t *seg_host, int64_t n_variants, int64_t n_evals, int32_t k,
                           const sa_arch *arch, const sa_variants *variants, const sa_configs *configs, float *score,
                           int32_t *occ_waves, int32_t *topk_idx, float *topk_val, void *workspace,
                           size_t workspace_bytes, void *stream, int32_t reps, sa_plan_shape *best, float *best_ms);

#ifdef __cplusplus
}
#endif

#endif /* SA_H_ */
