/*
 * CPU oracle of the static performance model -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header, table or constant with the
 * GPU library: every definition below is written out again from the paper
 * (Lim, Norris, Malony, "Autotuning GPU Kernels via Static and Predictive
 * Analysis", arXiv:1701.08547).
 *
 * What it computes, per (kernel variant, launch configuration):
 *   - the active-block bound B* = min over the warp/wave, register and
 *     shared-memory (LDS) bounds (Sec. III-A, Eq. 1, Eqs. 3-5), and the
 *     active waves W* = B* x W_B of Eq. 2;
 *   - a predicted cost built on the instruction-mix time model of Eq. 6
 *     (Sec. III-B), weighted by branch divergence (Sec. II-A) and by how far
 *     the configuration falls short of hiding latency (Eq. 2 discussion);
 *   - the k best configurations of each variant (the autotuner keeps the
 *     fastest variant, Sec. II-C; the static search ranks parameter
 *     coordinates, Sec. III-C).
 *
 * Readings where the paper is silent or garbled (all listed in the design
 * notes):
 *   - Eq. 1 maximises, not minimises, the resident blocks: B* is the largest
 *     block count every resource admits, i.e. the minimum of the bounds.
 *   - Eq. 4 as printed is degenerate; the register bound is taken from its
 *     plain definition: the largest block count whose waves fit the register
 *     file.  The file is split into `simd_per_cu` partitions (SIMDs), each
 *     with `vgprs_per_simd_lane` registers per lane and
 *     max_waves_per_cu / simd_per_cu wave slots; a wave takes its register
 *     count rounded up to `vgpr_granule` on one partition.
 *   - How a block's waves share the partitions (Eqs. 3 and 4 count a
 *     multiprocessor's warps as one pool; a partitioned unit needs a rule):
 *     a block of at most simd_per_cu waves puts each wave on a different
 *     partition, so the partitions' wave places pool; a larger block is
 *     admitted only while every partition has ceil(W_B / simd_per_cu) free
 *     places, and its waves then go round-robin over the partitions.  With
 *     w places per partition the latter admits floor(P (w - c) / W_B) + 1
 *     blocks (P partitions, c = ceil(W_B / P), w >= c).  With one partition
 *     both reduce to the pooled floor(w / W_B).
 *   - Eq. 5 takes a floor (a ceiling would admit more LDS than exists); the
 *     allocation is rounded up to `lds_granule`.
 *   - Registers = 0 or LDS = 0 means "this resource does not limit" (the
 *     third case of Eqs. 4 and 5).
 *   - The score: Eq. 6 with O_fl = fp + int ops, O_mem = loads + stores,
 *     O_ctrl split into branches (amortised by the unroll factor U) and
 *     barriers (priced per wave of the block), O_reg = register moves; the
 *     per-thread cost is multiplied by (1 + d) for divergence fraction d and
 *     by F = 1 / (eta * util), where eta = min(1, W* U / w_sat) is latency
 *     hiding and util = G / (rounds * n_cu * B*) the grid-tail utilisation.
 *
 * Two arithmetic modes:
 *   - binary64 reference (`oracle_score_f64`), the definition;
 *   - the binary32 sequence (`oracle_score_f32`): the same formula evaluated
 *     as a fixed order of binary32 operations, round-to-nearest-even, no
 *     fused multiply-add, IEEE division.  Top-k decisions are taken on these
 *     binary32 scores so that both implementations decide in one precision.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Target descriptor: the paper's per-GPU limits (Table I) and instruction
 * weights (Table II), generalised so the same description covers the paper's
 * NVIDIA parts (one register pool per SM) and CDNA parts (four SIMDs). */
typedef struct {
  int32_t n_cu;                  /* mp: multiprocessors / compute units          */
  int32_t wave_size;             /* T_W: threads per warp / wave                 */
  int32_t max_threads_per_block; /* T_B                                          */
  int32_t max_waves_per_cu;      /* W_mp                                         */
  int32_t max_blocks_per_cu;     /* B_mp                                         */
  int32_t single_wave_exempt;    /* 1: one-wave blocks are not counted by B_mp   */
  int32_t simd_per_cu;           /* register-file partitions per CU              */
  int32_t vgprs_per_simd_lane;   /* registers per lane in one partition          */
  int32_t vgpr_granule;          /* register allocation unit per thread          */
  int32_t max_vgprs_per_thread;  /* R_T                                          */
  int32_t lds_per_cu;            /* shared-memory pool per CU (S_mp)             */
  int32_t lds_granule;           /* shared-memory allocation unit                */
  int32_t max_lds_per_block;     /* S_B                                          */
  int32_t w_sat;                 /* waves x unroll needed to hide latency        */
  int32_t max_unroll;            /* largest legal unroll factor                  */
  int32_t max_grid;              /* largest legal grid (blocks)                  */
  float cpi_fp, cpi_int, cpi_mem, cpi_ctrl, cpi_sync, cpi_reg; /* c_f, ..., c_r  */
} oracle_arch;

#define OR_COUNT_MAX ((int32_t)1 << 24) /* counts must be < 2^24               */
#define OR_BAR_MAX ((int32_t)1 << 14)   /* barrier count must be <= 2^14        */
#define OR_INF_BLOCKS ((int64_t)1 << 40)

static int64_t or_ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t or_round_up(int64_t a, int64_t g) { return or_ceil_div(a, g) * g; }
static int64_t or_min(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t or_max(int64_t a, int64_t b) { return a > b ? a : b; }

/* A variant whose counts fall outside the documented range makes every one of
 * its configurations illegal (never an undefined result). */
static int or_variant_valid(int32_t n_fp, int32_t n_int, int32_t n_ld, int32_t n_st,
                            int32_t n_br, int32_t n_bar, int32_t n_reg, float d) {
  if (n_fp < 0 || n_fp >= OR_COUNT_MAX) return 0;
  if (n_int < 0 || n_int >= OR_COUNT_MAX) return 0;
  if (n_ld < 0 || n_ld >= OR_COUNT_MAX) return 0;
  if (n_st < 0 || n_st >= OR_COUNT_MAX) return 0;
  if (n_br < 0 || n_br >= OR_COUNT_MAX) return 0;
  if (n_reg < 0 || n_reg >= OR_COUNT_MAX) return 0;
  if (n_bar < 0 || n_bar > OR_BAR_MAX) return 0;
  if (!(d >= 0.0f && d <= 1.0f)) return 0; /* also rejects NaN */
  return 1;
}

/* Blocks of W_B waves that partitions with w wave places each admit. */
static int64_t or_blocks_on_partitions(const oracle_arch *a, int64_t w, int64_t W_B) {
  int64_t P = a->simd_per_cu;
  if (W_B <= P) return (P * w) / W_B;
  int64_t c = or_ceil_div(W_B, P);
  return w >= c ? (P * (w - c)) / W_B + 1 : 0;
}

/* Eq. 3: blocks allowed by the wave slots of one CU, including the block-slot
 * limit B_mp (waived for one-wave blocks when the target says so). */
static int64_t or_G_W(const oracle_arch *a, int64_t W_B) {
  int64_t by_waves = or_blocks_on_partitions(a, a->max_waves_per_cu / a->simd_per_cu, W_B);
  int64_t by_slots = (W_B == 1 && a->single_wave_exempt) ? OR_INF_BLOCKS : a->max_blocks_per_cu;
  return or_min(by_slots, by_waves);
}

/* Eq. 4, plain reading: waves that fit one partition's register file, capped
 * by its wave slots, then whole blocks over the partitions. */
static int64_t or_G_R(const oracle_arch *a, int64_t R, int64_t W_B) {
  if (R == 0) return OR_INF_BLOCKS;           /* no register demand: not limiting */
  if (R > a->max_vgprs_per_thread) return 0;  /* beyond the per-thread maximum  */
  int64_t per_wave = or_round_up(R, a->vgpr_granule);
  int64_t slots = a->max_waves_per_cu / a->simd_per_cu;
  int64_t waves_per_simd = or_min(slots, a->vgprs_per_simd_lane / per_wave);
  return or_blocks_on_partitions(a, waves_per_simd, W_B);
}

/* Eq. 5 with a floor: blocks whose LDS allocations fit the per-CU pool. */
static int64_t or_G_S(const oracle_arch *a, int64_t S) {
  if (S == 0) return OR_INF_BLOCKS;
  if (S > a->max_lds_per_block) return 0;
  return a->lds_per_cu / or_round_up(S, a->lds_granule);
}

/* Eq. 1 and Eq. 2.  Returns B* (0 when the launch is illegal); *W_B_out gets
 * the waves per block. */
static int64_t or_active_blocks(const oracle_arch *a, int32_t T, int32_t R, int32_t S,
                                int64_t *W_B_out) {
  *W_B_out = 0;
  if (T < 1 || T > a->max_threads_per_block) return 0;
  if (R < 0 || S < 0) return 0;
  int64_t W_B = or_ceil_div(T, a->wave_size);
  *W_B_out = W_B;
  int64_t g_w = or_G_W(a, W_B);
  int64_t g_r = or_G_R(a, R, W_B);
  int64_t g_s = or_G_S(a, S);
  return or_min(g_w, or_min(g_r, g_s));
}

static int or_config_legal(const oracle_arch *a, int32_t U, const int32_t *G) {
  if (U < 1 || U > a->max_unroll) return 0;
  if (G && (*G < 1 || *G > a->max_grid)) return 0;
  return 1;
}

/* Occupancy bound in waves per CU, W* = B* x W_B (Eq. 2's numerator); 0 for
 * an illegal (variant, configuration).  `G` may be NULL (no grid dimension). */
int32_t oracle_occupancy(const oracle_arch *a, int32_t T, int32_t U, int32_t R,
                         const int32_t *G, int32_t S, int32_t variant_valid) {
  if (!variant_valid || !or_config_legal(a, U, G)) return 0;
  int64_t W_B;
  int64_t B = or_active_blocks(a, T, R, S, &W_B);
  return (int32_t)(B * W_B);
}

int32_t oracle_active_blocks(const oracle_arch *a, int32_t T, int32_t R, int32_t S) {
  int64_t W_B;
  return (int32_t)or_active_blocks(a, T, R, S, &W_B);
}

/* Latency-hiding / grid-tail factor F = num / den (see header).  Requires B* >= 1. */
static void or_F_terms(const oracle_arch *a, int64_t B, int64_t W_B, int32_t U,
                       const int32_t *G, int64_t *num, int64_t *den) {
  int64_t x = B * W_B * (int64_t)U; /* W* x U */
  int64_t hide = or_max(a->w_sat, x);
  if (!G) {
    *num = hide;
    *den = x;
  } else {
    int64_t cap = (int64_t)a->n_cu * B;      /* blocks resident on the whole GPU */
    int64_t rounds = or_ceil_div(*G, cap);   /* waves of blocks the grid needs   */
    *num = rounds * cap * hide;
    *den = (int64_t)(*G) * x;
  }
}

/* Binary64 reference score; +inf when the configuration is illegal. */
double oracle_score_f64(const oracle_arch *a, int32_t n_fp, int32_t n_int, int32_t n_ld,
                        int32_t n_st, int32_t n_br, int32_t n_bar, int32_t n_reg, int32_t S,
                        float d, int32_t T, int32_t U, int32_t R, const int32_t *G) {
  if (!or_variant_valid(n_fp, n_int, n_ld, n_st, n_br, n_bar, n_reg, d)) return INFINITY;
  if (!or_config_legal(a, U, G)) return INFINITY;
  int64_t W_B;
  int64_t B = or_active_blocks(a, T, R, S, &W_B);
  if (B == 0) return INFINITY;
  /* Eq. 6: f = c_f O_fl + c_m O_mem + c_b O_ctrl + c_r O_reg */
  double O_fl = (double)a->cpi_fp * n_fp + (double)a->cpi_int * n_int;
  double O_mem = (double)a->cpi_mem * ((double)n_ld + (double)n_st);
  double O_ctrl = (double)a->cpi_ctrl * n_br / U + (double)a->cpi_sync * ((double)n_bar * W_B);
  double O_reg = (double)a->cpi_reg * n_reg;
  double E = (O_fl + O_mem + O_ctrl + O_reg) * (1.0 + (double)d);
  int64_t num, den;
  or_F_terms(a, B, W_B, U, G, &num, &den);
  return E * ((double)num / (double)den);
}

/* The binary32 sequence.  Every statement is one binary32 operation (or an
 * exact integer step); -ffp-contract=off keeps them unfused. */
float oracle_score_f32(const oracle_arch *a, int32_t n_fp, int32_t n_int, int32_t n_ld,
                       int32_t n_st, int32_t n_br, int32_t n_bar, int32_t n_reg, int32_t S,
                       float d, int32_t T, int32_t U, int32_t R, const int32_t *G) {
  if (!or_variant_valid(n_fp, n_int, n_ld, n_st, n_br, n_bar, n_reg, d)) return INFINITY;
  if (!or_config_legal(a, U, G)) return INFINITY;
  int64_t W_B;
  int64_t B = or_active_blocks(a, T, R, S, &W_B);
  if (B == 0) return INFINITY;
  /* per-variant part */
  float s1 = a->cpi_fp * (float)n_fp;
  float s2 = a->cpi_int * (float)n_int;
  float s3 = a->cpi_mem * (float)(n_ld + n_st);
  float s6 = a->cpi_reg * (float)n_reg;
  float P = s1 + s2;
  P = P + s3;
  P = P + s6;
  float A4 = a->cpi_ctrl * (float)n_br;
  float D = 1.0f + d;
  /* per-configuration part */
  float a4 = A4 / (float)U;
  float a5 = a->cpi_sync * (float)((int32_t)(n_bar * W_B));
  float E = P + a4;
  E = E + a5;
  float Ed = E * D;
  int64_t num, den;
  or_F_terms(a, B, W_B, U, G, &num, &den);
  float F = (float)num / (float)den;
  return Ed * F;
}

/* ---------------------------------------------------------------- batches */

/* Total order used for selection: smaller score first, then smaller local
 * index.  Scores are compared as binary32 values (all legal scores are
 * finite and >= 0). */
typedef struct {
  float score;
  int32_t idx;
} or_key;

static int or_key_cmp(const void *pa, const void *pb) {
  const or_key *a = (const or_key *)pa, *b = (const or_key *)pb;
  if (a->score < b->score) return -1;
  if (a->score > b->score) return 1;
  return (a->idx > b->idx) - (a->idx < b->idx);
}

/* Selection for one segment: sort the legal entries, keep the first k. */
static void or_topk_segment(const float *score, int64_t n, int32_t k, int32_t *idx, float *val,
                            or_key *scratch) {
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i)
    if (score[i] < INFINITY) { /* excludes +inf (illegal) and NaN */
      scratch[m].score = score[i];
      scratch[m].idx = (int32_t)i;
      ++m;
    }
  qsort(scratch, (size_t)m, sizeof(or_key), or_key_cmp);
  for (int32_t j = 0; j < k; ++j) {
    if (j < m) {
      idx[j] = scratch[j].idx;
      if (val) val[j] = scratch[j].score;
    } else {
      idx[j] = -1;
      if (val) val[j] = INFINITY;
    }
  }
}

/* Segmented top-k over given keys (CSR `seg`, n_var + 1 offsets). */
int oracle_topk(const float *keys, const int64_t *seg, int64_t n_var, int32_t k, int32_t *idx,
                float *val, int32_t nthreads) {
  int64_t maxlen = 0;
  for (int64_t v = 0; v < n_var; ++v) maxlen = or_max(maxlen, seg[v + 1] - seg[v]);
  int failed = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    or_key *scratch = (or_key *)malloc(sizeof(or_key) * (size_t)(maxlen > 0 ? maxlen : 1));
    if (!scratch) {
#pragma omp atomic write
      failed = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t v = 0; v < n_var; ++v)
        or_topk_segment(keys + seg[v], seg[v + 1] - seg[v], k, idx + v * k, val ? val + v * k : NULL,
                        scratch);
      free(scratch);
    }
  }
  return failed ? -1 : 0;
}

/* Whole model over a CSR batch.  Variant arrays have n_var entries; config
 * arrays have seg[n_var] entries; `grid` may be NULL.  Any output may be NULL.
 * k <= 0 or idx == NULL skips the selection. */
int oracle_run(const oracle_arch *a, const int32_t *n_fp, const int32_t *n_int,
               const int32_t *n_ld, const int32_t *n_st, const int32_t *n_br, const int32_t *n_bar,
               const int32_t *n_reg, const int32_t *lds, const float *div, const int64_t *seg,
               const int32_t *block, const int32_t *unroll, const int32_t *regs,
               const int32_t *grid, int64_t n_var, int32_t *occ, float *score32, double *score64,
               int32_t k, int32_t *idx, float *val, int32_t nthreads) {
  int64_t maxlen = 0;
  for (int64_t v = 0; v < n_var; ++v) maxlen = or_max(maxlen, seg[v + 1] - seg[v]);
  int want_topk = (k > 0 && idx != NULL);
  int failed = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    float *seg_scores = NULL;
    or_key *scratch = NULL;
    if (want_topk) {
      seg_scores = (float *)malloc(sizeof(float) * (size_t)(maxlen > 0 ? maxlen : 1));
      scratch = (or_key *)malloc(sizeof(or_key) * (size_t)(maxlen > 0 ? maxlen : 1));
      if (!seg_scores || !scratch) {
#pragma omp atomic write
        failed = 1;
      }
    }
#pragma omp for schedule(dynamic, 1)
    for (int64_t v = 0; v < n_var; ++v) {
      int32_t nreg = n_reg ? n_reg[v] : 0;
      int32_t valid =
          or_variant_valid(n_fp[v], n_int[v], n_ld[v], n_st[v], n_br[v], n_bar[v], nreg, div[v]);
      for (int64_t e = seg[v]; e < seg[v + 1]; ++e) {
        const int32_t *G = grid ? &grid[e] : NULL;
        if (occ) occ[e] = oracle_occupancy(a, block[e], unroll[e], regs[e], G, lds[v], valid);
        float s32 = 0.0f;
        if (score32 || want_topk)
          s32 = oracle_score_f32(a, n_fp[v], n_int[v], n_ld[v], n_st[v], n_br[v], n_bar[v], nreg,
                                 lds[v], div[v], block[e], unroll[e], regs[e], G);
        if (score32) score32[e] = s32;
        if (score64)
          score64[e] = oracle_score_f64(a, n_fp[v], n_int[v], n_ld[v], n_st[v], n_br[v], n_bar[v],
                                        nreg, lds[v], div[v], block[e], unroll[e], regs[e], G);
        if (want_topk && seg_scores) seg_scores[e - seg[v]] = s32;
      }
      if (want_topk && seg_scores && scratch)
        or_topk_segment(seg_scores, seg[v + 1] - seg[v], k, idx + v * k, val ? val + v * k : NULL,
                        scratch);
    }
    free(seg_scores);
    free(scratch);
  }
  return failed ? -1 : 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Per-configuration terms of the model, binary64, for the learned
 * correction's features: out[9 i + 0..8] = W_B, G_W, G_R, G_S, B*, W*, E', F,
 * score (E', F and score are +inf / 0 for illegal configurations; unbounded
 * G_R / G_S are reported as 2^40).  `G` may be NULL. */
void oracle_terms(const oracle_arch *a, int32_t n_fp, int32_t n_int, int32_t n_ld, int32_t n_st, int32_t n_br,
                  int32_t n_bar, int32_t n_reg, int32_t S, float d, int64_t n, const int32_t *T,
                  const int32_t *U, const int32_t *R, const int32_t *G, double *out) {
  for (int64_t i = 0; i < n; ++i) {
    double *o = out + 9 * i;
    const int32_t *g = G ? &G[i] : NULL;
    int64_t W_B = or_ceil_div(T[i] > 0 ? T[i] : 1, a->wave_size);
    o[0] = (double)W_B;
    o[1] = (double)or_G_W(a, W_B);
    o[2] = (double)(R[i] >= 0 ? or_G_R(a, R[i], W_B) : 0);
    o[3] = (double)(S >= 0 ? or_G_S(a, S) : 0);
    int64_t Wb2;
    int valid = or_variant_valid(n_fp, n_int, n_ld, n_st, n_br, n_bar, n_reg, d) && or_config_legal(a, U[i], g);
    int64_t B = valid ? or_active_blocks(a, T[i], R[i], S, &Wb2) : 0;
    o[4] = (double)B;
    o[5] = (double)(B * W_B);
    if (B == 0) {
      o[6] = INFINITY;
      o[7] = 0.0;
      o[8] = INFINITY;
      continue;
    }
    double O_fl = (double)a->cpi_fp * n_fp + (double)a->cpi_int * n_int;
    double O_mem = (double)a->cpi_mem * ((double)n_ld + (double)n_st);
    double O_ctrl = (double)a->cpi_ctrl * n_br / U[i] + (double)a->cpi_sync * ((double)n_bar * W_B);
    double O_reg = (double)a->cpi_reg * n_reg;
    double E = (O_fl + O_mem + O_ctrl + O_reg) * (1.0 + (double)d);
    int64_t num, den;
    or_F_terms(a, B, W_B, U[i], g, &num, &den);
    double F = (double)num / (double)den;
    o[6] = E;
    o[7] = F;
    o[8] = E * F;
  }
}
