// Internal interface between the C-ABI layer (sa_api.hip) and the gfx950
// kernels (sa_eval.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa.h"

namespace sa {

constexpr int kWaveSize = 64;           // gfx950 wavefront
constexpr int kWavesPerBlock = 4;       // independent waves per workgroup
constexpr int kBlockThreads = kWaveSize * kWavesPerBlock;
constexpr int kItems = 4;               // rows of 64 evaluations in flight per wave
constexpr int kCandCap = 512;           // candidate keys buffered per wave (LDS)
constexpr int kTabBMax = 16384;         // occupancy table entries (bytes, dynamic LDS)
constexpr int kMaxWB = 64;              // largest waves-per-block the tables hold
constexpr int kMaxUnroll = 64;
constexpr int32_t kTileMin = 1024;      // evaluations per wave-tile, smallest
constexpr int32_t kTileMax = 65536;
constexpr int32_t kTileDefault = 8192;

// Blocks of WB waves admitted by `simd` partitions with w wave places each
// (Eqs. 3-4 on a partitioned CU): up to `simd` waves a block puts each wave
// on a different partition and the places pool; a larger block needs
// c = ceil(WB / simd) free places on every partition and deals its waves
// round-robin, which admits floor(simd (w - c) / WB) + 1 blocks.
__host__ __device__ inline int32_t blocks_on_partitions(int32_t w, int32_t WB, int32_t simd) {
  if (WB <= simd) return simd * w / WB;
  const int32_t c = (WB + simd - 1) / simd;
  return w >= c ? simd * (w - c) / WB + 1 : 0;
}

// The same without a division: simd = 2^simd_shift, mwb = ceil(2^16 / WB)
// (floor(x mwb / 2^16) = floor(x / WB) for x < 1024, and x <= simd x max
// waves per partition stays below that).
__host__ __device__ inline int32_t blocks_on_partitions_m(int32_t w, int32_t WB, int32_t simd_shift, uint32_t mwb) {
  const int32_t simd = 1 << simd_shift;
  if (WB <= simd) return (int32_t)(((uint32_t)(w << simd_shift) * mwb) >> 16);
  const int32_t c = (WB + simd - 1) >> simd_shift;
  return w >= c ? (int32_t)(((uint32_t)((w - c) << simd_shift) * mwb) >> 16) + 1 : 0;
}

// Descriptor as the kernels read it: the public fields plus the sizes and
// division constants the host derives from them once per call.
struct KArch {
  int32_t n_cu, ws, max_threads, max_waves, max_blocks, exempt, simd, vgprs, vgpr_gran, max_vgprs;
  int32_t lds_cu, lds_gran, max_lds, w_sat, max_unroll, max_grid;
  float cfp, cint, cmem, cctrl, csync, creg;
  int32_t nw;      // ceil(max_threads / ws): largest W_B
  int32_t nr;      // ceil(max_vgprs / vgpr_gran): largest register granule count
  int32_t ws_shift;    // log2(ws)         (wave size is a power of two)
  int32_t gran_shift;  // log2(vgpr_gran)  (register granule is a power of two)
  int32_t simd_shift;  // log2(simd)       (partition count is a power of two)
};

struct KVariants {
  const int32_t *n_fp, *n_int, *n_ld, *n_st, *n_br, *n_bar, *n_reg, *lds;
  const float *div;
};

struct KConfigs {
  const int64_t *seg;
  const int32_t *block, *unroll, *regs, *grid;
};

struct EvalLaunch {
  KArch arch;
  KVariants var;
  KConfigs cfg;
  const float *keys;      // sa_topk input (keys mode)
  int64_t n_var, n_evals;
  int32_t *occ;           // optional outputs
  float *score;
  int32_t *topk_idx;
  float *topk_val;
  uint64_t *frag;         // 2 slots of k keys per wave-tile
  int32_t k;
  int32_t tile;           // evaluations per wave-tile
  int64_t n_tiles;
  int32_t need_score;
  int32_t vec;            // every streamed column 16-byte aligned: vector loads
  int32_t tab_wsimd_off;  // dynamic LDS layout of the occupancy tables
  int32_t dyn_lds_bytes;
};

// Model: score the configurations; Keys: select over given keys; Suggest:
// score, selecting only within the paper's reduced search space; Product:
// score a product space shared by every variant, values derived from each
// evaluation's local index instead of loaded.
enum class Mode { Model, Keys, Suggest, Product };

// A product space for Mode::Product: value lists of block, unroll, registers
// and grid (a count of 1 and value 1 without a grid), grid fastest.
constexpr int kProductMaxValues = 64;
struct KProduct {
  int32_t n[4];
  uint32_t magic[3];  // ceil(2^32 / n) for grid, registers, unroll; 0 when n = 1
  int32_t size;       // n[0] n[1] n[2] n[3]
  int32_t vals[4][kProductMaxValues];
};

// A plan cuts a CSR batch into workgroup items.  kind 0: whole segments
// [v0, v1) per wave.  kind 1: a range of one segment, listed as one equal
// part per wave (the first part's e0 to the last part's e1; the kernel deals
// the range's chunks to the waves in turn, so the parts give each wave's
// share of the work, not its rows), merged in LDS; `slot` < 0 means the item
// covers the whole segment, else its k keys go to fragment slot `slot` and a
// split record names the slots to combine.
struct PlanItem {
  int32_t kind;
  int32_t slot;
  int64_t v;
};
struct PlanWave {
  int64_t e0, e1;  // kind 1: this wave's equal part of the item's range
  int64_t v0, v1;  // kind 0: segments of this wave
};
struct PlanSplit {
  int64_t v;
  int64_t first_slot;
  int64_t n_slots;
  int64_t pad;
};
struct PlanDev {
  const PlanItem *items;
  const PlanWave *waves;   // n_items x wpb
  const PlanSplit *splits;
  int64_t n_items, n_splits;
  // the item queue's ticket counter (zero between launches: the workgroup
  // taking a launch's last ticket returns it to zero)
  uint32_t *queue;
};

// Launch shape of a plan: evaluations per wave part, items per lane (1, 2,
// 4: 16-, 8- or 4-byte loads), waves per workgroup (4, 8, 16).
struct PlanShape {
  int32_t tile, items, wpb;
};

// ---------------------------------------------------------------- learned correction

struct MlpDev {
  const uint16_t *W1, *W2, *w3;  // bf16: [128][32], [128][128], [128]
  const float *b1, *b2, *b3;     // [128], [128], [1]
  const float *mean, *inv_std;   // [24]
};

hipError_t launch_features(const EvalLaunch &L, float *feat, hipStream_t stream);
hipError_t launch_suggest(const EvalLaunch &L, uint64_t *kept, hipStream_t stream);
hipError_t launch_headroom(const EvalLaunch &L, const int32_t *block, const int32_t *regs, int64_t n, int32_t *r_star,
                           int32_t *s_star, hipStream_t stream);
hipError_t launch_corrected(const EvalLaunch &L, const MlpDev &M, bool has_grid, hipStream_t stream);
hipError_t launch_mlp_fwd(const MlpDev &M, const float *feat, int64_t n, float *delta, hipStream_t stream);

hipError_t launch_eval(const EvalLaunch &L, Mode mode, bool has_grid, bool topk, hipStream_t stream);
hipError_t launch_product(const EvalLaunch &L, const KProduct &P, bool has_grid, bool topk, hipStream_t stream);
hipError_t launch_plan(const EvalLaunch &L, const PlanDev &P, const PlanShape &S, Mode mode, bool has_grid, bool topk,
                       int n_cu, hipStream_t stream);
hipError_t launch_split_merge(const EvalLaunch &L, const PlanDev &P, hipStream_t stream);
hipError_t launch_merge(const EvalLaunch &L, hipStream_t stream);

}  // namespace sa
