// Host interface of the fused corrected pass beyond its launch (which
// sa_internal.h declares).
#pragma once

#include <stdint.h>

namespace sa {

// Wave-tile of the corrected pass over n_evals evaluations: the largest
// power of two from kTileMin that leaves the most loaded resident wave no
// more evaluations than kTileMin does (fewer per-piece set-ups and
// fragments, the same critical path).  Never below kTileMin, so workspace
// sized for kTileMin always suffices.
int32_t corrected_tile(int64_t n_evals, int32_t dyn_lds_bytes, bool has_grid);

}  // namespace sa
