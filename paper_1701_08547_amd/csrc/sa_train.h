// Internal interface of the learned correction's training step between its
// C-ABI layer (sa_mlp_api.hip) and its kernels (sa_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sa_internal.h"

namespace sa {

// Flat parameter / gradient layout (fp32 master weights, Adam moments,
// per-workgroup gradient partials): W1 | b1 | W2 | b2 | w3 | b3 | loss.
constexpr int64_t kPartW1 = 0;
constexpr int64_t kPartB1 = kPartW1 + 128 * 32;
constexpr int64_t kPartW2 = kPartB1 + 128;
constexpr int64_t kPartB2 = kPartW2 + 128 * 128;
constexpr int64_t kPartW3 = kPartB2 + 128;
constexpr int64_t kPartB3 = kPartW3 + 128;
constexpr int64_t kPartUsed = kPartB3 + 1;  // parameters
constexpr int64_t kPartLoss = kPartUsed;    // loss (sum over the workgroup's rows)
constexpr int64_t kPartStride = 20992;      // >= kPartLoss + 1, multiple of 256

struct TrainBufs {
  float *delta;   // [n] Delta (pairwise loss: the forward before the ranking kernel)
  float *gdelta;  // [n] dL/dDelta (pairwise loss)
  float *loss;    // [n] per-row loss terms (pairwise loss)
  float *part;    // [partials][kPartStride]
};

struct TrainState {
  float *master, *m, *v;  // [kPartStride]
};

// Adam's constants; the bias corrections 1 - beta^t come either from the host
// (step > 0) or from the device counter *step_counter, which the training
// kernel advances before the update reads it (steps replayed from a captured
// graph).
struct AdamArgs {
  float lr, beta1, beta2, eps, bc1, bc2;
  float inv_n;            // scale of the summed loss entry
  double beta1_d, beta2_d;  // the betas in binary64, for 1 - beta^t as the host computes it
  int64_t *step_counter;  // nullable
};

// Workgroups (and gradient partials) of one step over n rows.
int64_t train_partials(int64_t n);

// group = 0: squared error against target; group > 0: pairwise ranking loss
// over groups of `group` consecutive rows with target = log runtime.
hipError_t launch_train_step(const MlpDev &M, TrainState S, const float *feat, const float *target, int64_t n,
                             TrainBufs T, AdamArgs h, float *grad_out, int32_t group, hipStream_t stream);

}  // namespace sa
