// Internal interface between the network library (mlp.hip) and the
// simulator side of the surrogate (surrogate.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "npx.h"

namespace npx {
// The network's own input rows, for a producer that writes them directly:
// rows [0, rows) x columns [0, width) at x (row stride ld), each entry the
// feature standardised, (f - mean[f]) * inv_std[f], rounded to bf16 (bf16) or
// kept float, and zero in the padding (columns >= the feature count, rows >=
// the batch). sur_forward_input then runs the layers on them.
struct SurInput {
  void* x;
  int64_t ld;
  int width, rows;
  const float* mean;
  const float* inv_std;
  bool bf16;
};
npx_status sur_input(npx_sur* s, int batch, SurInput* in);
npx_status sur_forward_input(npx_sur* s, int batch, float* y, int64_t ldy, hipStream_t st);

}  // namespace npx
