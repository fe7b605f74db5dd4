// Row-skipping SpMM instances for f32 B (all value encodings: the column
// records hold FP32 values; FP8 row scales are applied in the epilogue).
#include "spmm_kernel.h"

namespace rosko {
int32_t spmm_dispatch_bf32(const SpmmArgs& g, int MRt, int V, int H, int depth, hipStream_t s) {
  return dispatch_tile<ROSKO_F32>(g, MRt, V, H, depth, s);
}
}  // namespace rosko
