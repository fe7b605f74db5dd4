// Row-skipping SpMM instances: f32 packed values, f32 B.
#include "spmm_kernel.h"

namespace rosko {
int32_t spmm_dispatch_f32_f32(const SpmmArgs& g, int H, int V, int G, hipStream_t s) {
  return dispatch_tile<ROSKO_F32, ROSKO_F32>(g, H, V, G, s);
}
}  // namespace rosko
