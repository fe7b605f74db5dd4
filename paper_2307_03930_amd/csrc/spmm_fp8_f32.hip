// Row-skipping SpMM instances: fp8 packed values, f32 B.
#include "spmm_kernel.h"

namespace rosko {
int32_t spmm_dispatch_fp8_f32(const SpmmArgs& g, int H, int V, int G, hipStream_t s) {
  return dispatch_tile<ROSKO_FP8_E4M3, ROSKO_F32>(g, H, V, G, s);
}
}  // namespace rosko
