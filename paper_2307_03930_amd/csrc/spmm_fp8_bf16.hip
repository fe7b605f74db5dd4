// Row-skipping SpMM instances: fp8 packed values, bf16 B.
#include "spmm_kernel.h"

namespace rosko {
int32_t spmm_dispatch_fp8_bf16(const SpmmArgs& g, int H, int V, int G, hipStream_t s) {
  return dispatch_tile<ROSKO_FP8_E4M3, ROSKO_BF16>(g, H, V, G, s);
}
}  // namespace rosko
