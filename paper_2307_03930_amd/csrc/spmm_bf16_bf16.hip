// Row-skipping SpMM instances: bf16 packed values, bf16 B.
#include "spmm_kernel.h"

namespace rosko {
int32_t spmm_dispatch_bf16_bf16(const SpmmArgs& g, int H, int V, int G, hipStream_t s) {
  return dispatch_tile<ROSKO_BF16, ROSKO_BF16>(g, H, V, G, s);
}
}  // namespace rosko
