// Row-skipping SpMM instances for bf16 B (all value encodings: the column
// records hold FP32 values; FP8 row scales are applied in the epilogue).
#include "spmm_kernel.h"

namespace rosko {
int32_t spmm_dispatch_bbf16(const SpmmArgs& g, int H, int V, int G, hipStream_t s) {
  return dispatch_tile<ROSKO_BF16>(g, H, V, G, s);
}
}  // namespace rosko
