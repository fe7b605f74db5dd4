// Host side of the batched pack (rosko_pack_batch): one matrix's arguments
// after validation, and the launcher that groups the matrices whose single
// pass shares a kernel form into one grid.
#pragma once

#include "internal.h"

namespace rosko {

constexpr int32_t kPackBatchMax = ROSKO_PACK_BATCH_MAX;

struct PackTask {
  const float* A;
  int64_t R, S, lda;
  int32_t mr, val_dtype;
  void* ws;
  PackWs L;
  rosko_packed* out;
};

// Enqueues the packs of tasks[0..n) on s (the FP8 row scales already
// enqueued): each as launch_pack would, except that the single passes of
// matrices with the same value type and tile form share launches.
int32_t launch_pack_batch(const PackTask* tasks, int32_t n, hipStream_t s);

}  // namespace rosko
