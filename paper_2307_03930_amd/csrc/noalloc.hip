// rosko_spmm_noalloc: the sparse SpMM for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, hosts
// that forbid allocation).  The only device memory rosko_spmm needs beyond
// A, B and C is the K-split partial tiles of its workspace; here they live in
// a file-scope device array of fixed size, one copy per GPU, held until the
// process ends.  Its device address is looked up once per device with
// hipGetSymbolAddress (the array's name in host code is only a stand-in)
// and the kernels receive that address as their workspace pointer.
#include <algorithm>
#include <mutex>

#include "internal.h"

namespace rosko {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;   // ROSKO_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == ROSKO_NOALLOC_SCRATCH_BYTES, "header and library disagree");

__device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The scratch address on the current device (looked up on the first call).
int32_t scratch_address(float** out) {
  int dev = -1;
  ROSKO_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d outside the %d devices the scratch table holds", dev, kMaxDevices);
    return ROSKO_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    ROSKO_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return ROSKO_OK;
}

}  // namespace
}  // namespace rosko

using namespace rosko;

extern "C" int32_t rosko_spmm_noalloc(const rosko_packed* A, const void* B, int32_t b_dtype,
                                      int64_t N, int64_t ldb, float* C, int64_t ldc,
                                      int32_t beta, const rosko_plan* plan, void* stream) {
  clear_error();
  if (A == nullptr) {
    set_error("packed matrix is null");
    return ROSKO_EINVAL;
  }
  if (A->mr < 1 || A->mr > 256 || A->M < 0 || A->K < 0 || N < 0) {
    set_error("invalid packed matrix or N");
    return ROSKO_EINVAL;
  }
  rosko_plan p = plan ? *plan : auto_plan(A, N);
  int32_t st = normalize_plan(A, N, &p);
  if (st) return st;
  if (p.path != ROSKO_PATH_SPARSE) {
    set_error("rosko_spmm_noalloc runs the sparse path only (plan path %d)", p.path);
    return ROSKO_EUNSUPPORTED;
  }
  // partials of k_split copies of C must fit the scratch: an automatic plan
  // takes as many splits as fit (none if two do not), a caller's plan that
  // needs more is refused
  const size_t per_split = sizeof(float) * (size_t)A->M * (size_t)N;
  if (p.k_split > 1 && per_split * (size_t)p.k_split > kScratchBytes) {
    if (plan != nullptr) {
      set_error("plan needs %zu bytes of K-split partials, the no-allocation scratch holds %zu",
                per_split * (size_t)p.k_split, kScratchBytes);
      return ROSKO_ESMALLBUF;
    }
    const size_t fit = per_split ? kScratchBytes / per_split : 1;
    p.k_split = fit >= 2 ? (int32_t)std::min<size_t>(fit, (size_t)p.k_split) : 1;
  }
  float* ws = nullptr;
  size_t ws_bytes = 0;
  if (p.k_split > 1) {
    if ((st = scratch_address(&ws))) return st;
    ws_bytes = kScratchBytes;
  }
  // the same checks and kernels as rosko_spmm, with the scratch as workspace
  return rosko_spmm(A, B, b_dtype, N, ldb, C, ldc, beta, &p, ws, ws_bytes, stream);
}
