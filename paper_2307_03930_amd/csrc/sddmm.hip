// dA for C = A*B: the gradient of every kept entry (m, k) of A is the dot
// product of dC row m with B row k; pruned entries get none (an SDDMM on A's
// mask), and the result is written in A's packed order so it lines up with
// the packed values.
//
// A workgroup takes one panel; its wavefronts stride over the panel's kept
// columns.  For a column the wave keeps the selected B row in registers
// (lanes over N) and reuses it for every value of the column, which is the
// column-wise reuse the packed format exposes; each value's dot product is
// finished with a wave reduction.
#include "internal.h"

namespace rosko {
namespace {

constexpr int kSdW = 4;        // waves per workgroup
constexpr int kSdMaxV = 32;    // B values held per lane (N <= 2048 in registers)

template <int VB>
__global__ void __launch_bounds__(64 * kSdW)
k_sddmm(const int64_t* __restrict__ panel_col_ptr, const int32_t* __restrict__ col_ind,
        const int32_t* __restrict__ col_nnz, const int64_t* __restrict__ col_ptr,
        const uint8_t* __restrict__ loc, int64_t M, int32_t mr, const float* __restrict__ dC,
        int64_t lddc, const float* __restrict__ B, int64_t ldb, int64_t N,
        float* __restrict__ dA) {
  const int64_t p = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t c_lo = panel_col_ptr[p], c_hi = panel_col_ptr[p + 1];
  for (int64_t c = c_lo + wid; c < c_hi; c += kSdW) {
    const int64_t k = col_ind[c];
    const int n = col_nnz[c];
    const int64_t z0 = col_ptr[c];
    const float* brow = B + k * ldb;
    float b[VB];
#pragma unroll
    for (int j = 0; j < VB; ++j) {
      const int64_t col = lane + 64 * j;
      b[j] = (col < N) ? brow[col] : 0.0f;
    }
    for (int t = 0; t < n; ++t) {
      const int64_t z = z0 + t;
      const int64_t m = p * mr + loc[z];
      const float* g = dC + m * lddc;
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j < VB; ++j) {
        const int64_t col = lane + 64 * j;
        if (col < N) acc = fmaf(g[col], b[j], acc);
      }
      // lanes beyond N in the register window contribute exact zeros
      for (int64_t base = 64 * VB; base < N; base += 64) {
        const int64_t col = base + lane;
        if (col < N) acc = fmaf(g[col], brow[col], acc);
      }
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
      if (lane == 0) dA[z] = acc;
    }
  }
}

}  // namespace

int32_t launch_sddmm(const rosko_packed* A, const float* dC, int64_t lddc, const float* B,
                     int64_t ldb, int64_t N, float* dA_val, hipStream_t s) {
  if (A->n_panels == 0) return ROSKO_OK;
  const int64_t vb = ceil_div(N, 64);
#define RK_SD(VB_)                                                                          \
  hipLaunchKernelGGL(k_sddmm<VB_>, dim3((unsigned)A->n_panels), dim3(64 * kSdW), 0, s,       \
                     A->panel_col_ptr, A->col_ind, A->col_nnz, A->col_ptr, A->loc, A->M,     \
                     A->mr, dC, lddc, B, ldb, N, dA_val)
  if (vb <= 1) RK_SD(1);
  else if (vb <= 4) RK_SD(4);
  else if (vb <= 16) RK_SD(16);
  else RK_SD(kSdMaxV);
#undef RK_SD
  ROSKO_LAUNCH_CHECK("k_sddmm");
  return ROSKO_OK;
}

}  // namespace rosko
