// Row-skipping outer-product SpMM on gfx950 (Alg. 2, Sec. 4.2).
//
// A workgroup owns one C tile: the mr rows of one panel times 64*V columns.
// Each of its W wavefronts takes a contiguous share of the panel's kept
// columns.  For a kept column the wave loads the B row it selects (lane l
// holds V consecutive columns), then for each of the column's values
// multiply-accumulates that row into C-tile row loc -- rows whose A entry is
// zero are never touched, which is the row skipping.  The C tile lives in
// VGPRs for the whole K range (the K-first schedule of Sec. 2.2 / 4.2) and is
// written once.
//
// The C row is a run-time index, yet the tile must stay in registers.  The
// tile is pinned to the fixed VGPR range v[64 : 64+MR*V) through inline-asm
// register constraints, row r of column j at v[64 + j*MR + r].  Every value
// of A is applied by one asm block: s_set_gpr_idx_on with the (wave-uniform)
// row index turns on relative addressing for the FMA's addend and result,
// V v_fma_f32 follow, and s_set_gpr_idx_off ends the mode.  The row index is
// masked to MR-1 so the relative access can never leave the pinned range.
// The wave's partial tiles are summed in LDS in a fixed order (no atomics),
// so results are reproducible bit for bit.
#include <algorithm>

#include "internal.h"

namespace rosko {
namespace {

__global__ void __launch_bounds__(256)
k_fill_zero(float* __restrict__ C, int64_t M, int64_t N, int64_t ldc) {
  const int64_t total = M * N;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const int64_t m = i / N, n = i - m * N;
    C[m * ldc + n] = 0.0f;
  }
}

}  // namespace
int32_t launch_fill_zero(float* C, int64_t M, int64_t N, int64_t ldc, hipStream_t s) {
  if (M == 0 || N == 0) return ROSKO_OK;
  const int64_t blocks = std::min<int64_t>(ceil_div(M * N, 256), 65536);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, C, M, N, ldc);
  ROSKO_LAUNCH_CHECK("k_fill_zero");
  return ROSKO_OK;
}

// Smallest supported register-tile height holding mr rows.
static int tile_height(int32_t mr) {
  if (mr <= 8) return 8;
  if (mr <= 16) return 16;
  if (mr <= 32) return 32;
  if (mr <= 64) return 64;
  if (mr <= 128) return 128;
  return 0;
}

int32_t launch_spmm_sparse(const rosko_packed* A, const void* B, int32_t b_dtype, int64_t N,
                           int64_t ldb, float* C, int64_t ldc, int32_t beta,
                           const rosko_plan& plan, hipStream_t s) {
  SpmmArgs g{};
  g.panel_col_ptr = A->panel_col_ptr;
  g.col_ind = A->col_ind;
  g.col_nnz = A->col_nnz;
  g.col_ptr = A->col_ptr;
  g.loc = A->loc;
  g.val = A->val;
  g.row_scale = A->row_scale;
  g.B = B;
  g.C = C;
  g.M = A->M;
  g.N = N;
  g.ldb = ldb;
  g.ldc = ldc;
  g.mr = A->mr;
  g.n_panels = A->n_panels;
  g.beta = beta;
  const int V = plan.cols_per_lane, W = plan.waves;
  const size_t eb = (b_dtype == ROSKO_F32) ? 4 : 2;
  g.vec = (V > 0) && (ldb % V == 0) && (ldc % V == 0) && (N % V == 0) &&
          ((uintptr_t)B % (eb * V) == 0) && ((uintptr_t)C % (4 * V) == 0);
  const int H = tile_height(A->mr);
  const bool bf = (b_dtype == ROSKO_BF16);
  switch (A->val_dtype) {
    case ROSKO_F32: return bf ? spmm_dispatch_f32_bf16(g, H, V, W, s) : spmm_dispatch_f32_f32(g, H, V, W, s);
    case ROSKO_BF16: return bf ? spmm_dispatch_bf16_bf16(g, H, V, W, s) : spmm_dispatch_bf16_f32(g, H, V, W, s);
    default: return bf ? spmm_dispatch_fp8_bf16(g, H, V, W, s) : spmm_dispatch_fp8_f32(g, H, V, W, s);
  }
}

}  // namespace rosko
