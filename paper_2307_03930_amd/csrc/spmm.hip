// Row-skipping outer-product SpMM on gfx950 (Alg. 2, Sec. 4.2) -- host side.
//
// Kernel (spmm_kernel.h): a workgroup owns up to 8 panels (one wavefront
// each) and one chunk of 64*V columns of C.  It walks its K range in blocks
// of B rows that all its threads load together into LDS (double-buffered,
// so the next block is in flight while the current one is used); each
// wavefront then walks its panel's kept columns inside the block: it reads
// the B row segment its column selects from LDS and, for every value of the
// column, multiply-accumulates it into C-tile row loc.  Rows whose A entry is
// zero are never touched -- the row skipping -- and a staged B row is reused
// by every value of the column and by every panel of the workgroup.  The C
// tile stays in VGPRs for the whole K range (the K-first schedule of Sec. 2.2
// / 4.2) and is written once.
//
// The C row is a run-time index, yet the tile must stay in registers.  The
// tile is pinned to the fixed VGPR range v[64 : 64+MR*V) through inline-asm
// register constraints, row r of column j at v[64 + j*MR + r].  Every value
// of A is applied by one asm block: s_set_gpr_idx_on with the (wave-uniform)
// row index turns on relative addressing for the FMA's addend and result,
// V v_fma_f32 follow, and s_set_gpr_idx_off ends the mode.  The row index is
// masked to MR-1 so the relative access can never leave the pinned range.
//
// Small M x N outputs cannot fill the GPU with whole-K tiles, so K may be cut
// into k_split ranges; partial tiles then go to a workspace and
// k_reduce_splits adds them in split order (no atomics, reproducible).
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

// Split-K epilogue: C[m][n] = (beta ? C[m][n] : 0) + s_m * sum_s ws[s][m][n],
// the partials added in split order (fixed, so the result is reproducible).
__global__ void __launch_bounds__(256)
k_reduce_splits(const float* __restrict__ ws, int32_t S, int64_t M, int64_t N,
                const float* __restrict__ row_scale, float* __restrict__ C, int64_t ldc,
                int32_t beta) {
  const int64_t total = M * N;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const int64_t m = i / N, n = i - m * N;
    float acc = ws[i];
    for (int32_t s = 1; s < S; ++s) acc += ws[(int64_t)s * total + i];
    if (row_scale) acc *= row_scale[m];
    float* c = C + m * ldc + n;
    *c = beta ? *c + acc : acc;
  }
}

// Smallest supported register-tile height holding mr rows.
int tile_height(int32_t mr) {
  if (mr <= 8) return 8;
  if (mr <= 16) return 16;
  if (mr <= 32) return 32;
  if (mr <= 64) return 64;
  if (mr <= 128) return 128;
  return 0;
}

bool tile_supported(int H, int V) {
  return (H == 8 && V == 4) || (H == 16 && V == 4) || (H == 32 && (V == 4 || V == 2)) ||
         (H == 64 && V == 2) || (H == 128 && V == 1);
}

int64_t n_kblocks(int64_t K) { return (K + ROSKO_KSTEP - 1) / ROSKO_KSTEP; }

}  // namespace

int32_t launch_fill_zero(float* C, int64_t M, int64_t N, int64_t ldc, hipStream_t s) {
  if (M == 0 || N == 0) return ROSKO_OK;
  const int64_t blocks = std::min<int64_t>(ceil_div(M * N, 256), 65536);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, C, M, N, ldc);
  ROSKO_LAUNCH_CHECK("k_fill_zero");
  return ROSKO_OK;
}

// The analytic fallback plan.  The register tile is the widest the panel
// height allows (128 accumulators per lane).  Panels of one workgroup share
// each staged block of B rows, so a workgroup takes as many panels as exist
// up to 8.  K is then split until the grid has about two workgroups per
// compute unit, within the K blocks available and a workspace of at most
// 4x the output.
rosko_plan auto_plan(const rosko_packed* A, int64_t N) {
  rosko_plan p{};
  p.path = ROSKO_PATH_SPARSE;
  const int H = tile_height(A->mr);
  p.cols_per_lane = (H <= 32) ? 4 : (H == 64 ? 2 : 1);
  if (H == 32 && N <= 128) p.cols_per_lane = 2;
  const int64_t P = A->n_panels;
  p.panels_per_wg = P >= 8 ? 8 : (P >= 4 ? 4 : (P >= 2 ? 2 : 1));
  const int64_t n_pg = ceil_div(P, p.panels_per_wg);
  const int64_t chunks = ceil_div(N, 64 * p.cols_per_lane);
  const int64_t target = 512;
  int64_t S = ceil_div(target, std::max<int64_t>(1, n_pg * chunks));
  S = std::min<int64_t>(S, std::max<int64_t>(1, n_kblocks(A->K)));
  S = std::min<int64_t>(S, 4);
  p.k_split = (int32_t)std::max<int64_t>(1, S);
  return p;
}

int32_t normalize_plan(const rosko_packed* A, int64_t N, rosko_plan* p) {
  (void)N;
  if (p->path == ROSKO_PATH_AUTO) {
    *p = auto_plan(A, N);
    return ROSKO_OK;
  }
  if (p->path != ROSKO_PATH_SPARSE) {
    set_error("plan path %d not supported", p->path);
    return ROSKO_EUNSUPPORTED;
  }
  const int H = tile_height(A->mr);
  if (!tile_supported(H, p->cols_per_lane)) {
    set_error("unsupported register tile: mr %d (height %d) with %d columns per lane", A->mr,
              H, p->cols_per_lane);
    return ROSKO_EUNSUPPORTED;
  }
  const int G = p->panels_per_wg;
  if (G != 1 && G != 2 && G != 4 && G != 8) {
    set_error("unsupported panels per workgroup %d (1, 2, 4 or 8)", G);
    return ROSKO_EUNSUPPORTED;
  }
  if (p->k_split < 1) {
    set_error("k_split %d < 1", p->k_split);
    return ROSKO_EINVAL;
  }
  const int64_t nkb = std::max<int64_t>(1, n_kblocks(A->K));
  if (p->k_split > nkb) p->k_split = (int32_t)nkb;
  return ROSKO_OK;
}

size_t spmm_ws_bytes(const rosko_packed* A, int64_t N, const rosko_plan& p) {
  if (p.k_split <= 1) return 0;
  return sizeof(float) * (size_t)p.k_split * (size_t)A->M * (size_t)N;
}

int32_t launch_spmm_sparse(const rosko_packed* A, const void* B, int32_t b_dtype, int64_t N,
                           int64_t ldb, float* C, int64_t ldc, int32_t beta,
                           const rosko_plan& plan, float* ws, size_t ws_bytes, hipStream_t s) {
  SpmmArgs g{};
  g.rec = A->rec;
  g.row_scale = (A->val_dtype == ROSKO_FP8_E4M3) ? A->row_scale : nullptr;
  g.kblk_ptr = A->kblk_ptr;
  g.B = B;
  g.C = C;
  g.ws = ws;
  g.M = A->M;
  g.K = A->K;
  g.N = N;
  g.ldb = ldb;
  g.ldc = ldc;
  g.mr = A->mr;
  g.n_panels = A->n_panels;
  g.beta = beta;
  const int V = plan.cols_per_lane, G = plan.panels_per_wg;
  g.k_split = std::max(1, plan.k_split);
  g.n_chunks = ceil_div(N, 64 * V);
  const size_t eb = (b_dtype == ROSKO_F32) ? 4 : 2;
  g.vec = (ldb % V == 0) && (ldc % V == 0) && (N % V == 0) &&
          ((uintptr_t)B % (eb * V) == 0) && ((uintptr_t)C % (4 * V) == 0);
  g.ws_vec = (N % V == 0) && ((uintptr_t)ws % (4 * V) == 0);
  if (g.k_split > 1) {
    const size_t need = spmm_ws_bytes(A, N, plan);
    if (ws == nullptr || ws_bytes < need) {
      set_error("spmm workspace %zu bytes < %zu (k_split %d)", ws_bytes, need, g.k_split);
      return ROSKO_ESMALLBUF;
    }
  }
  const int H = tile_height(A->mr);
  const int32_t st = (b_dtype == ROSKO_BF16) ? spmm_dispatch_bbf16(g, H, V, G, s)
                                             : spmm_dispatch_bf32(g, H, V, G, s);
  if (st != ROSKO_OK || g.k_split == 1) return st;
  const int64_t blocks = std::min<int64_t>(ceil_div(A->M * N, 256), 4096);
  hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)blocks), dim3(256), 0, s, ws, g.k_split,
                     A->M, N, A->val_dtype == ROSKO_FP8_E4M3 ? A->row_scale : nullptr, C, ldc,
                     beta);
  ROSKO_LAUNCH_CHECK("k_reduce_splits");
  return ROSKO_OK;
}

}  // namespace rosko
