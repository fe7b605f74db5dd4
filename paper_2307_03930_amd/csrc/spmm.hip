// Row-skipping outer-product SpMM on gfx950 (Alg. 2, Sec. 4.2) -- host side.
//
// Kernel (spmm_kernel.h).  A wavefront owns one panel (mr rows) and one
// chunk of 64*V columns of C, its C tile held in VGPRs for its whole run of
// the panel's column records (the K-first schedule of Sec. 2.2 / 4.2).  Per
// kept column it reads the B row segment the column selects (V elements per
// lane) and, for every value of the column, multiply-accumulates it into
// tile row loc; rows whose A entry is zero are never touched -- the row
// skipping -- and the B segment is reused by every value of the column.
//
// The column's data arrives as one 64-byte record per column (packing writes
// it beside the canonical arrays): header (k, count), row bytes, values.  A
// wavefront loads a record as a single VGPR (lane l holds dword l & 15) and
// the B segment with one vector load, several columns ahead of their use, so
// a column never waits on a dependent load round trip.
//
// The C row is a run-time index, yet the tile must stay in registers.  The
// tile is pinned to a fixed VGPR range through inline-asm register
// constraints, row r of column j at v[base + j*MR + r].  The column's values
// are applied by a run of equal-sized value blocks entered through one
// computed jump per column (at the block of value count-1); each block cuts
// its row byte to log2(MR) bits, makes it the index of VGPR-relative
// addressing (SRC2 and DST of the FMA), and issues V v_fmac_f32 whose A
// operand is the value's lane of the record VGPR broadcast by DPP
// row_newbcast.  The cut keeps every relative access inside the pinned range.
//
// Small M x N outputs cannot fill the GPU with one wavefront per tile, so a
// panel's records are cut into k_split * H equal runs: H wavefronts of one
// workgroup add their tiles through LDS in a fixed order, and with
// k_split > 1 the workgroups' tiles go to a workspace that k_reduce_splits
// adds in split order (no atomics, so results are reproducible).
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
// blockIdx.y strides over rows; a thread handles 4 consecutive columns with
// float4 accesses when VEC (N, ldc and the pointers allow it), and issues the
// loads of up to 8 splits before it adds any, so a call costs about one
// memory round trip per 8 splits.
template <bool VEC>
__global__ void __launch_bounds__(256)
k_reduce_splits(const float* __restrict__ ws, int32_t S, int64_t M, int64_t N,
                const float* __restrict__ row_scale, const int32_t* __restrict__ row_perm,
                float* __restrict__ C, int64_t ldc, int32_t beta) {
  const int64_t MN = M * N;
  const int64_t n = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (n >= N) return;
  for (int64_t m = blockIdx.y; m < M; m += gridDim.y) {
    const float* src = ws + m * N + n;
    float* c = C + perm_row(row_perm, m, M) * ldc + n;
    const float sc = row_scale ? row_scale[m] : 1.0f;
    if (VEC) {
      float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      for (int32_t s0 = 0; s0 < S; s0 += 8) {
        float4 x[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          // splits past S re-read the last one (in bounds) and are not added
          const int32_t sl = s0 + t < S ? s0 + t : S - 1;
          x[t] = *reinterpret_cast<const float4*>(src + sl * MN);
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          if (s0 + t < S) {
            if (s0 + t == 0) {
              acc = x[0];
            } else {
              acc.x += x[t].x; acc.y += x[t].y; acc.z += x[t].z; acc.w += x[t].w;
            }
          }
        }
      }
      if (row_scale) { acc.x *= sc; acc.y *= sc; acc.z *= sc; acc.w *= sc; }
      if (beta) {
        const float4 o = *reinterpret_cast<const float4*>(c);
        acc.x += o.x; acc.y += o.y; acc.z += o.z; acc.w += o.w;
      }
      *reinterpret_cast<float4*>(c) = acc;
    } else {
      for (int j = 0; j < 4 && n + j < N; ++j) {
        float acc = src[j];
        for (int32_t s = 1; s < S; ++s) acc += src[s * MN + j];
        if (row_scale) acc *= sc;
        c[j] = beta ? c[j] + acc : acc;
      }
    }
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


}  // namespace

int32_t launch_fill_zero(float* C, int64_t M, int64_t N, int64_t ldc, hipStream_t s) {
  if (M == 0 || N == 0) return ROSKO_OK;
  const int64_t blocks = std::min<int64_t>(ceil_div(M * N, 256), 65536);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, C, M, N, ldc);
  ROSKO_LAUNCH_CHECK("k_fill_zero");
  return ROSKO_OK;
}

// Parallel shape of the sparse path.  A wavefront's time is set by the
// length of its run of records (each costs a few hundred cycles of scalar
// work around its values), so the panel's records are cut into H runs per
// workgroup (added through LDS) and, while runs stay long, into k_split
// workgroups (added by k_reduce_splits, which costs a launch and a pass over
// k_split copies of C):
//   H = 4 from 64 records per panel, 2 from 32, else 1 (but 1 for
//   128-accumulator tiles on grids of 512 tiles or more, below);
//   k_split > 1 only when a run of the H-way cut exceeds kSplitRun records:
//   then as many as keep runs of at least kMinRun records and the grid within
//   what the SIMDs can hold at once (wavefronts per SIMD by the tile's VGPR
//   budget), at most 8.
// Records per panel come from nrec (or from nnz at about 8 values per record
// when nrec is unknown).
static void auto_parallelism(const rosko_packed* A, int64_t N, int V, int32_t* H_out,
                             int32_t* S_out) {
  const int64_t P = std::max<int64_t>(1, A->n_panels);
  const int64_t chunks = std::max<int64_t>(1, ceil_div(N, 64 * V));
  const int64_t tiles = P * chunks;
  constexpr int64_t kMinRun = 64, kSplitRun = 100;
  int64_t per_panel = 1 << 30;
  if (A->nrec >= 0) per_panel = A->nrec / P;
  else if (A->nnz >= 0) per_panel = A->nnz / (8 * P);
  const int H = per_panel >= 64 ? 4 : (per_panel >= 32 ? 2 : 1);
  const int64_t run = per_panel / H;
  // wavefronts per SIMD to aim for: 64-accumulator tiles fit 5 (about 100
  // VGPRs), smaller ones 8; 128-accumulator tiles fit 3 (about 160 VGPRs),
  // but 2 measured faster (fewer copies of C to add)
  const int accs = tile_height(A->mr) * V;
  const int64_t per_simd = accs >= 128 ? 2 : (accs >= 64 ? 5 : 8);
  const int64_t cap = 1024 * per_simd;                     // 256 CUs x 4 SIMDs
  int64_t S = 1;
  if (run > kSplitRun) {
    S = std::min<int64_t>(run / kMinRun, cap / (tiles * H));
    S = std::max<int64_t>(1, std::min<int64_t>(S, 8));
  }
  *H_out = H;
  *S_out = (int32_t)S;
  // 128-accumulator tiles on a grid of kWideGridTiles tiles or more: a
  // 4-wavefront workgroup's LDS reduction (two 32 KB tile images) leaves
  // room for 2 workgroups per CU, which that grid already fills, while
  // one-wavefront workgroups need no LDS and fit 3 per SIMD by VGPRs.  So
  // one wavefront per tile and as many splits as fill those 3 per SIMD, at
  // most 8 (measured: 4096 x 4096 at 90%, N = 2048: 270 us against 284 us
  // for 4 wavefronts, 1024 tiles; with 104-416 tiles 4 wavefronts stay
  // faster).
  constexpr int64_t kWideGridTiles = 512;
  if (accs >= 128 && tiles >= kWideGridTiles) {
    int64_t S1 = std::min<int64_t>(per_panel / kMinRun, 3 * 1024 / tiles);
    *H_out = 1;
    *S_out = (int32_t)std::max<int64_t>(1, std::min<int64_t>(S1, 8));
  }
}

// B rows in flight per wavefront: 4 (8 measured no faster on any tile).
static int32_t auto_depth(int, int) { return 4; }

// The analytic fallback plan: the register tile is the widest the panel
// height allows (128 accumulators per lane), narrowed when N is small; the
// parallel shape from auto_parallelism.
rosko_plan auto_plan(const rosko_packed* A, int64_t N) {
  rosko_plan p{};
  p.path = ROSKO_PATH_SPARSE;
  const int MRt = tile_height(A->mr);
  p.cols_per_lane = (MRt <= 32) ? 4 : (MRt == 64 ? 2 : 1);
  if (MRt == 32 && N <= 128) p.cols_per_lane = 2;
  auto_parallelism(A, N, p.cols_per_lane, &p.waves_per_tile, &p.k_split);
  p.depth = auto_depth(MRt, p.cols_per_lane);
  return p;
}

int32_t normalize_plan(const rosko_packed* A, int64_t N, rosko_plan* p) {
  if (p->path == ROSKO_PATH_AUTO) {
    *p = auto_plan(A, N);
    return ROSKO_OK;
  }
  if (p->path == ROSKO_PATH_DENSE) return ROSKO_OK;   // no further parameters
  if (p->path != ROSKO_PATH_SPARSE) {
    set_error("plan path %d not supported", p->path);
    return ROSKO_EUNSUPPORTED;
  }
  const int MRt = tile_height(A->mr);
  if (!tile_supported(MRt, p->cols_per_lane)) {
    set_error("unsupported register tile: mr %d (height %d) with %d columns per lane", A->mr,
              MRt, p->cols_per_lane);
    return ROSKO_EUNSUPPORTED;
  }
  if (p->waves_per_tile == 0 || p->k_split == 0) {   // 0 fields: the library's choice
    int32_t h, sp;
    auto_parallelism(A, N, p->cols_per_lane, &h, &sp);
    if (p->waves_per_tile == 0) p->waves_per_tile = h;
    if (p->k_split == 0) p->k_split = sp;
  }
  const int H = p->waves_per_tile;
  if (H != 1 && H != 2 && H != 4) {
    set_error("unsupported waves per tile %d (1, 2 or 4)", H);
    return ROSKO_EUNSUPPORTED;
  }
  if (p->k_split < 1) {
    set_error("k_split %d < 1", p->k_split);
    return ROSKO_EINVAL;
  }
  if (p->k_split > ROSKO_MAX_K_SPLIT) p->k_split = ROSKO_MAX_K_SPLIT;
  if (p->depth == 0) p->depth = auto_depth(MRt, p->cols_per_lane);
  if (p->depth != 4 && p->depth != 8) {
    set_error("unsupported depth %d (4 or 8)", p->depth);
    return ROSKO_EUNSUPPORTED;
  }
  return ROSKO_OK;
}

size_t spmm_ws_bytes(const rosko_packed* A, int64_t N, const rosko_plan& p) {
  if (p.path == ROSKO_PATH_DENSE) return dense_ws_bytes(A, N, ROSKO_F32);
  if (p.k_split <= 1) return 0;
  return sizeof(float) * (size_t)p.k_split * (size_t)A->M * (size_t)N;
}

// Shared body: rec (A's or a caller's copy), B with b_rows rows of ldb
// elements (flat: ldb 1 and every row start a multiple of 4 elements).
static int32_t spmm_sparse_core(const rosko_packed* A, const uint32_t* rec, const void* B,
                                int32_t b_dtype, int64_t N, int64_t ldb, int64_t b_rows,
                                bool flat, float* C, int64_t ldc, int32_t beta,
                                const rosko_plan& plan, float* ws, size_t ws_bytes,
                                hipStream_t s) {
  SpmmArgs g{};
  g.rec = rec;
  g.row_scale = (A->val_dtype == ROSKO_FP8_E4M3) ? A->row_scale : nullptr;
  g.kblk_ptr = A->kblk_ptr;
  g.row_perm = A->row_perm;
  g.B = B;
  g.C = C;
  g.ws = ws;
  g.M = A->M;
  g.K = A->K;
  g.N = N;
  g.ldb = ldb;
  g.ldc = ldc;
  g.b_rows = b_rows;
  g.mr = A->mr;
  g.n_panels = A->n_panels;
  g.beta = beta;
  const int H = plan.waves_per_tile;
  g.k_split = std::max(1, plan.k_split);
  g.rec_bound = A->nrec >= 0 ? std::min(A->nrec, A->nrec_cap) : A->nrec_cap;
  const size_t eb = (b_dtype == ROSKO_F32) ? 4 : 2;
  // The record loop reads B and the records with buffer loads at 32-bit
  // offsets and V-wide aligned B units, and stores V-wide C units.  When
  // the requested tile's V does not fit B and C (N, ldb, ldc or a pointer
  // not a multiple of V), the one-column tile (128 x 1) runs instead, which
  // needs no alignment beyond the element size.  A flat B guarantees its row
  // starts are multiples of 4 elements, so ldb does not enter.  Beyond
  // 32-bit offsets the call is refused.
  auto vec_ok = [&](int v) {
    return (flat || ldb % v == 0) && (ldc % v == 0) && (N % v == 0) &&
           ((uintptr_t)B % (eb * v) == 0) && ((uintptr_t)C % (4 * v) == 0);
  };
  int V = plan.cols_per_lane, MRt = tile_height(A->mr);
  if (!vec_ok(V)) {
    V = 1;
    MRt = 128;
    if (!vec_ok(1)) {
      set_error("B or C is not aligned to its element size");
      return ROSKO_EUNSUPPORTED;
    }
  }
  // a wavefront's records lie inside one panel: at most K kept columns of
  // ceil(mr / 12) records each (plus the loop's read-ahead)
  const uint64_t panel_rec = (uint64_t)A->K * (uint64_t)ceil_div(A->mr, kRecVals) + 64;
  if ((uint64_t)b_rows * (uint64_t)ldb * eb >= (1ull << 32) || panel_rec * 64u >= (1ull << 32)) {
    set_error("B (%lld x %lld elements) or a panel's records exceed 4 GiB of buffer offsets",
              (long long)b_rows, (long long)ldb);
    return ROSKO_EUNSUPPORTED;
  }
  g.n_chunks = ceil_div(N, 64 * V);
  g.vec = 1;
  g.ws_vec = (N % V == 0) && ((uintptr_t)ws % (4 * V) == 0);
  if (g.k_split > 1) {
    const size_t need = spmm_ws_bytes(A, N, plan);
    if (ws == nullptr || ws_bytes < need) {
      set_error("spmm workspace %zu bytes < %zu (k_split %d)", ws_bytes, need, g.k_split);
      return ROSKO_ESMALLBUF;
    }
  }
  const int32_t st = (b_dtype == ROSKO_BF16) ? spmm_dispatch_bbf16(g, MRt, V, H, plan.depth, s)
                                             : spmm_dispatch_bf32(g, MRt, V, H, plan.depth, s);
  if (st != ROSKO_OK || g.k_split == 1) return st;
  const bool rvec = (N % 4 == 0) && (ldc % 4 == 0) && ((uintptr_t)C % 16 == 0) &&
                    ((uintptr_t)ws % 16 == 0);
  const dim3 grid((unsigned)ceil_div(ceil_div(N, 4), 256),
                  (unsigned)std::min<int64_t>(A->M, 65535));
  const float* rs = A->val_dtype == ROSKO_FP8_E4M3 ? A->row_scale : nullptr;
  if (rvec)
    hipLaunchKernelGGL(k_reduce_splits<true>, grid, dim3(256), 0, s, ws, g.k_split, A->M, N,
                       rs, A->row_perm, C, ldc, beta);
  else
    hipLaunchKernelGGL(k_reduce_splits<false>, grid, dim3(256), 0, s, ws, g.k_split, A->M, N,
                       rs, A->row_perm, C, ldc, beta);
  ROSKO_LAUNCH_CHECK("k_reduce_splits");
  return ROSKO_OK;
}

int32_t launch_spmm_sparse(const rosko_packed* A, const void* B, int32_t b_dtype, int64_t N,
                           int64_t ldb, float* C, int64_t ldc, int32_t beta,
                           const rosko_plan& plan, float* ws, size_t ws_bytes, hipStream_t s) {
  return spmm_sparse_core(A, A->rec, B, b_dtype, N, ldb, A->K, false, C, ldc, beta, plan, ws,
                          ws_bytes, s);
}

int32_t launch_spmm_sparse_flat(const rosko_packed* A, const uint32_t* rec, const float* B,
                                int64_t b_rows, int64_t N, float* C, int64_t ldc, int32_t beta,
                                const rosko_plan& plan, float* ws, size_t ws_bytes,
                                hipStream_t s) {
  return spmm_sparse_core(A, rec ? rec : A->rec, B, ROSKO_F32, N, 1, b_rows, true, C, ldc,
                          beta, plan, ws, ws_bytes, s);
}

}  // namespace rosko
