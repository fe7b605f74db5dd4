// Internal declarations shared by the library's HIP translation units.
// Nothing here is part of the public ABI (include/rosko.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rosko.h"

namespace rosko {

// Error state (per host thread) and helpers.
void set_error(const char* fmt, ...);
void clear_error();

#define ROSKO_HIP_CHECK(call)                                                          \
  do {                                                                                 \
    hipError_t e__ = (call);                                                           \
    if (e__ != hipSuccess) {                                                           \
      ::rosko::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e__),       \
                         __FILE__, __LINE__);                                          \
      return ROSKO_EHIP;                                                               \
    }                                                                                  \
  } while (0)

// Launch check right after a kernel launch.
#define ROSKO_LAUNCH_CHECK(name)                                                       \
  do {                                                                                 \
    hipError_t e__ = hipGetLastError();                                                \
    if (e__ != hipSuccess) {                                                           \
      ::rosko::set_error("launch of %s failed: %s", name, hipGetErrorString(e__));     \
      return ROSKO_EHIP;                                                               \
    }                                                                                  \
  } while (0)

// ---------------------------------------------------------------- packing
// Workspace layout (byte offsets, 256-byte aligned) for packing an
// R x S matrix (R rows split into panels of mr) given as rows x cols.
struct PackWs {
  size_t counts;       // int32 [P*S]        values per (panel, column)
  size_t tile_sums;    // int64 [3*NT]       (values, kept columns, records) per tile
  size_t tile_offs;    // int64 [3*NT]       exclusive prefix of tile_sums
  size_t totals;       // int64 [4]          nnz, ncols, overflow flag, nrec
  size_t transposed;   // float [R*S]        dense transpose (transpose packing only)
  size_t bytes;        // total
  int64_t P, NT;       // panels; tiles of 64 * cpl (panel, column) pairs
  int32_t cpl;         // pairs per lane (pack_cols_per_lane)
  int32_t rr;          // rows per lane load (pack_rows_per_lane)
};
constexpr int kPackTile = 64;        // lanes per tile: one wavefront
constexpr int kRecVals = 12;         // values per 16-dword column record
constexpr int kPackThreads = 64;
// (panel, column) pairs per lane: 4 for mr <= 8, 2 for mr <= 16, else 1, so
// a lane sees about 32 entries and a tile 64 * cols pairs whatever mr is.
// (panel, column) pairs per lane in a packing tile: one for panels of more
// than 16 rows, and for panels of up to 16 rows while the grid stays within
// kOnePairMaxTiles tiles (more, shorter tiles spread a small matrix over more
// SIMDs); otherwise 4 (up to 8 rows) or 2 (up to 16), about 32 entries a lane.
constexpr int64_t kOnePairMaxTiles = 1280;
inline int pack_cols_per_lane(int32_t mr, int64_t pairs) {
  if (mr > 16 || pairs <= kOnePairMaxTiles * 64) return 1;
  return mr <= 8 ? 4 : 2;
}
// Rows a lane loads per pair: the panel height bound of the tile shape
// (8 or 16 with one pair per lane for small panels), 32 per batch above.
inline int pack_rows_per_lane(int32_t mr, int cpl) {
  if (cpl == 4 || mr <= 8) return 8;
  if (cpl == 2 || mr <= 16) return 16;
  return 32;
}
// Up to this many tiles the write pass adds up the tile sums before its own
// tile itself (no separate scan launch); beyond, a one-workgroup scan runs.
constexpr int64_t kLocalPrefixTiles = 4096;
// Up to this many tiles (panels of up to 32 rows) the write pass counts its
// own columns and takes its offset from the aggregates the tiles before it
// publish: one launch, no count pass (see the single-pass notes in
// pack.hip).  kFusedSpin: re-reads of a missing aggregate before the tile
// counts that tile again itself.
constexpr int64_t kFusedMaxTiles = 2048;
constexpr int32_t kFusedSpin = 32;
PackWs pack_ws_layout(int64_t R, int64_t S, int32_t mr, bool transpose);
// rosko_pack_set_mode
int32_t set_pack_mode(int32_t mode);

// Enqueue count + tile scan (everything rosko_pack_query needs).
int32_t launch_pack_count_scan(const float* A, int64_t R, int64_t S, int64_t lda, int32_t mr,
                               void* ws, const PackWs& L, const rosko_packed* out,
                               hipStream_t s);
// Enqueue the whole packing: count, then either the write pass with local
// tile prefixes (which also closes the pointer arrays and the totals), or
// the scan and the write pass reading its prefixes.
int32_t launch_pack(const float* A, int64_t R, int64_t S, int64_t lda, int32_t mr,
                    int32_t val_dtype, void* ws, const PackWs& L, const rosko_packed* out,
                    hipStream_t s);
int32_t launch_row_scale(const float* A, int64_t R, int64_t S, int64_t lda, float* scale,
                         hipStream_t s);
int32_t launch_transpose(const float* A, int64_t M, int64_t K, int64_t lda, float* At,
                         hipStream_t s);

// ------------------------------------------------------------------- SpMM
// Kernel arguments of the row-skipping SpMM (device pointers of the packed
// matrix, B and C).
struct SpmmArgs {
  const uint32_t* rec;          // column records, 16 dwords each
  const float* row_scale;       // FP8 row scales, else null
  const int64_t* kblk_ptr;      // record index per (panel, K block)
  const int32_t* row_perm;      // C row of each packed row, or null
  const void* B;
  float* C;
  float* ws;           // k_split x M x N partial tiles (k_split > 1)
  int64_t M, K, N, ldb, ldc;
  int64_t n_chunks;    // ceil(N / (64 * cols_per_lane))
  int64_t rec_bound;   // records the record array holds (nrec when known, never above
                       // its capacity): every record read stays below it
  int64_t b_rows;      // rows of B the buffer holds (K; more for the direct convolution,
                       // whose records name element offsets of a flat input)
  int32_t mr, n_panels;
  int32_t beta;
  int32_t k_split;
  int32_t vec;         // B/C rows allow V-wide vector access (alignment, N % V)
  int32_t ws_vec;      // workspace rows allow V-wide vector access
};
// One dispatcher per B dtype; MRt = register-tile height, V = columns per
// lane, H = wavefronts per tile, depth = B rows in flight (4 or 8).
int32_t spmm_dispatch_bf32(const SpmmArgs& g, int MRt, int V, int H, int depth, hipStream_t s);
int32_t spmm_dispatch_bbf16(const SpmmArgs& g, int MRt, int V, int H, int depth, hipStream_t s);

// Plan helpers (spmm.hip): the automatic plan, validation/normalisation of a
// caller's plan, and the workspace a plan needs.
rosko_plan auto_plan(const rosko_packed* A, int64_t N);
int32_t normalize_plan(const rosko_packed* A, int64_t N, rosko_plan* p);
size_t spmm_ws_bytes(const rosko_packed* A, int64_t N, const rosko_plan& p);

int32_t launch_spmm_sparse(const rosko_packed* A, const void* B, int32_t b_dtype, int64_t N,
                           int64_t ldb, float* C, int64_t ldc, int32_t beta,
                           const rosko_plan& plan, float* ws, size_t ws_bytes, hipStream_t s);
// The same with the records taken from `rec` (nullptr: A's) and B a flat
// array of b_rows "rows" one element apart (ldb 1) whose row starts are all
// multiples of 4 elements, so V-wide loads stay aligned (direct convolution).
int32_t launch_spmm_sparse_flat(const rosko_packed* A, const uint32_t* rec, const float* B,
                                int64_t b_rows, int64_t N, float* C, int64_t ldc, int32_t beta,
                                const rosko_plan& plan, float* ws, size_t ws_bytes,
                                hipStream_t s);
int32_t launch_fill_zero(float* C, int64_t M, int64_t N, int64_t ldc, hipStream_t s);

// Dense-MFMA path (dense.hip): workspace bytes (b_dtype ROSKO_F32 gives the
// larger, FP32 operand size) and the launch.
size_t dense_ws_bytes(const rosko_packed* A, int64_t N, int32_t b_dtype);
int32_t launch_spmm_dense(const rosko_packed* A, const void* B, int32_t b_dtype, int64_t N,
                          int64_t ldb, float* C, int64_t ldc, int32_t beta, void* ws,
                          size_t ws_bytes, hipStream_t s);

// ------------------------------------------------------ scheduler (sched.hip)
size_t features_ws_bytes(int64_t M, int64_t K);
int32_t launch_features(const float* A, int64_t M, int64_t K, int64_t lda, int64_t N, void* ws,
                        float* f, hipStream_t s);
int32_t launch_normalize(const float* X, int64_t Bn, int32_t F, const float* mu,
                         const float* sigma, float* Xn, hipStream_t s);
int32_t launch_mlp_forward(const float* prm, int32_t F, int32_t H, int32_t C, const float* X,
                           int64_t Bn, float* H1, float* H2, float* Y, hipStream_t s);
int32_t launch_mlp_backward(const float* prm, int32_t F, int32_t H, int32_t C, const float* X,
                            const float* H1, const float* H2, const float* Y, const float* T,
                            const float* mask, int64_t Bn, float* grads, float* ws, float* loss,
                            hipStream_t s);
int32_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                    float b2, float eps, int32_t t, hipStream_t s);
int32_t launch_argmin(const float* Y, int64_t Bn, int32_t C, int32_t* out, hipStream_t s);

// ---------------------------------------------------------------- SDDMM
// Workspace of the SDDMM (partial dot products over column chunks of N).
size_t sddmm_ws_bytes(const rosko_packed* A, int64_t N);
int32_t launch_sddmm(const rosko_packed* A, const float* dC, int64_t lddc, const float* B,
                     int64_t ldb, int64_t N, float* dA_val, int64_t dA_cap, float* ws,
                     size_t ws_bytes, hipStream_t s);
int32_t launch_scatter_dense(const rosko_packed* A, const float* vals, int64_t n_vals,
                             float* out, int64_t ldo, hipStream_t s);

// --------------------------------------------------------- CSR packing
// Workspace of rosko_pack_csr (byte offsets, 256-byte aligned): totals
// first (so rosko_pack_csr_result finds them at offset 0), then the row and
// panel offsets, the sort's keys and values (in and out), the column
// numbering, per-column starts, keys and record counts, the record offsets,
// and the library scratch of the sort and scans at `temp`.
constexpr int kCsrTotals = 8;
constexpr int kCsrTotNnz = 0, kCsrTotNcols = 1, kCsrTotOverflow = 2, kCsrTotNrec = 3,
              kCsrTotBad = 4;
struct CsrWs {
  size_t totals, rowlen, rowoff, seen, pofs, kin, kout, vin, vout, hd, cid, colstart, colk, nr,
      rptr, temp, bytes;
  int64_t P, nz;
};
CsrWs csr_ws_layout(int64_t M, int64_t nz, int32_t mr);
int32_t csr_temp_bytes(const CsrWs& L, int64_t M, int64_t K, size_t* bytes, hipStream_t s);
// out == nullptr: the counting passes only (for rosko_pack_csr_query).
int32_t launch_pack_csr(const int64_t* row_ptr, const int32_t* col_idx, const float* val,
                        const int32_t* perm, int64_t M, int64_t K, int64_t nz_in, int32_t mr,
                        int32_t val_dtype, void* ws, size_t ws_bytes, const rosko_packed* out,
                        hipStream_t s);
// Row order (inspector): fixed workspace part and the sort's scratch.
size_t order_ws_bytes_fixed(int64_t M);
int32_t order_temp_bytes(int64_t M, size_t* bytes, hipStream_t s);
int32_t launch_row_order(const int64_t* row_ptr, int64_t M, int32_t mr, int32_t mode,
                         void* ws, size_t ws_bytes, int32_t* perm, hipStream_t s);

// ------------------------------------------------ direct convolution
// Geometry of the padded-pitch grid (conv.hip): row pitch Wq >= W + 2 with
// H * Wq a multiple of 4, plane (H + 2) * Wq, T the length of each of the
// four shifted input copies, N = H * Wq output columns.
struct ConvGeom {
  int64_t Wq, plane, T, N;
};
ConvGeom conv_geometry(int64_t C_in, int64_t H, int64_t W);
int32_t launch_conv_input(const float* X, int64_t C_in, int64_t H, int64_t W, float* Bc,
                          hipStream_t s);
int32_t launch_conv_records(const rosko_packed* A, int64_t nrec, int64_t C_in, int64_t H,
                            int64_t W, uint32_t* rec_out, hipStream_t s);
int32_t launch_conv_unpad(const float* Yq, int64_t ldy, int64_t C_out, int64_t H, int64_t W,
                          int64_t Wq, float* Y, hipStream_t s);

// Matrix row of packed row `row` under an optional row order (clamped into
// 0..M-1, so no content of the order can move an access outside).
__device__ __forceinline__ int64_t perm_row(const int32_t* perm, int64_t row, int64_t M) {
  if (perm == nullptr) return row;
  const int64_t m = perm[row];
  return m < 0 ? 0 : (m >= M ? M - 1 : m);
}

// Round x up to a multiple of a (a > 0).
inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline int64_t ceil_div(int64_t x, int64_t a) { return (x + a - 1) / a; }

}  // namespace rosko
