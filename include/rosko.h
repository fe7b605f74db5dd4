/*
 * rosko.h -- C ABI of the MI355X (gfx950) Rosko library, librosko.so.
 *
 * Rosko computes C = A*B where A is an unstructured-sparse M x K matrix (a
 * pruned weight) and B a dense K x N matrix, as a sum of outer products in
 * which the result row of each zero entry of an A column is skipped (Sec. 3,
 * Fig. 4).  A is first packed into mr-row panels; in every panel each column
 * keeps only its nonzero values, their row indices inside the panel and a
 * per-column count, and empty columns are dropped (Alg. 1, Sec. 4.1, Fig. 5).
 * The product then streams, for each kept column, the B row it selects and
 * multiply-accumulates it into the panel's C rows named by the row indices
 * (Alg. 2).
 *
 * Conventions for every call:
 *   - Matrices are row-major with an explicit leading dimension (elements).
 *   - Pointers named as "device" must point to GPU memory of the current HIP
 *     device; "host" pointers to ordinary process memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     GPU work is enqueued on it and the call returns without waiting, unless
 *     the call's comment says it synchronises.
 *   - The library never allocates device memory.  Scratch space is passed in
 *     as a device workspace `ws` of at least the size the matching
 *     *_workspace_size call reports.  The caller owns every buffer.
 *   - Every call returns a status code and never aborts.  On failure,
 *     rosko_last_error() (per host thread) describes the reason.  Argument
 *     checks happen on the host before any GPU work is enqueued; a failed
 *     check enqueues nothing.  Faults of enqueued kernels surface at the
 *     caller's next synchronisation of the stream.
 *   - Sizes M, K, N equal to 0 are valid and do no work, except that
 *     rosko_spmm with beta = 0 still zero-fills an M x N output when K = 0.
 */
#ifndef ROSKO_H
#define ROSKO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------- */
#define ROSKO_OK 0
#define ROSKO_EINVAL (-1)        /* invalid argument (null pointer, bad size) */
#define ROSKO_EUNSUPPORTED (-2)  /* valid but not implemented (dtype, mr, plan) */
#define ROSKO_ESMALLBUF (-3)     /* a caller buffer or workspace is too small */
#define ROSKO_EHIP (-4)          /* a HIP runtime call failed */
#define ROSKO_EINTERNAL (-5)     /* internal inconsistency */

/* ---- value encodings of the packed values --------------------------- */
#define ROSKO_F32 0       /* IEEE binary32, the source bits unchanged */
#define ROSKO_BF16 1      /* bfloat16, round to nearest even; NaN -> 0x7FC0 */
#define ROSKO_FP8_E4M3 2  /* OCP E4M3FN of x / s_m, nearest-even, saturating
                             to +-448, NaN -> 0x7F; s_m = max_k |A[m][k]| / 448
                             in FP32 (1.0 for an all-zero row) */

/* ---- packed sparse matrix (Alg. 1 applied to every mr-row panel) ----
 *
 * Panel p holds rows [p*mr, min(M, (p+1)*mr)).  Inside a panel, kept columns
 * are in ascending k and the values of a column in ascending row; panels are
 * concatenated in ascending p.  An entry is kept when its FP32 bits other
 * than the sign are not all zero (so -0.0 is dropped; NaN, Inf and
 * subnormals are kept).  The kept structure never depends on val_dtype.
 *
 * All arrays are device memory owned by the caller:
 *   panel_nz_ptr [n_panels+1] int64  first value slot of each panel; [n_panels] = nnz
 *   panel_col_ptr[n_panels+1] int64  first column slot of each panel; [n_panels] = ncols
 *   col_ind  [ncols]   int32   k of each kept column (the paper's col_ind)
 *   col_nnz  [ncols]   int32   values in the column (the paper's nnz array)
 *   col_ptr  [ncols+1] int64   first value slot of each column; [ncols] = nnz
 *                              (a prefix sum of col_nnz, kept so a kernel can
 *                              start inside a panel without rescanning it)
 *   loc      [nnz]     uint8   row of the value inside its panel (loc_m)
 *   val      [nnz]     4, 2 or 1 bytes per value by val_dtype (A_p)
 *   row_scale[M]       float   s_m for ROSKO_FP8_E4M3, otherwise unused (may be NULL)
 *   rec      [nrec * 16] uint32  column records: the GPU execution copy of
 *                              the panels.  Every kept column becomes
 *                              ceil(nnz/12) records of 16 dwords, in packed
 *                              order: dword 0 = (k << 8) | count (1..12),
 *                              dwords 1..3 = the values' in-panel rows, one
 *                              byte each (value t in byte t%4 of dword
 *                              1 + t/4), dwords 4..15 = the values as FP32
 *                              bits (BF16 decoded exactly; FP8 as the code's
 *                              value, without s_m); unused bytes are zero.
 *                              One scalar load fetches a column.
 *   kblk_ptr [n_panels * (ceil(K / ROSKO_KSTEP) + 1)] int64
 *                              at [p * (nkb + 1) + j]: the first record of
 *                              panel p whose column has k >= j * ROSKO_KSTEP
 *                              (the panel's end if none); j = nkb is the end
 *                              of the panel.  Lets a workgroup start a K
 *                              range inside a panel.
 *   row_perm [M]       int32   optional row order (NULL: none): packed row i
 *                              holds row row_perm[i] of the matrix, which must
 *                              be a permutation of 0..M-1.  Set by the caller
 *                              before rosko_pack_csr (which packs in that
 *                              order); the dense packers require NULL.
 *                              rosko_spmm writes packed row i's result to C
 *                              row row_perm[i], so C keeps the matrix's own
 *                              row order; rosko_spmm_backward reads dC row
 *                              row_perm[i] for it and rosko_scatter_dense
 *                              writes it to row row_perm[i].
 * nnz_cap, ncols_cap and nrec_cap are the capacities of the caller's
 * buffers (col_ptr must hold ncols_cap+1 entries).  rosko_spmm reads values in
 * batches of 8 and row bytes by aligned dwords, so val and loc must stay
 * readable for ROSKO_READ_SLACK entries past nnz (allocate nnz_cap +
 * ROSKO_READ_SLACK entries); the extra entries are never used.  nnz and ncols are written by
 * rosko_pack_query / rosko_pack_result on the host side only. */
#define ROSKO_KSTEP 128
typedef struct rosko_packed {
  int64_t M, K;
  int32_t mr;          /* panel height, 1..256 */
  int32_t n_panels;    /* ceil(M / mr) */
  int32_t val_dtype;   /* ROSKO_F32 / ROSKO_BF16 / ROSKO_FP8_E4M3 */
  int32_t reserved;
  int64_t nnz_cap, ncols_cap, nrec_cap;
  int64_t nnz, ncols, nrec;  /* host copies when known, else -1 */
  int64_t *panel_nz_ptr;
  int64_t *panel_col_ptr;
  int32_t *col_ind;
  int32_t *col_nnz;
  int64_t *col_ptr;
  uint8_t *loc;
  void *val;
  float *row_scale;
  int64_t *kblk_ptr;
  uint32_t *rec;
  int32_t *row_perm;
} rosko_packed;

/* ---- execution plan for rosko_spmm ----------------------------------
 * A wavefront owns one panel and one chunk of 64*cols_per_lane columns of C,
 * with its C tile in VGPRs, and applies a run of the panel's column records.
 * Each panel's records are cut into k_split * waves_per_tile runs of equal
 * length.  The waves_per_tile wavefronts of one workgroup take consecutive
 * runs and add their tiles through LDS; with k_split > 1 the workgroups'
 * tiles go to the workspace and a second kernel adds them in a fixed order
 * (so results do not depend on timing) and applies the FP8 row scale and
 * beta.
 * path:           ROSKO_PATH_SPARSE (row-skipping vector kernel),
 *                 ROSKO_PATH_DENSE (every panel densified from the packed form
 *                 and multiplied on the matrix cores: BF16 MFMA when A's
 *                 values and B are exactly BF16 -- BF16 or FP8 values with a
 *                 BF16 B -- else FP32 MFMA; the other fields are ignored;
 *                 its workspace holds the densified A and the transposed
 *                 B), or
 *                 ROSKO_PATH_AUTO to let the library choose everything.
 * cols_per_lane:  1, 2 or 4.  The register tile (panel height rounded up to
 *                 8/16/32/64/128, times cols_per_lane) must be one of 8x4,
 *                 16x4, 32x4, 32x2, 64x2, 128x1; other pairs return
 *                 ROSKO_EUNSUPPORTED.  Panel heights above 128 are packed but
 *                 not multiplied by this path.
 * waves_per_tile: 1, 2 or 4; 0 lets the library choose.
 * k_split:        1 .. ROSKO_MAX_K_SPLIT (larger values are clamped); 0 lets
 *                 the library choose.
 * depth:          columns whose B rows a wavefront keeps in flight, 4 or 8;
 *                 0 lets the library choose.  */
#define ROSKO_PATH_AUTO (-1)
#define ROSKO_PATH_SPARSE 0
#define ROSKO_PATH_DENSE 1
#define ROSKO_MAX_K_SPLIT 64
typedef struct rosko_plan {
  int32_t path;
  int32_t cols_per_lane;
  int32_t waves_per_tile;
  int32_t k_split;
  int32_t depth;
} rosko_plan;

/* ---- packing (Alg. 1, Sec. 4.1) --------------------------------------- */

/* Device workspace bytes needed by rosko_pack_query / rosko_pack /
 * rosko_pack_result for an M x K matrix with panel height mr.  transpose != 0
 * sizes it for rosko_pack_transpose instead.  EINVAL for negative sizes or mr
 * outside 1..256. */
int32_t rosko_pack_workspace_size(int64_t M, int64_t K, int32_t mr, int32_t transpose,
                                  size_t *bytes);

/* Counts the kept values, kept columns and column records that packing A
 * (device, M x K, row-major, lda >= K) with panel height mr produces.
 * SYNCHRONISES `stream` to return the totals in *nnz, *ncols and *nrec
 * (host).  ws: device workspace.  EUNSUPPORTED if K >= 2^24. */
int32_t rosko_pack_query(const float *A, int64_t M, int64_t K, int64_t lda, int32_t mr,
                         void *ws, size_t ws_bytes, void *stream, int64_t *nnz, int64_t *ncols,
                         int64_t *nrec);

/* Packs A (device, M x K, lda >= K) into `out`.  The caller sets out->M, K,
 * mr, val_dtype, the capacities and the buffer pointers; the call sets
 * out->n_panels.  The packed arrays are bit-identical to those Alg. 1
 * produces with the panel order above.  Writes never exceed the capacities;
 * if the matrix needs more, the excess is dropped and rosko_pack_result
 * reports ROSKO_ESMALLBUF.  Asynchronous. */
int32_t rosko_pack(const float *A, int64_t M, int64_t K, int64_t lda, int32_t mr,
                   int32_t val_dtype, void *ws, size_t ws_bytes, rosko_packed *out,
                   void *stream);

/* Packs the transpose: the K x M matrix A^T, given A (device, M x K, lda).
 * out->M must be K and out->K must be M.  Used for dB = A^T dC.  Asynchronous. */
int32_t rosko_pack_transpose(const float *A, int64_t M, int64_t K, int64_t lda, int32_t mr,
                             int32_t val_dtype, void *ws, size_t ws_bytes, rosko_packed *out,
                             void *stream);

/* One matrix of rosko_pack_batch: the arguments of rosko_pack (stream aside),
 * or with transpose != 0 those of rosko_pack_transpose (A is M x K and A^T
 * is packed: out->M = K, out->K = M, ws sized with transpose != 0). */
typedef struct rosko_pack_job {
  const float *A;
  int64_t M, K, lda;
  int32_t mr, val_dtype;
  int32_t transpose, reserved;
  void *ws;
  size_t ws_bytes;
  rosko_packed *out;
} rosko_pack_job;

/* Packs jobs[0..n) as n calls of rosko_pack (or rosko_pack_transpose) would
 * (Alg. 1, Sec. 4.1), with
 * the same packed arrays bit for bit, in fewer launches: where the packing
 * mode gives a matrix the single pass, the matrices whose single pass has
 * the same value type and tile form (panel-height bound, pairs per lane,
 * record staging) share one grid, up to 8 to a launch, so their dispatch and
 * memory latencies overlap instead of adding up.  Each tile adds up only the
 * published totals of its own matrix, in that matrix's workspace.  The other
 * matrices are packed one by one, as rosko_pack would.  Every job is checked
 * as rosko_pack (rosko_pack_transpose) checks its arguments before anything
 * is enqueued (the transposes of the transpose jobs come first): the first
 * failing job's status is returned and nothing is enqueued.  The jobs'
 * workspaces must be pairwise disjoint and their `out` structs distinct
 * (EINVAL otherwise); their packed buffers must not overlap either (not
 * checked).  n: 0 .. ROSKO_PACK_BATCH_MAX (EINVAL otherwise).
 * Asynchronous; rosko_pack_result on a job's workspace gives its totals. */
#define ROSKO_PACK_BATCH_MAX 64
int32_t rosko_pack_batch(int32_t n, const rosko_pack_job *jobs, void *stream);

/* As rosko_pack_query, for packing A^T (K x M) from A (M x K, lda); ws sized
 * with transpose != 0.  SYNCHRONISES `stream`. */
int32_t rosko_pack_transpose_query(const float *A, int64_t M, int64_t K, int64_t lda,
                                   int32_t mr, void *ws, size_t ws_bytes, void *stream,
                                   int64_t *nnz, int64_t *ncols, int64_t *nrec);

/* After rosko_pack / rosko_pack_transpose with the same ws: SYNCHRONISES the
 * stream, stores the totals in packed->nnz / ncols, and returns
 * ROSKO_ESMALLBUF if they exceeded the capacities. */
int32_t rosko_pack_result(const void *ws, size_t ws_bytes, rosko_packed *packed, void *stream);

/* How rosko_pack and rosko_pack_transpose enqueue Alg. 1's running offsets
 * (Sec. 4.1); a setting for the whole process, ROSKO_PACK_AUTO at load.
 * Every mode gives the same packed arrays, bit for bit; they differ in
 * launches and time.
 *   ROSKO_PACK_AUTO:     one launch for grids of up to 2048 tiles of 64
 *                        (panel, column) pairs and panels of up to 32 rows,
 *                        when the stream is not capturing a graph: each tile
 *                        counts its own columns, publishes its totals in the
 *                        workspace, and adds up those of the tiles before it;
 *                        a tile whose totals have not appeared after a few
 *                        re-reads is counted again from A, so no wait
 *                        depends on another workgroup having run.  Other
 *                        grids: two launches, a count pass then the write.
 *   ROSKO_PACK_TWO_PASS: the count pass, then the write, for every grid.
 *   ROSKO_PACK_RECOUNT:  as AUTO, but no tile publishes, so each one counts
 *                        every tile before it itself (time quadratic in the
 *                        tiles: for testing that path).
 * A pack in flight keeps the mode it was enqueued with.  The single pass
 * takes a published word only if it carries the launch's tag (unique within
 * the process) and a marker bit, so words that earlier packs left in the
 * workspace are never taken; a workspace that last held unrelated data could
 * hold a matching word by chance (about 2^-33 per word for arbitrary bits),
 * which would misplace that pack's offsets (writes still stay within the
 * capacities).  rosko_pack_query on the same workspace first overwrites those
 * words, as does ROSKO_PACK_TWO_PASS.  EINVAL for any other value. */
#define ROSKO_PACK_AUTO 0
#define ROSKO_PACK_TWO_PASS 1
#define ROSKO_PACK_RECOUNT 2
int32_t rosko_pack_set_mode(int32_t mode);

/* ---- packing from compressed sparse rows (graph matrices, Sec. 5.5) ----
 * The input is an M x K matrix in CSR form on the device: row_ptr [M+1]
 * int64 (row m's entries are [row_ptr[m], row_ptr[m+1]), within
 * 0..nnz_in), col_idx [nnz_in] int32 (columns in 0..K-1, in any order within
 * a row, no column twice in a row), val [nnz_in] FP32.  Entries whose FP32
 * bits other than the sign are all zero are dropped, as in the dense
 * packers.  The packed arrays are bit-identical to rosko_pack of the dense
 * matrix whose row i is CSR row row_perm[i] (row i when row_perm is NULL).
 * Limits: M and nnz_in below 2^31, K below 2^24.  Any mr in 1..256.  The
 * workspace holds the sort of each panel's entries by column (rocPRIM) and
 * is about 52 bytes per stored entry; its size depends on the device, so
 * the size call needs a current HIP device (ROSKO_EHIP otherwise). */
int32_t rosko_pack_csr_workspace_size(int64_t M, int64_t K, int64_t nnz_in, int32_t mr,
                                      size_t *bytes);

/* Counts the kept values, kept columns and column records of packing the
 * CSR matrix in the row order row_perm (NULL: none).  SYNCHRONISES `stream`
 * and returns the totals in *nnz, *ncols, *nrec (host).  ROSKO_EINVAL if
 * the input breaks the rules above (row_perm not a permutation, row
 * pointers outside 0..nnz_in or decreasing, a column outside 0..K-1, a
 * column twice in a row); the checks run on the device. */
int32_t rosko_pack_csr_query(const int64_t *row_ptr, const int32_t *col_idx, const float *val,
                             const int32_t *row_perm, int64_t M, int64_t K, int64_t nnz_in,
                             int32_t mr, void *ws, size_t ws_bytes, void *stream, int64_t *nnz,
                             int64_t *ncols, int64_t *nrec);

/* Packs the CSR matrix into `out` in the row order out->row_perm (set by
 * the caller, NULL for none).  The caller sets out->M, K, mr, the
 * capacities and the buffer pointers as for rosko_pack.  Writes never
 * exceed the capacities.  Asynchronous; rosko_pack_csr_result reports the
 * outcome. */
int32_t rosko_pack_csr(const int64_t *row_ptr, const int32_t *col_idx, const float *val,
                       int64_t M, int64_t K, int64_t nnz_in, int32_t mr, int32_t val_dtype,
                       void *ws, size_t ws_bytes, rosko_packed *out, void *stream);

/* After rosko_pack_csr with the same ws: SYNCHRONISES the stream, stores
 * the totals in packed->nnz / ncols / nrec, and returns ROSKO_EINVAL for
 * invalid input (the packed arrays are then unusable) or ROSKO_ESMALLBUF if
 * the totals exceeded the capacities. */
int32_t rosko_pack_csr_result(const void *ws, size_t ws_bytes, rosko_packed *packed,
                              void *stream);

/* ---- row order (an inspector for the row reordering of Sec. 6) --------
 * Chooses row_perm for rosko_pack_csr from the CSR row lengths alone
 * (stored entries per row, row_ptr [M+1] int64, device):
 *   ROSKO_ORDER_DEGREE:   rows by descending length, ties by ascending row,
 *                         so each panel holds rows of similar density;
 *   ROSKO_ORDER_BALANCED: the length-sorted rows dealt to the panels in a
 *                         serpentine (panel order reversing every round of
 *                         mr rows' worth), so every panel gets one row from
 *                         each band of lengths and the panels' entry counts
 *                         come out close (nonzero-balanced panels).
 * perm [M] int32 (device) receives the order.  ws: device workspace of the
 * size rosko_row_order_workspace_size reports (needs a current device).
 * Asynchronous. */
#define ROSKO_ORDER_DEGREE 0
#define ROSKO_ORDER_BALANCED 1
int32_t rosko_row_order_workspace_size(int64_t M, size_t *bytes);
int32_t rosko_row_order(const int64_t *row_ptr, int64_t M, int32_t mr, int32_t mode, void *ws,
                        size_t ws_bytes, int32_t *perm, void *stream);

/* ---- SpMM (Alg. 2) ------------------------------------------------------ */

/* Device workspace bytes rosko_spmm needs for A (only its shape and mr are
 * read), N columns and `plan` (NULL = the automatic plan): 4*k_split*M*N
 * for the sparse path when k_split > 1, else 0; for the dense path the
 * densified A and transposed B at FP32 size,
 * 4*(ceil(n_panels*mr / 128)*128 + ceil(N / 128)*128) * ceil(K / 32)*32
 * (rounded to 256-byte pieces), enough for either operand type. */
int32_t rosko_spmm_workspace_size(const rosko_packed *A, int64_t N, const rosko_plan *plan,
                                  size_t *bytes);

/* C = A*B (beta = 0) or C += A*B (beta = 1), with A packed, B (device,
 * A->K x N, row-major, ldb >= N) in FP32 (b_dtype ROSKO_F32) or BF16
 * (ROSKO_BF16, raw 16-bit patterns), C (device, A->M x N FP32, ldc >= N).
 * Accumulation is FP32; FP8 values are multiplied by s_m once per output.
 * plan may be NULL (automatic).  ws (device) must hold the bytes
 * rosko_spmm_workspace_size reports for the same plan (may be NULL when that
 * is 0).  Asynchronous. */
int32_t rosko_spmm(const rosko_packed *A, const void *B, int32_t b_dtype, int64_t N,
                   int64_t ldb, float *C, int64_t ldc, int32_t beta, const rosko_plan *plan,
                   void *ws, size_t ws_bytes, void *stream);

/* ---- sparse direct convolution (Sec. 1: the outer-product method applied
 * to convolution without im2col) ----------------------------------------
 * A 3x3 convolution, stride 1, zero padding 1, of a channels-first input X
 * (device FP32, C_in x H x W) with a pruned weight, as the row-skipping
 * product of the packed weight matrix A (C_out x 9*C_in, column
 * c*9 + ky*3 + kx -- the im2col order; packed with rosko_pack) and the input
 * itself.  The output is produced on a padded-pitch grid: Yq[o][y*Wq + x] is
 * Y[o][y][x] for x < W; columns x >= W of each grid row hold values of no
 * meaning.  Row k of the implicit im2col matrix is the run of the
 * zero-padded input (C_in planes of (H+2) x Wq, the image at rows 1..H and
 * columns 1..W) that starts at c*(H+2)*Wq + ky*Wq + kx, so the SpMM kernels
 * run unchanged on records that name those starts; the input is stored four
 * times, copy r shifted left by r elements, so every start is a multiple of
 * 4 elements of one copy (aligned vector loads).  Limit: 4*T < 2^24. */

/* Row pitch Wq (>= W + 2, H*Wq a multiple of 4) and copy length T (host). */
int32_t rosko_conv_geometry(int32_t C_in, int32_t H, int32_t W, int64_t *Wq, int64_t *T);

/* Writes the four shifted copies of the zero-padded input: Bc (device,
 * 4*T floats).  Asynchronous. */
int32_t rosko_conv_input(const float *X, int32_t C_in, int32_t H, int32_t W, float *Bc,
                         void *stream);

/* A's column records with each column index replaced by its tap's start in
 * the four copies (for this C_in, H, W), into rec_out (device, rec_cap >=
 * A->nrec records of 16 dwords).  A->K must be 9*C_in and A->nrec known.
 * Asynchronous. */
int32_t rosko_conv_records(const rosko_packed *A, int32_t C_in, int32_t H, int32_t W,
                           uint32_t *rec_out, int64_t rec_cap, void *stream);

/* Workspace bytes of rosko_conv for A and plan (NULL: automatic), as
 * rosko_spmm's for N = H*Wq columns. */
int32_t rosko_conv_workspace_size(const rosko_packed *A, int32_t H, int32_t W,
                                  const rosko_plan *plan, size_t *bytes);

/* Yq = conv(X) (beta 0) or Yq += conv(X) (beta 1) on the padded-pitch grid:
 * Yq device FP32, A->M x (H*Wq), ldy >= H*Wq; Bc from rosko_conv_input,
 * rec_conv from rosko_conv_records.  Sparse path only (a dense plan returns
 * ROSKO_EUNSUPPORTED); FP8 row scales and A's row order apply as in
 * rosko_spmm.  Asynchronous. */
int32_t rosko_conv(const rosko_packed *A, const uint32_t *rec_conv, const float *Bc,
                   int32_t C_in, int32_t H, int32_t W, float *Yq, int64_t ldy, int32_t beta,
                   const rosko_plan *plan, void *ws, size_t ws_bytes, void *stream);

/* Y (device, C_out x H x W) = the meaningful columns of Yq.  Asynchronous. */
int32_t rosko_conv_unpad(const float *Yq, int64_t ldy, int64_t C_out, int32_t H, int32_t W,
                         float *Y, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid allocation): rosko_spmm on
 * the sparse path with no workspace argument.  The K-split partial tiles go
 * to a device array of ROSKO_NOALLOC_SCRATCH_BYTES inside the library, one
 * per GPU, held until the process ends (its address is looked up on the
 * first call on each device).  Nothing is allocated.  An automatic plan
 * (plan NULL) takes only as many K splits as fit the scratch; a caller's
 * plan whose partials (4 * k_split * M * N bytes) exceed it returns
 * ROSKO_ESMALLBUF, and the dense path returns ROSKO_EUNSUPPORTED.  Every
 * call on one GPU shares that GPU's scratch: calls that overlap in time on
 * one GPU (other streams, other host threads) race and must be serialised
 * by the caller.  No part of the scratch needs to start at zero: a call
 * writes every partial it reads.  Arguments and results otherwise as
 * rosko_spmm.  Asynchronous. */
#define ROSKO_NOALLOC_SCRATCH_BYTES (32u << 20)
int32_t rosko_spmm_noalloc(const rosko_packed *A, const void *B, int32_t b_dtype, int64_t N,
                           int64_t ldb, float *C, int64_t ldc, int32_t beta,
                           const rosko_plan *plan, void *stream);

/* ---- backward of C = A*B (training decomposition, Sec. 5.4) ------------
 * dB = A^T dC, computed as a Rosko SpMM over At, the packed transpose of A
 * (from rosko_pack_transpose; FP32 values).  dA = (dC B^T) restricted to the
 * kept entries of A, written as one FP32 value per kept entry in A's packed
 * order (an SDDMM; pruned entries get no gradient).  dC (device, A->M x N,
 * lddc), B (device FP32, A->K x N, ldb).  dB (device, A->K x N, lddb) or
 * dA_val (device, dA_cap floats, at least A's nnz) may be NULL to skip that
 * gradient; no entry at or beyond dA_cap (or A->nnz_cap) is written, and
 * every index read from A's packed arrays is clamped into A's capacities,
 * so a pack that overflowed its buffers cannot move an access outside them.
 * At may be NULL when dB is.  ws: device workspace (256-byte aligned) of
 * at least the size rosko_spmm_backward_workspace_size reports for the same
 * A (NULL when dA is not wanted), At (NULL when dB is not wanted) and N: the
 * K-split partials of dB's SpMM, and for panels of up to 32 rows the SDDMM's
 * partial dot products over column chunks of N (1024 columns for panels of
 * up to 8 rows, 512 for up to 16, 256 for up to 32; 4 * ceil(N / chunk) *
 * A->nnz_cap bytes when N exceeds one chunk), added in chunk order into dA.
 * A smaller ws returns ROSKO_ESMALLBUF.  Asynchronous. */
int32_t rosko_spmm_backward_workspace_size(const rosko_packed *A, const rosko_packed *At,
                                           int64_t N, size_t *bytes);
int32_t rosko_spmm_backward(const rosko_packed *A, const rosko_packed *At, const float *B,
                            int64_t ldb, const float *dC, int64_t lddc, int64_t N, float *dB,
                            int64_t lddb, float *dA_val, int64_t dA_cap, void *ws,
                            size_t ws_bytes, void *stream);

/* Scatters one FP32 value per stored entry of A, given in A's packed order
 * (as rosko_spmm_backward writes dA), into the dense M x K array out (device,
 * row-major, ldo >= K): out[m][k] = vals[z] for the entry z at (m, k).  Other
 * entries of out are not written (zero-fill them first for a dense
 * gradient).  Only the first min(n_vals, A->nnz_cap) entries are read;
 * indices are clamped as in rosko_spmm_backward.  This is the inverse of
 * packing's value placement (Alg. 1), used to hand the masked weight
 * gradient of the training decomposition (Sec. 5.4) back in the weight's own
 * dense layout.  Asynchronous. */
int32_t rosko_scatter_dense(const rosko_packed *A, const float *vals, int64_t n_vals,
                            float *out, int64_t ldo, void *stream);

/* ---- learned plan selection (in place of Sec. 4.2's analytic tiling; the
 * auto-tuning of the exposed parameters that Sec. 6 leaves open) ----------
 * The choice of panel height mr, register tile and path is made per matrix
 * from ROSKO_NFEAT statistics of A by a Linear(F,H)-ReLU-Linear(H,H)-ReLU-
 * Linear(H,C) network that predicts, for each of the ROSKO_SCHED_CANDIDATES
 * candidates, log(runtime / best runtime); the candidate with the smallest
 * prediction is taken.  The analytic rule is the fallback.  All device
 * arrays are FP32, row-major; every call is asynchronous on `stream`.
 * Candidates (index: path, mr, cols_per_lane):
 *   0: sparse, 8, 4     1: sparse, 16, 4    2: sparse, 32, 4
 *   3: sparse, 32, 2    4: sparse, 64, 2    5: sparse, 128, 1
 *   6: dense-MFMA (packed with mr 32)
 * Feature f (0-based), with "kept" the value test of Alg. 1 and panels of
 * r rows cut as packing cuts them:
 *   0 log2 M, 1 log2 K, 2 log2 N, 3 d = nnz/(M K), 4 log10(d + 1e-6),
 *   5 CV of the row counts, 6 fraction of empty rows, 7 CV of the column
 *   counts, 8 fraction of empty columns, 9 nnz / kept panel columns (r = 32),
 *   10 kept panel columns (r = 32) / (ceil(M/32) K), 11 nnz / kept panel
 *   columns (r = 8), 12 CV of the 32-row panel counts, 13 max / mean of the
 *   32-row panel counts, 14 log2(1 + nnz N), 15 log2(M N)
 * (CV = population standard deviation / mean; a ratio with a zero
 * denominator is 0). */
#define ROSKO_NFEAT 16
#define ROSKO_SCHED_CANDIDATES 7

/* Device workspace bytes rosko_features needs for an M x K matrix. */
int32_t rosko_features_workspace_size(int64_t M, int64_t K, size_t *bytes);
/* features (device, ROSKO_NFEAT floats) of A (device, M x K, lda >= K)
 * multiplied by N columns.  M <= 2^21.  Deterministic (integer counts). */
int32_t rosko_features(const float *A, int64_t M, int64_t K, int64_t lda, int64_t N, void *ws,
                       size_t ws_bytes, float *features, void *stream);

/* Number of parameters of the network: F*H + H + H*H + H + H*C + C, laid
 * out as W1 [F,H], b1 [H], W2 [H,H], b2 [H], W3 [H,C], b3 [C] (W is
 * [in, out]; a layer computes X W + b). */
int32_t rosko_mlp_param_count(int32_t F, int32_t H, int32_t C, int64_t *n);
/* Xn[b][i] = (X[b][i] - mu[i]) / sigma[i] for a batch x F matrix. */
int32_t rosko_mlp_normalize(const float *X, int64_t batch, int32_t F, const float *mu,
                            const float *sigma, float *Xn, void *stream);
/* Forward pass: H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), Y = H2 W3 + b3
 * (H1, H2: batch x H, kept for the backward; Y: batch x C). */
int32_t rosko_mlp_forward(const float *params, int32_t F, int32_t H, int32_t C, const float *X,
                          int64_t batch, float *H1, float *H2, float *Y, void *stream);
/* Loss L = sum(mask (Y - T)^2) / max(1, sum mask) into *loss (device) and
 * its gradient with respect to every parameter into grads (same layout as
 * params).  ws: device scratch of batch * (C + 2 H) floats. */
int32_t rosko_mlp_backward(const float *params, int32_t F, int32_t H, int32_t C, const float *X,
                           const float *H1, const float *H2, const float *Y, const float *T,
                           const float *mask, int64_t batch, float *grads, float *ws,
                           float *loss, void *stream);
/* One Adam step (t >= 1, bias-corrected) over n parameters, in place on
 * params, m and v. */
int32_t rosko_adam_step(float *params, const float *grads, float *m, float *v, int64_t n,
                        float lr, float beta1, float beta2, float eps, int32_t t, void *stream);
/* out[b] = the first index of the smallest entry of row b of Y (batch x C). */
int32_t rosko_argmin_rows(const float *Y, int64_t batch, int32_t C, int32_t *out, void *stream);
/* Candidate `index`: the panel height to pack with (*mr) and the plan to
 * multiply with (waves_per_tile and k_split 0: chosen by the library). */
int32_t rosko_sched_candidate(int32_t index, int32_t *mr, rosko_plan *plan);
/* The analytic fallback rule on host features: a 3 x 3 table over the
 * density (bands at 0.02 and 0.3) and log2 N (bands at 6 and 11) whose cells
 * hold the candidate fastest (geometric mean of repack + SpMM time) over the
 * training problems of the random-shape corpus in that cell:
 *   d < 0.02:        N < 64: 0, N < 2048: 1, else 3
 *   0.02 <= d < 0.3: N < 64: 1, else 3
 *   d >= 0.3:        N < 64: 1, N < 2048: 3, else 6 (dense-MFMA). */
int32_t rosko_sched_analytic(const float *features_host, int32_t *index);

/* The value-type rule: the network and the analytic rule were fitted on
 * FP32 values times FP32 B.  When the values are BF16 or FP8 and B is BF16,
 * the dense path runs on the BF16 matrix cores (16x the FP32 vector rate),
 * so from density features_host[3] >= 0.015 it sets *index to the dense
 * candidate (ROSKO_SCHED_CANDIDATES - 1); otherwise *index is left as it is.
 * The threshold is the crossover measured on a 4096 x 4096 matrix times a
 * 4096 x 2048 BF16 B (dense 98-106 us at every density; sparse 123 us at
 * density 0.02, 98-100 us at 0.015, 72-74 us at 0.01); both paths' times
 * scale with N, and the dense one with M*K against the sparse one's nnz, so
 * the crossover is a density.  val_dtype
 * ROSKO_F32 / BF16 / FP8_E4M3, b_dtype ROSKO_F32 / BF16.  Host only. */
int32_t rosko_sched_precision(const float *features_host, int32_t val_dtype, int32_t b_dtype,
                              int32_t *index);

/* Plan selection: the candidate (index, panel height to pack with, plan) for
 * a matrix with statistics features_host (ROSKO_NFEAT host floats, from
 * rosko_features), stored as val_dtype and multiplied by a B of b_dtype.
 * With params (host, the rosko_mlp_param_count(ROSKO_NFEAT, 64,
 * ROSKO_SCHED_CANDIDATES) weights of the plan network, layout as
 * rosko_mlp_*) and its per-feature normalisation mu, sigma (host), the
 * network's forward pass runs on the host in FP32 and its arg-min is taken;
 * with params NULL the analytic rule decides; then rosko_sched_precision
 * applies the value-type rule.  The caller owns the weights (the library
 * stores none).  Synchronous, host only. */
int32_t rosko_plan_select(const float *features_host, const float *params, const float *mu,
                          const float *sigma, int32_t val_dtype, int32_t b_dtype,
                          int32_t *index, int32_t *mr, rosko_plan *plan);

/* ---- errors ----------------------------------------------------------- */
const char *rosko_status_str(int32_t status);
const char *rosko_last_error(void);   /* per host thread; "" if none */
int32_t rosko_abi_version(void);      /* 11 */

#ifdef __cplusplus
}
#endif
#endif /* ROSKO_H */
