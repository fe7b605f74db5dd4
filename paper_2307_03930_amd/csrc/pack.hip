// Rosko packing on gfx950 (Alg. 1, Sec. 4.1), as two or three passes:
//   count  -- values per (panel, column) and per-tile sums,
//   scan   -- exclusive prefix over tiles (one workgroup, exact integers);
//             skipped when there are at most kLocalPrefixTiles tiles, where
//             each write workgroup adds up the sums of the tiles before its
//             own (and the last one closes the pointer arrays),
//   write  -- per (panel, column): col_ind / col_nnz / col_ptr at its slot and
//             the column's values and in-panel rows at its value offset.
// A tile is 64 (panel, column) pairs, one per lane of a one-wavefront
// workgroup, so even small matrices spread over many CUs.
// The flattened index f = p*S + k walks panels, then columns, which is the
// packed order, so the prefix of the counts at f is exactly the value offset
// (and the prefix of "count > 0" the column slot) that Alg. 1's running
// indices reach there.  All arithmetic on offsets is integer, hence the
// packed arrays are bit-identical to a sequential run of Alg. 1.
#include <atomic>
#include <chrono>

#include "encode.h"
#include "internal.h"
#include "pack_batch.h"

namespace rosko {

namespace {

// Values, kept columns and column records of a range of (panel, column)
// pairs; the scans below carry all three.
struct Tri { int64_t a, b, c; };

// Rows i0 .. i0+N-1 of a column into registers, all N loads issued before
// any of them is used.  `last` is the column's entry in a row at or below
// the panel's last row that is still in the matrix (the hot callers pass its
// entry in the matrix's last row, R - 1): an address past it is clamped to
// it (lda > 0), and the caller masks the entries at or past the panel's
// rows.  Every address is an add of the lane-independent offset j * lda and
// a minimum.  A lane-dependent 64-bit row index times lda would take two
// multiplies per row, the second of which reads the high half of a register
// pair that the compiler may have handed to a load still in flight, and the
// wait it then inserts splits the loads into several round trips; the
// scheduling barrier keeps the first use of a row from being placed before
// the last load.
template <int N>
__device__ __forceinline__ void load_col(const float* __restrict__ col, int64_t lda, int i0,
                                         const float* last, float* x) {
  const float* b = col + (int64_t)i0 * lda;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const float* a = b + (int64_t)j * lda;
    x[j] = *(a < last ? a : last);
  }
  __builtin_amdgcn_sched_barrier(0);
}
// The same, clamped to the panel's last row (rows >= 1).
__device__ __forceinline__ void load_rows32(const float* __restrict__ col, int64_t lda, int i0,
                                            int rows, float* x) {
  load_col<32>(col, lda, i0, col + (int64_t)(rows - 1) * lda, x);
}

// Records a kept column of `cnt` values occupies.
__device__ __forceinline__ int64_t n_records(int cnt) {
  return (cnt + kRecVals - 1) / kRecVals;
}

// Inclusive wave prefix sum, then exclusive block prefix.
__device__ __forceinline__ Tri wave_incl_scan(Tri v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t ta = __shfl_up(v.a, d, 64);
    int64_t tb = __shfl_up(v.b, d, 64);
    int64_t tc = __shfl_up(v.c, d, 64);
    if (lane >= d) { v.a += ta; v.b += tb; v.c += tc; }
  }
  return v;
}

// Exclusive scan across a block of blockDim.x threads (multiple of 64, at
// most 1024).  Returns the thread's exclusive prefix; *total gets the sum.
__device__ Tri block_excl_scan(Tri v, Tri* total) {
  __shared__ Tri wsum[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  Tri inc = wave_incl_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  Tri base{0, 0, 0}, tot{0, 0, 0};
  for (int w = 0; w < nw; ++w) {
    if (w < wid) { base.a += wsum[w].a; base.b += wsum[w].b; base.c += wsum[w].c; }
    tot.a += wsum[w].a; tot.b += wsum[w].b; tot.c += wsum[w].c;
  }
  __syncthreads();
  *total = tot;
  return Tri{base.a + inc.a - v.a, base.b + inc.b - v.b, base.c + inc.c - v.c};
}

// Inclusive prefix sum over a wavefront of 32-bit integers with DPP: three
// row shifts of the input, shifts by 4 and 8 inside each 16-lane row, then
// the row totals broadcast forward (row_bcast:15 into rows 1 and 3,
// row_bcast:31 into rows 2 and 3).  Lanes without a source add 0.
__device__ __forceinline__ int wave_incl_sum(int x) {
  int v = x;
  v += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, x, 0x113, 0xf, 0xf, true);   // row_shr:3
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xe, false);  // row_shr:4, lanes 4..15
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xc, false);  // row_shr:8, lanes 8..15
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Exclusive prefix and total of (values, kept columns, records) over a
// one-wavefront tile; per-tile sums fit 32 bits (64 columns of at most 256
// rows).
struct Tri32 { int a, b, c; };
__device__ __forceinline__ Tri32 wave_excl_scan3(int c, Tri32* total) {
  const int b = c != 0, r = (int)n_records(c);
  const int ia = wave_incl_sum(c), ib = wave_incl_sum(b), ic = wave_incl_sum(r);
  *total = Tri32{__builtin_amdgcn_readlane(ia, 63), __builtin_amdgcn_readlane(ib, 63),
                 __builtin_amdgcn_readlane(ic, 63)};
  return Tri32{ia - c, ib - b, ic - r};
}

// ------------------------------------------------------------------ count
// Tile t covers flattened indices [t*T, t*T+T), T = 64 * CPL; lane x handles
// f = t*T + 64*j + x for j < CPL (at every j adjacent lanes -> adjacent
// columns, so the row loads are coalesced).  CPL = 1: all rows of the column
// in batches of 32; CPL > 1 (mr <= 32 / CPL): the column's rows in one batch
// of 32 / CPL loads.
template <int CPL, int RR>
__global__ void __launch_bounds__(kPackThreads)
k_pack_count(const float* __restrict__ A, int64_t R, int64_t S, int64_t lda, int32_t mr,
             int64_t P, int32_t* __restrict__ counts, int64_t* __restrict__ tile_sums) {
  static_assert(kPackTile == 64 && kPackThreads == 64, "one wavefront per tile");
  static_assert(RR == 32 ? CPL == 1 : CPL * RR <= 32, "rows per lane load");
  // rows per pair: RR (the panel height bound) in one load round, or for
  // RR = 32 (one pair per lane, panels above 16 rows) batches of 32
  constexpr int RMAX = RR;
  const int64_t total = P * S;
  const int64_t fb = (int64_t)blockIdx.x * (64 * CPL) + threadIdx.x;
  Tri32 sum{0, 0, 0};
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int64_t f = fb + 64 * j;
    int c = 0;
    if (f < total) {
      const int64_t p = f / S, k = f - p * S;
      const int64_t r0 = p * mr;
      const int rows = (int)((R - r0) < mr ? (R - r0) : mr);
      const float* col = A + r0 * lda + k;
      const float* last = A + (R - 1) * lda + k;
      if constexpr (RR == 32) {
        for (int i0 = 0; i0 < rows; i0 += 32) {
          float x[32];
          load_col<32>(col, lda, i0, last, x);
#pragma unroll
          for (int i = 0; i < 32; ++i) c += (i0 + i < rows) & kept(x[i]);
        }
      } else {
        float x[RMAX];
        load_col<RMAX>(col, lda, 0, last, x);
#pragma unroll
        for (int i = 0; i < RMAX; ++i) c += (i < rows) & kept(x[i]);
      }
      counts[f] = c;
    }
    Tri32 t;
    (void)wave_excl_scan3(c, &t);
    sum.a += t.a;
    sum.b += t.b;
    sum.c += t.c;
  }
  if (threadIdx.x == 0) {
    tile_sums[3 * blockIdx.x] = sum.a;
    tile_sums[3 * blockIdx.x + 1] = sum.b;
    tile_sums[3 * blockIdx.x + 2] = sum.c;
  }
}

// Totals (nnz, ncols, overflow flag, nrec) and the closing entries of the
// pointer arrays, from the grand sums; one thread.
__device__ void close_packing(Tri tot, int64_t* __restrict__ totals, int64_t P, int64_t S,
                              int64_t nnz_cap, int64_t ncols_cap, int64_t nrec_cap,
                              int64_t* __restrict__ panel_nz_ptr,
                              int64_t* __restrict__ panel_col_ptr, int64_t* __restrict__ col_ptr,
                              int64_t* __restrict__ kblk_ptr) {
  const int64_t nkb = (S + ROSKO_KSTEP - 1) / ROSKO_KSTEP;
  totals[0] = tot.a;
  totals[1] = tot.b;
  totals[2] = (tot.a > nnz_cap || tot.b > ncols_cap || tot.c > nrec_cap) ? 1 : 0;
  totals[3] = tot.c;
  if (panel_nz_ptr) {
    panel_nz_ptr[P] = tot.a;
    panel_col_ptr[P] = tot.b;
    if (tot.b <= ncols_cap) col_ptr[tot.b] = tot.a;
    if (P > 0) kblk_ptr[(P - 1) * (nkb + 1) + nkb] = tot.c;   // end of the last panel
  }
}

// ------------------------------------------------------------------- scan
// One workgroup: exclusive prefix over the tile sums, totals, the overflow
// flag, and the closing entries of the pointer arrays.
constexpr int kScanThreads = 1024;   // 16 wavefronts
constexpr int kScanJ = 8;            // tile rows per wavefront segment
__global__ void __launch_bounds__(kScanThreads)
k_pack_scan(const int64_t* __restrict__ tile_sums, int64_t* __restrict__ tile_offs, int64_t NT,
            int64_t* __restrict__ totals, int64_t P, int64_t S, int64_t nnz_cap,
            int64_t ncols_cap, int64_t nrec_cap, int64_t* __restrict__ panel_nz_ptr,
            int64_t* __restrict__ panel_col_ptr, int64_t* __restrict__ col_ptr,
            int64_t* __restrict__ kblk_ptr) {
  // Tiles in chunks of 16 x 64 x kScanJ.  Wavefront w takes the contiguous
  // segment of 64 x kScanJ tiles at w; lane l holds tiles 64 j + l of it
  // (coalesced loads, kept in registers), and the segment is scanned row by
  // row with the 32-bit wave sums: a tile's sums and a segment's totals fit
  // 32 bits (at most 512 tiles of at most 64 x 256 values).  The segment
  // totals are joined in LDS in 64 bits, with the carry of earlier chunks.
  __shared__ int64_t seg[3][kScanThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int NW = kScanThreads / 64;
  constexpr int64_t CH = (int64_t)NW * 64 * kScanJ;
  Tri carry{0, 0, 0};
  for (int64_t base = 0; base < NT; base += CH) {
    const int64_t s0 = base + (int64_t)wid * 64 * kScanJ + lane;
    int va[kScanJ], vb[kScanJ], vc[kScanJ];
#pragma unroll
    for (int j = 0; j < kScanJ; ++j) {
      const int64_t t = s0 + 64 * j;
      const bool ok = t < NT;
      va[j] = ok ? (int)tile_sums[3 * t] : 0;
      vb[j] = ok ? (int)tile_sums[3 * t + 1] : 0;
      vc[j] = ok ? (int)tile_sums[3 * t + 2] : 0;
    }
    int ea[kScanJ], eb[kScanJ], ec[kScanJ];
    int ra = 0, rb = 0, rc = 0;
#pragma unroll
    for (int j = 0; j < kScanJ; ++j) {
      const int ia = wave_incl_sum(va[j]), ib = wave_incl_sum(vb[j]), ic = wave_incl_sum(vc[j]);
      ea[j] = ra + ia - va[j];
      eb[j] = rb + ib - vb[j];
      ec[j] = rc + ic - vc[j];
      ra += __builtin_amdgcn_readlane(ia, 63);
      rb += __builtin_amdgcn_readlane(ib, 63);
      rc += __builtin_amdgcn_readlane(ic, 63);
    }
    if (lane == 0) {
      seg[0][wid] = ra;
      seg[1][wid] = rb;
      seg[2][wid] = rc;
    }
    __syncthreads();
    Tri pre = carry, tot = carry;
#pragma unroll 1
    for (int w = 0; w < NW; ++w) {
      if (w < wid) { pre.a += seg[0][w]; pre.b += seg[1][w]; pre.c += seg[2][w]; }
      tot.a += seg[0][w];
      tot.b += seg[1][w];
      tot.c += seg[2][w];
    }
    __syncthreads();   // seg is rewritten by the next chunk
#pragma unroll
    for (int j = 0; j < kScanJ; ++j) {
      const int64_t t = s0 + 64 * j;
      if (t < NT) {
        tile_offs[3 * t] = pre.a + ea[j];
        tile_offs[3 * t + 1] = pre.b + eb[j];
        tile_offs[3 * t + 2] = pre.c + ec[j];
      }
    }
    carry = tot;
  }
  if (threadIdx.x == 0)
    close_packing(carry, totals, P, S, nnz_cap, ncols_cap, nrec_cap, panel_nz_ptr, panel_col_ptr,
                  col_ptr, kblk_ptr);
  // With no columns at all every panel starts at 0 (the write pass, which
  // sets panel starts at k = 0, has nothing to visit).
  if (S == 0 && panel_nz_ptr) {
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
      panel_nz_ptr[p] = 0;
      panel_col_ptr[p] = 0;
      kblk_ptr[p] = 0;        // nkb = 0: one entry (the end) per panel
    }
  }
}

// The values of one kept column (rows 0..rows-1 of its panel, the first 32
// already in xs): values and in-panel rows at their offset z, and the
// column records (header, row bytes, FP32 values, unused slots zero) from
// record r.  Writes stop at the capacities.
template <int DT>
__device__ __forceinline__ void write_column(const float* __restrict__ col, int64_t lda, int rows,
                                             float* xs, uint32_t k, int64_t r0, int64_t z,
                                             int64_t r, int64_t nnz_cap, int64_t nrec_cap,
                                             uint8_t* __restrict__ loc, void* __restrict__ val,
                                             const float* __restrict__ row_scale,
                                             uint32_t* __restrict__ rec) {
  int in_rec = 0;
  uint32_t lw0 = 0u, lw1 = 0u, lw2 = 0u;     // row bytes of the open record
  auto flush = [&](int cnt) {
    if (r < nrec_cap) {
      uint32_t* d = rec + r * 16;
      *reinterpret_cast<uint4*>(d) = make_uint4((k << 8) | (uint32_t)cnt, lw0, lw1, lw2);
      for (int t = cnt; t < kRecVals; ++t) d[4 + t] = 0u;
    }
    lw0 = lw1 = lw2 = 0u;
    ++r;
  };
  for (int i0 = 0; i0 < rows; i0 += 32) {
    if (i0 > 0) load_rows32(col, lda, i0, rows, xs);
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) {
      const int i = i0 + jj;
      const float x = xs[jj];
      if (i >= rows || !kept(x)) continue;
      uint32_t vbits;
      if (DT == ROSKO_F32) {
        vbits = __float_as_uint(x);
      } else if (DT == ROSKO_BF16) {
        const uint16_t h = enc_bf16(x);
        vbits = dec_bf16(h);
        if (z < nnz_cap) reinterpret_cast<uint16_t*>(val)[z] = h;
      } else {
        const uint8_t q = enc_fp8(__fdiv_rn(x, row_scale[r0 + i]));
        vbits = dec_fp8(q);
        if (z < nnz_cap) reinterpret_cast<uint8_t*>(val)[z] = q;
      }
      if (z < nnz_cap) {
        loc[z] = (uint8_t)i;
        if (DT == ROSKO_F32) reinterpret_cast<float*>(val)[z] = x;
      }
      const uint32_t rb = (uint32_t)i << (8 * (in_rec & 3));
      if (in_rec < 4) lw0 |= rb;
      else if (in_rec < 8) lw1 |= rb;
      else lw2 |= rb;
      if (r < nrec_cap) rec[r * 16 + 4 + in_rec] = vbits;
      ++z;
      if (++in_rec == kRecVals) { flush(kRecVals); in_rec = 0; }
    }
  }
  if (in_rec) flush(in_rec);
}

// ------------------------------------------------------------------ write
// LOCAL: the tile's prefix is the sum of the tile sums before it, added up
// here (lanes stride over the tiles, then a fixed-order wave reduction:
// integers, so any order is exact); the last tile closes the arrays.
// Otherwise the prefix comes from the scan pass (tile_offs).
template <int DT, bool LOCAL>
__global__ void __launch_bounds__(kPackThreads)
k_pack_write(const float* __restrict__ A, int64_t R, int64_t S, int64_t lda, int32_t mr,
             int64_t P, const int32_t* __restrict__ counts, const int64_t* __restrict__ tile_offs,
             const int64_t* __restrict__ tile_sums, int64_t* __restrict__ totals,
             int64_t nnz_cap, int64_t ncols_cap, int64_t* __restrict__ panel_nz_ptr,
             int64_t* __restrict__ panel_col_ptr, int32_t* __restrict__ col_ind,
             int32_t* __restrict__ col_nnz, int64_t* __restrict__ col_ptr,
             uint8_t* __restrict__ loc, void* __restrict__ val,
             const float* __restrict__ row_scale, int64_t* __restrict__ kblk_ptr,
             int64_t nrec_cap, uint32_t* __restrict__ rec) {
  const int64_t total = P * S;
  const int64_t nkb = (S + ROSKO_KSTEP - 1) / ROSKO_KSTEP;
  static_assert(kPackTile == kPackThreads, "one (panel, column) pair per thread");
  const int64_t f = (int64_t)blockIdx.x * kPackTile + threadIdx.x;
  const bool valid = f < total;
  const int c = valid ? counts[f] : 0;
  const int64_t p = valid ? f / S : 0, k = valid ? f - p * S : 0;
  const int64_t r0 = p * mr;
  const int rows = valid ? (int)((R - r0) < mr ? (R - r0) : mr) : 0;
  const float* col = A + r0 * lda + k;
  // the column's first 32 rows, issued before the prefix loads so that the
  // two round trips overlap
  float xs[32];
  if (c > 0) load_rows32(col, lda, 0, rows, xs);
  Tri carry{0, 0, 0};
  if constexpr (LOCAL) {
    static_assert(kPackThreads == 64, "the local prefix is a one-wavefront reduction");
    // lanes stride over the tiles before this one, 8 tiles in flight each
    const int64_t nb = blockIdx.x;
    for (int64_t i = threadIdx.x; i < nb; i += 64 * 8) {
      int64_t va[8], vb[8], vc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t t = (i + 64 * u < nb) ? i + 64 * u : 0;
        va[u] = tile_sums[3 * t];
        vb[u] = tile_sums[3 * t + 1];
        vc[u] = tile_sums[3 * t + 2];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (i + 64 * u < nb) { carry.a += va[u]; carry.b += vb[u]; carry.c += vc[u]; }
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      carry.a += __shfl_xor(carry.a, d, 64);
      carry.b += __shfl_xor(carry.b, d, 64);
      carry.c += __shfl_xor(carry.c, d, 64);
    }
  } else {
    carry = Tri{tile_offs[3 * blockIdx.x], tile_offs[3 * blockIdx.x + 1],
                tile_offs[3 * blockIdx.x + 2]};
  }
  // block scan of the tile in flattened order, plus the carry of the tiles before
  Tri tot;
  const Tri e = block_excl_scan(Tri{c, c != 0, n_records(c)}, &tot);
  const int64_t nz_off = carry.a + e.a;
  const int64_t col_slot = carry.b + e.b;
  const int64_t rec_off = carry.c + e.c;
  if (valid) {
    if (k == 0) {
      panel_nz_ptr[p] = nz_off;
      panel_col_ptr[p] = col_slot;
    }
    // the exclusive record prefix at a block start is the first record of
    // the panel with k >= that start (or the panel's end); at k = 0 it is
    // also the end of the previous panel
    if (k % ROSKO_KSTEP == 0) kblk_ptr[p * (nkb + 1) + k / ROSKO_KSTEP] = rec_off;
    if (k == 0 && p > 0) kblk_ptr[(p - 1) * (nkb + 1) + nkb] = rec_off;
  }
  if (valid && c > 0) {
    if (col_slot < ncols_cap) {
      col_ind[col_slot] = (int32_t)k;
      col_nnz[col_slot] = c;
      col_ptr[col_slot] = nz_off;
    }
    write_column<DT>(col, lda, rows, xs, (uint32_t)k, r0, nz_off, rec_off, nnz_cap, nrec_cap,
                     loc, val, row_scale, rec);
  }
  if constexpr (LOCAL) {
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
      carry.a += tot.a;
      carry.b += tot.b;
      carry.c += tot.c;
      close_packing(carry, totals, P, S, nnz_cap, ncols_cap, nrec_cap, panel_nz_ptr,
                    panel_col_ptr, col_ptr, kblk_ptr);
    }
  }
}

// ------------------------------------------------------- write (mr <= 64)
// Same output as k_pack_write, organised for the SIMD: each lane still reads
// its own column (coalesced across the tile's 64 columns), but instead of
// storing its values one by one it drops every entry into LDS -- a kept one
// into its value slot inside the tile's contiguous output range and its row
// into its record's row words, others into a per-lane discard slot -- so
// there is no branch per row.  The wavefront then copies the ranges out with
// coalesced stores (records as 16-byte vectors, copied from their staged
// images or assembled from the record table and the staged values); the
// per-column arrays go last, so the workgroup barriers (which wait for
// outstanding stores) find none.
// LDS is sized per instantiation from RT, the largest panel height it takes
// (8 with 4 columns per lane, 16 with 2, 32 or 64 with 1): a tile holds at
// most 64 * CPL * RT values in 64 * CPL * ceil(RT / 12) records.  Beyond
// kImageMaxTiles tiles the records are staged only as a 5-dword table
// (header, row words, first value slot) and their 64-byte images built
// during the copy-out, so panels of up to 32 rows need 15-16 KB per
// workgroup and many workgroups share a CU; for fewer tiles the images are
// staged whole (25-29 KB), which shortens each tile's own chain.
constexpr int kLdsMaxRows = 64;
constexpr int64_t kImageMaxTiles = 1024;   // about 4 tiles per CU

// Where a write tile's running offsets start: the scan pass (kPfxScan), the
// sums of the tiles before it from the count pass, added up by the tile
// itself (kPfxLocal), or, with no count pass at all, the aggregates that the
// tiles before it publish as they go (kPfxFused, below).
constexpr int kPfxScan = 0, kPfxLocal = 1, kPfxFused = 2;

// ------------------------------------------------- single-pass prefix
// A tile counts its own columns from the rows it loads for staging, so the
// count pass is not needed; what it still needs is the sum over the tiles
// before it.  Each tile publishes its aggregate (values, kept columns,
// records) as one 64-bit word: the launch's tag in the high half, a marker
// bit and the three counts in the low half (at most 2048 / 256 / 256 in a
// tile of 64 columns per lane-pair, so 13 + 9 + 9 bits).  A word counts only
// if it carries this launch's tag and the marker, so words left by earlier
// launches are never taken.  Then each tile reads the words of all tiles
// before it; one that is not there yet is re-read a few times and, if still
// missing, counted again from A by the whole wavefront, exactly as its own
// tile would.  So the result never depends on another workgroup having run
// (no wait can hang), and every offset is the same exact integer sum as in
// the two-pass forms.
constexpr int kLbPerLane = 16;   // words in flight per lane: 1024 tiles a round

__device__ __forceinline__ uint64_t agg_word(uint32_t tag, Tri32 s) {
  return ((uint64_t)tag << 32) | (uint64_t(1) << 31) | (uint64_t)(uint32_t)s.a |
         ((uint64_t)(uint32_t)s.b << 13) | ((uint64_t)(uint32_t)s.c << 22);
}
__device__ __forceinline__ bool agg_ready(uint64_t w, uint32_t tag) {
  return (uint32_t)(w >> 32) == tag && ((w >> 31) & 1u);
}

// (values, kept columns, records) of tile `tile`, counted from A the way the
// tile itself counts them; the same in every lane.  Called by the whole
// wavefront.
template <int CPL, int RT>
__device__ __forceinline__ Tri32 tile_aggregate(const float* __restrict__ A, int64_t R, int64_t S, int64_t lda,
                                int32_t mr, int64_t total, int64_t tile) {
  constexpr int RMAX = RT < 32 ? RT : 32;   // RT <= 32: one load round holds the panel
  const int lane = threadIdx.x & 63;
  Tri32 sum{0, 0, 0};
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int64_t f = tile * (64 * CPL) + 64 * j + lane;
    int c = 0;
    if (f < total) {
      const int64_t p = f / S, k = f - p * S, r0 = p * mr;
      const int rows = (int)((R - r0) < mr ? (R - r0) : mr);
      const float* col = A + r0 * lda + k;
      float x[RMAX];
      load_col<RMAX>(col, lda, 0, A + (R - 1) * lda + k, x);
#pragma unroll
      for (int i = 0; i < RMAX; ++i) c += (i < rows) & kept(x[i]);
    }
    Tri32 t;
    (void)wave_excl_scan3(c, &t);
    sum.a += t.a;
    sum.b += t.b;
    sum.c += t.c;
  }
  return sum;
}

// lb_issue: the words of tiles base + 64 u + lane, u < kLbPerLane, loaded
// from addresses clamped to the tiles before t (t > 0; words past t are
// ignored by the caller).
__device__ __forceinline__ void lb_issue(const uint64_t* flags, int64_t t, int64_t base,
                                         uint64_t* w) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < kLbPerLane; ++u) {
    const int64_t i = base + 64 * u + lane;
    w[u] = __hip_atomic_load(flags + (i < t ? i : t - 1), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
  // all the loads before any use of their words: the compiler keeps atomic
  // loads in program order and would otherwise test the first word (and so
  // wait for it) before issuing the second
  __builtin_amdgcn_sched_barrier(0);
}

// lookback_sum: the sum of the aggregates of tiles [0, t), read in rounds
// of kLbPerLane words per lane.  Lane l takes tiles l, l + 64, ...;
// the words still missing are re-read together (one round trip per
// re-read, a short sleep between) up to `spin` times.  A round with every
// word present is added up as it is; otherwise the round is done again on
// the slow path (kept out of the unrolled code, so the kernel stays small):
// its words loaded once more and each one still missing counted from A, one
// tile at a time by the whole wavefront.  A word and a count of the same
// tile are the same integers, so either gives the exact sum.
template <int CPL, int RT>
__device__ __forceinline__ Tri lookback_sum(const uint64_t* flags, int64_t t, uint32_t tag,
                                            int32_t spin, const float* __restrict__ A,
                                            int64_t R, int64_t S, int64_t lda, int32_t mr,
                                            int64_t total) {
  const int lane = threadIdx.x & 63;
  Tri acc{0, 0, 0};
  for (int64_t base = 0; base < t; base += 64 * kLbPerLane) {
    uint64_t w[kLbPerLane];
    lb_issue(flags, t, base, w);
    bool miss[kLbPerLane];
#pragma unroll
    for (int u = 0; u < kLbPerLane; ++u)
      miss[u] = base + 64 * u + lane < t && !agg_ready(w[u], tag);
    bool any = false;
    for (int r = 0; r < spin; ++r) {
      any = false;
#pragma unroll
      for (int u = 0; u < kLbPerLane; ++u) any |= miss[u];
      if (!__any(any)) break;
      __builtin_amdgcn_s_sleep(2);
      uint64_t nw[kLbPerLane];
      lb_issue(flags, t, base, nw);
#pragma unroll
      for (int u = 0; u < kLbPerLane; ++u) {
        if (miss[u]) w[u] = nw[u];
        miss[u] = miss[u] && !agg_ready(nw[u], tag);
      }
    }
    any = false;
#pragma unroll
    for (int u = 0; u < kLbPerLane; ++u) any |= miss[u];
    if (!__any(any)) {
#pragma unroll
      for (int u = 0; u < kLbPerLane; ++u) {
        if (base + 64 * u + lane < t) {
          acc.a += (int64_t)(w[u] & 0x1FFFu);
          acc.b += (int64_t)((w[u] >> 13) & 0x1FFu);
          acc.c += (int64_t)((w[u] >> 22) & 0x1FFu);
        }
      }
    } else {
#pragma unroll 1
      for (int u = 0; u < kLbPerLane; ++u) {
        const int64_t i = base + 64 * u + lane;
        uint64_t x = __hip_atomic_load(flags + (i < t ? i : t - 1), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        uint64_t m = __ballot(i < t && !agg_ready(x, tag));
        while (m) {                      // wave-uniform
          const int l = __builtin_ctzll(m);
          m &= m - 1;
          const Tri32 sg = tile_aggregate<CPL, RT>(A, R, S, lda, mr, total, base + 64 * u + l);
          if (lane == l) x = agg_word(tag, sg);
        }
        if (i < t) {
          acc.a += (int64_t)(x & 0x1FFFu);
          acc.b += (int64_t)((x >> 13) & 0x1FFu);
          acc.c += (int64_t)((x >> 22) & 0x1FFu);
        }
      }
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    acc.a += __shfl_xor(acc.a, d, 64);
    acc.b += __shfl_xor(acc.b, d, 64);
    acc.c += __shfl_xor(acc.c, d, 64);
  }
  return acc;
}

template <int DT>
__device__ __forceinline__ uint32_t value_code(float x, const float* __restrict__ row_scale,
                                               int64_t row) {
  if (DT == ROSKO_F32) return __float_as_uint(x);
  if (DT == ROSKO_BF16) return enc_bf16(x);
  return enc_fp8(__fdiv_rn(x, row_scale[row]));
}
template <int DT>
__device__ __forceinline__ uint32_t code_bits(uint32_t code) {
  if (DT == ROSKO_F32) return code;
  if (DT == ROSKO_BF16) return dec_bf16((uint16_t)code);
  return dec_fp8((uint8_t)code);
}

// One tile (64*CPL (panel, column) pairs, one wavefront) of the write pass:
// tile `tile` of a grid of `ntiles` tiles over the matrix.
template <int DT, int PFX, int CPL, int RT, bool TABLE>
__device__ __forceinline__ void pack_write_tile(
    const float* __restrict__ A, int64_t R, int64_t S, int64_t lda, int32_t mr, int64_t P,
    const int32_t* __restrict__ counts, const int64_t* __restrict__ tile_offs,
    const int64_t* __restrict__ tile_sums, uint64_t* flags, uint32_t tag, int32_t spin,
    int32_t publish, int64_t* __restrict__ totals, int64_t nnz_cap, int64_t ncols_cap,
    int64_t* __restrict__ panel_nz_ptr, int64_t* __restrict__ panel_col_ptr,
    int32_t* __restrict__ col_ind, int32_t* __restrict__ col_nnz, int64_t* __restrict__ col_ptr,
    uint8_t* __restrict__ loc, void* __restrict__ val, const float* __restrict__ row_scale,
    int64_t* __restrict__ kblk_ptr, int64_t nrec_cap, uint32_t* __restrict__ rec, int64_t tile,
    int64_t ntiles) {
  static_assert(kPackTile == 64 && kPackThreads == 64, "one wavefront per tile");
  static_assert((CPL == 4 && RT == 8) || (CPL == 2 && RT == 16) ||
                    (CPL == 1 && (RT == 8 || RT == 16 || RT == 32 || RT == kLdsMaxRows)),
                "panel height bound of the instantiation");
  static_assert(PFX != kPfxFused || RT <= 32, "single pass: the whole column in one load round");
  // rows held per column: RT in one load round (RT <= 16, or RT = 32 / CPL),
  // else 32 in batches (one pair per lane, mr up to RT); records per column
  // at most ceil(RT / 12)
  constexpr int RMAX = RT < 32 ? RT : 32;
  constexpr int RPC = (RT + kRecVals - 1) / kRecVals;
  constexpr int kLdsVals = kPackTile * CPL * RT;     // values per tile, at most
  constexpr int kLdsRecs = kPackTile * CPL * RPC;    // records per tile, at most
  static_assert(CPL * RPC * kPackTile <= kLdsRecs && CPL * RMAX * kPackTile <= kLdsVals, "");
  // a tile's values, kept columns and records fit the 13, 9 and 9 bits of its
  // single-pass aggregate word (agg_word)
  static_assert(PFX != kPfxFused ||
                    (kLdsVals <= 0x1FFF && kPackTile * CPL <= 0x1FF && kLdsRecs <= 0x1FF),
                "single-pass aggregate fields");
  // the tile's values / rows as they go out, plus one discard slot per lane
  // for the entries that are not kept
  __shared__ uint32_t s_code[kLdsVals + 64];
  __shared__ uint8_t s_loc[kLdsVals + 64];
  // Records, in one of two forms.  TABLE: kTab dwords per record (header,
  // the three row words, the value slot of its first value), the 64-byte
  // images built from these and the staged values during the copy-out, then
  // one discard dword per lane for the rows of entries that are not kept;
  // the LDS footprint is smallest, for grids of many tiles.  Otherwise the
  // 64-byte images themselves, then a 512-dword discard area (dword 64 +
  // lane a dropped value, dword lane a dropped row, distinct banks); the
  // copy-out is one 16-byte read per store, for grids of a few tiles per CU
  // where a tile's own chain is the time.
  constexpr int kTab = 5;
  constexpr int kRaw = TABLE ? (kLdsRecs * kTab + 64 + 3) / 4 : kLdsRecs * 4 + 128;
  // FP8: the matrix row of each staged value (its scale is applied after
  // staging), so the records are always assembled from the table
  static_assert(DT != ROSKO_FP8_E4M3 || TABLE, "FP8 packs through the record table");
  __shared__ int32_t s_grow[DT == ROSKO_FP8_E4M3 ? kLdsVals + 64 : 1];
  __shared__ uint4 s_raw[kRaw];
  uint32_t* s_tab = reinterpret_cast<uint32_t*>(s_raw);   // TABLE: the table; else dwords
  uint8_t* s_tb = reinterpret_cast<uint8_t*>(s_raw);
  const int lane = threadIdx.x;
  const int64_t total = P * S;
  const int64_t nkb = (S + ROSKO_KSTEP - 1) / ROSKO_KSTEP;
  const int64_t fb = tile * (64 * CPL) + lane;
  const float* A_last = A + (R - 1) * lda;   // the matrix's last row (R >= 1)
  bool valid[CPL];
  int c[CPL], rows[CPL];
  int64_t p[CPL], k[CPL], r0[CPL];
  float xs[32];
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int64_t f = fb + 64 * j;
    valid[j] = f < total;
    if constexpr (PFX != kPfxFused) c[j] = valid[j] ? counts[f] : 0;
    p[j] = valid[j] ? f / S : 0;
    k[j] = valid[j] ? f - p[j] * S : 0;
    r0[j] = p[j] * mr;
    rows[j] = valid[j] ? (int)((R - r0[j]) < mr ? (R - r0[j]) : mr) : 0;
  }
  // rows, with the counts: one round trip (clamped reads of valid memory)
  if constexpr (RT >= 32) {
    if (rows[0] > 0) load_col<32>(A + r0[0] * lda + k[0], lda, 0, A_last + k[0], xs);
  } else {
#pragma unroll
    for (int j = 0; j < CPL; ++j)
      load_col<RMAX>(A + r0[j] * lda + k[j], lda, 0, A_last + k[j], xs + j * RMAX);
  }
  if constexpr (PFX == kPfxFused) {
    // the tile's own counts, from the rows just loaded (all of the panel:
    // RT <= 32 rows in one round)
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      int cnt = 0;
#pragma unroll
      for (int i = 0; i < RMAX; ++i) cnt += (i < rows[j]) & kept(xs[j * RMAX + i]);
      c[j] = cnt;
    }
  }
  // exclusive prefix in flattened order: the columns of j = 0 (lanes in
  // order), then j = 1, ...
  Tri32 e[CPL], run{0, 0, 0};
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    Tri32 t;
    const Tri32 x = wave_excl_scan3(c[j], &t);
    e[j] = Tri32{run.a + x.a, run.b + x.b, run.c + x.c};
    run.a += t.a;
    run.b += t.b;
    run.c += t.c;
  }
  Tri carry{0, 0, 0};
  // single pass: publish this tile's aggregate now; those of the tiles
  // before it are read after the staging below, which needs no offsets (by
  // then most of them are there)
  if constexpr (PFX == kPfxFused) {
    if (publish && lane == 0)
      __hip_atomic_store(flags + tile, agg_word(tag, run), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  } else if constexpr (PFX == kPfxLocal) {
    const int64_t nb = tile;
    for (int64_t i = lane; i < nb; i += 64 * 8) {
      int64_t va[8], vb[8], vc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t t = (i + 64 * u < nb) ? i + 64 * u : 0;
        va[u] = tile_sums[3 * t];
        vb[u] = tile_sums[3 * t + 1];
        vc[u] = tile_sums[3 * t + 2];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (i + 64 * u < nb) { carry.a += va[u]; carry.b += vb[u]; carry.c += vc[u]; }
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      carry.a += __shfl_xor(carry.a, d, 64);
      carry.b += __shfl_xor(carry.b, d, 64);
      carry.c += __shfl_xor(carry.c, d, 64);
    }
  } else {
    carry = Tri{tile_offs[3 * tile], tile_offs[3 * tile + 1], tile_offs[3 * tile + 2]};
  }
  const int nv = min(run.a, kLdsVals), nrec = min(run.c, kLdsRecs);
  // zero the tile's records (unused row bytes and value slots stay zero)
  if constexpr (TABLE) {
    for (int t = lane; t < nrec * kTab; t += 64) s_tab[t] = 0u;
  } else {
    for (int t = lane; t < nrec * 4; t += 64) s_raw[t] = make_uint4(0u, 0u, 0u, 0u);
  }
  __syncthreads();
  // entries -> LDS, no branch per row: a kept entry of rank r in its column
  // goes to value slot vbase + r, and its row to byte r % 12 of the row words
  // of record rbase + r / 12
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int vbase = e[j].a, rbase = e[j].c;
    int rank = 0;
    for (int i0 = 0; i0 < (RT >= 32 ? min(mr, RT) : RMAX); i0 += 32) {
      if (RT >= 32 && i0 > 0 && c[0] > 0 && i0 < rows[0])
        load_col<32>(A + r0[0] * lda + k[0], lda, i0, A_last + k[0], xs);
#pragma unroll
      for (int jj = 0; jj < RMAX; ++jj) {
        const int i = i0 + jj;
        const float x = xs[j * RMAX + jj];
        const int q = rbase + (int)((unsigned)rank / kRecVals), sl = rank - (q - rbase) * kRecVals;
        const bool kp = (c[j] > 0) & (i < rows[j]) & kept(x) & (vbase + rank < kLdsVals) &
                        (q < kLdsRecs);
        // FP8: the raw value and its matrix row now, the division by the row
        // scale and the encoding later for the kept values only
        const uint32_t code = DT == ROSKO_FP8_E4M3
                                  ? __float_as_uint(x)
                                  : value_code<DT>(x, row_scale, r0[j] + (i < rows[j] ? i : 0));
        const int vp = kp ? vbase + rank : kLdsVals + lane;
        s_code[vp] = code;
        s_loc[vp] = (uint8_t)i;
        if constexpr (DT == ROSKO_FP8_E4M3) s_grow[vp] = (int32_t)(r0[j] + i);
        if constexpr (TABLE) {
          const int rb = kp ? (q * kTab + 1) * 4 + sl : (kLdsRecs * kTab + lane) * 4;
          s_tb[rb] = (uint8_t)i;
        } else {
          const int rv = kp ? q * 16 + 4 + sl : kLdsRecs * 16 + 64 + lane;   // value dword
          const int rb = kp ? (q * 16 + 1) * 4 + sl : (kLdsRecs * 16 + lane) * 4;   // row byte
          s_tab[rv] = code_bits<DT>(code);
          s_tb[rb] = (uint8_t)i;
        }
        rank += kp ? 1 : 0;
      }
    }
#pragma unroll
    for (int jr = 0; jr < RPC; ++jr) {
      if (jr * kRecVals < c[j] && rbase + jr < kLdsRecs) {
        const uint32_t h = ((uint32_t)k[j] << 8) | (uint32_t)min(kRecVals, c[j] - jr * kRecVals);
        if constexpr (TABLE) {
          s_tab[(rbase + jr) * kTab] = h;
          s_tab[(rbase + jr) * kTab + 4] = (uint32_t)(vbase + jr * kRecVals);
        } else {
          s_tab[(rbase + jr) * 16] = h;
        }
      }
    }
  }
  __syncthreads();
  if constexpr (DT == ROSKO_FP8_E4M3) {
    // the kept values only: x / s_row (correctly rounded), then E4M3
    for (int t = lane; t < nv; t += 64)
      s_code[t] = value_code<DT>(__uint_as_float(s_code[t]), row_scale, s_grow[t]);
    __syncthreads();
  }
  if constexpr (PFX == kPfxFused)
    carry = lookback_sum<CPL, RT>(flags, tile, tag, spin, A, R, S, lda, mr, total);
  // coalesced copies of the tile's values, rows and records
  const int64_t z0 = carry.a, q0 = carry.c;
#pragma unroll 4
  for (int t = lane; t < nv; t += 64) {
    const int64_t z = z0 + t;
    const uint32_t code = s_code[t];
    const uint8_t row = s_loc[t];
    if (z < nnz_cap) {
      if (DT == ROSKO_F32) reinterpret_cast<uint32_t*>(val)[z] = code;
      else if (DT == ROSKO_BF16) reinterpret_cast<uint16_t*>(val)[z] = (uint16_t)code;
      else reinterpret_cast<uint8_t*>(val)[z] = (uint8_t)code;
      loc[z] = row;
    }
  }
  // record images, 16 bytes per lane: part 0 is the header and row words,
  // parts 1..3 values 4(part-1) .. 4(part-1)+3 (zero past the count)
#pragma unroll 4
  for (int t = lane; t < nrec * 4; t += 64) {
    const int q = t >> 2, part = t & 3;
    const uint32_t* tb = s_tab + q * kTab;
    uint4 w;
    if constexpr (!TABLE) {
      w = s_raw[t];
    } else if (part == 0) {
      w = make_uint4(tb[0], tb[1], tb[2], tb[3]);
    } else {
      const int cnt = (int)(tb[0] & 0xffu), v0 = (int)tb[4], sl = (part - 1) * 4;
      uint32_t x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int vs = v0 + sl + u;
        x[u] = (sl + u < cnt && vs < kLdsVals) ? code_bits<DT>(s_code[vs]) : 0u;
      }
      w = make_uint4(x[0], x[1], x[2], x[3]);
    }
    if (q0 + q < nrec_cap) reinterpret_cast<uint4*>(rec)[q0 * 4 + t] = w;
  }
  // per-column arrays and pointers last: nothing above waits on them
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    if (!valid[j]) continue;
    const int64_t nz_off = carry.a + e[j].a;
    const int64_t col_slot = carry.b + e[j].b;
    const int64_t rec_off = carry.c + e[j].c;
    if (k[j] == 0) {
      panel_nz_ptr[p[j]] = nz_off;
      panel_col_ptr[p[j]] = col_slot;
    }
    if (k[j] % ROSKO_KSTEP == 0) kblk_ptr[p[j] * (nkb + 1) + k[j] / ROSKO_KSTEP] = rec_off;
    if (k[j] == 0 && p[j] > 0) kblk_ptr[(p[j] - 1) * (nkb + 1) + nkb] = rec_off;
    if (c[j] > 0 && col_slot < ncols_cap) {
      col_ind[col_slot] = (int32_t)k[j];
      col_nnz[col_slot] = c[j];
      col_ptr[col_slot] = nz_off;
    }
  }
  if constexpr (PFX != kPfxScan) {
    if (tile == ntiles - 1 && lane == 0) {
      carry.a += run.a;
      carry.b += run.b;
      carry.c += run.c;
      close_packing(carry, totals, P, S, nnz_cap, ncols_cap, nrec_cap, panel_nz_ptr,
                    panel_col_ptr, col_ptr, kblk_ptr);
    }
  }
}

// The write pass of one matrix after its count pass.
template <int DT, int PFX, int CPL, int RT, bool TABLE>
__global__ void __launch_bounds__(kPackThreads)
k_pack_write_lds(const float* __restrict__ A, int64_t R, int64_t S, int64_t lda, int32_t mr,
                 int64_t P, const int32_t* __restrict__ counts,
                 const int64_t* __restrict__ tile_offs, const int64_t* __restrict__ tile_sums,
                 int64_t* __restrict__ totals, int64_t nnz_cap, int64_t ncols_cap,
                 int64_t* __restrict__ panel_nz_ptr, int64_t* __restrict__ panel_col_ptr,
                 int32_t* __restrict__ col_ind, int32_t* __restrict__ col_nnz,
                 int64_t* __restrict__ col_ptr, uint8_t* __restrict__ loc,
                 void* __restrict__ val, const float* __restrict__ row_scale,
                 int64_t* __restrict__ kblk_ptr, int64_t nrec_cap, uint32_t* __restrict__ rec) {
  static_assert(PFX != kPfxFused, "the single pass runs as k_pack_single");
  pack_write_tile<DT, PFX, CPL, RT, TABLE>(
      A, R, S, lda, mr, P, counts, tile_offs, tile_sums, nullptr, 0u, 0, 0, totals, nnz_cap,
      ncols_cap, panel_nz_ptr, panel_col_ptr, col_ind, col_nnz, col_ptr, loc, val, row_scale,
      kblk_ptr, nrec_cap, rec, (int64_t)blockIdx.x, (int64_t)gridDim.x);
}

// The single pass over up to kPackJobs matrices in one grid: job j owns
// tiles [tile0, tile0 + ntiles) of the grid (the jobs in order, job 0 from
// tile 0), and every tile adds up only the words of its own matrix's tiles,
// in that matrix's workspace.  One job is the single pass of one matrix.
struct PackJob {
  const float* A;
  int64_t R, S, lda, P;
  int32_t mr;
  int32_t reserved;
  uint64_t* flags;
  int64_t* totals;
  int64_t nnz_cap, ncols_cap, nrec_cap;
  int64_t* panel_nz_ptr;
  int64_t* panel_col_ptr;
  int32_t* col_ind;
  int32_t* col_nnz;
  int64_t* col_ptr;
  uint8_t* loc;
  void* val;
  const float* row_scale;
  int64_t* kblk_ptr;
  uint32_t* rec;
  int64_t tile0, ntiles;
};
constexpr int kPackJobs = 8;
struct PackJobs {
  PackJob job[kPackJobs];
  int32_t n;
};

template <int DT, int CPL, int RT, bool TABLE>
__global__ void __launch_bounds__(kPackThreads)
k_pack_single(const PackJobs jobs, uint32_t tag, int32_t spin, int32_t publish) {
  const int64_t b = blockIdx.x;
  int j = 0;
#pragma unroll
  for (int i = 1; i < kPackJobs; ++i)
    if (i < jobs.n && b >= jobs.job[i].tile0) j = i;
  const PackJob& J = jobs.job[j];
  const int64_t tile = b - J.tile0;
  if (tile < 0 || tile >= J.ntiles) return;      // a grid larger than its jobs' tiles
  pack_write_tile<DT, kPfxFused, CPL, RT, TABLE>(
      J.A, J.R, J.S, J.lda, J.mr, J.P, nullptr, nullptr, nullptr, J.flags, tag, spin, publish,
      J.totals, J.nnz_cap, J.ncols_cap, J.panel_nz_ptr, J.panel_col_ptr, J.col_ind, J.col_nnz,
      J.col_ptr, J.loc, J.val, J.row_scale, J.kblk_ptr, J.nrec_cap, J.rec, tile, J.ntiles);
}

// -------------------------------------------------------------- row scale
// One wave per row: s_m = max |A[m][k]| / 448 (FP32, correctly rounded),
// 1.0 for an all-zero row; NaN entries never win the comparison.
template <bool VEC>
__global__ void __launch_bounds__(256)
k_row_scale(const float* __restrict__ A, int64_t R, int64_t S, int64_t lda,
            float* __restrict__ scale) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= R) return;
  const float* a = A + row * lda;
  float amax = 0.0f;
  int64_t k0 = 0;
  if constexpr (VEC) {
    // 16-byte rows (A aligned, lda a multiple of 4): the first 4 floor(S/4)
    // entries as float4s, the rest one by one below.  The maximum does not
    // depend on the order the entries are visited in.
    const float4* a4 = reinterpret_cast<const float4*>(a);
    const int64_t n4 = S / 4;
#pragma unroll 4
    for (int64_t k = lane; k < n4; k += 64) {
      const float4 x = a4[k];
      float v = fabsf(x.x);
      if (v > amax) amax = v;
      v = fabsf(x.y);
      if (v > amax) amax = v;
      v = fabsf(x.z);
      if (v > amax) amax = v;
      v = fabsf(x.w);
      if (v > amax) amax = v;
    }
    k0 = n4 * 4;
  }
  for (int64_t k = k0 + lane; k < S; k += 64) {
    const float v = fabsf(a[k]);
    if (v > amax) amax = v;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const float o = __shfl_xor(amax, d, 64);
    if (o > amax) amax = o;
  }
  if (lane == 0) scale[row] = (amax == 0.0f) ? 1.0f : __fdiv_rn(amax, 448.0f);
}

// -------------------------------------------------------------- transpose
// 32x32 tiles through LDS (padded row to avoid bank conflicts).
__global__ void __launch_bounds__(256)
k_transpose(const float* __restrict__ A, int64_t M, int64_t K, int64_t lda,
            float* __restrict__ At) {
  __shared__ float t[32][33];
  const int64_t k0 = (int64_t)blockIdx.x * 32, m0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
#pragma unroll
  for (int i = 0; i < 32; i += 8) {
    const int64_t m = m0 + ty + i, k = k0 + tx;
    t[ty + i][tx] = (m < M && k < K) ? A[m * lda + k] : 0.0f;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 32; i += 8) {
    const int64_t k = k0 + ty + i, m = m0 + tx;
    if (k < K && m < M) At[k * M + m] = t[tx][ty + i];
  }
}

}  // namespace

static void launch_count(const float* A, int64_t R, int64_t S, int64_t lda, int32_t mr,
                         const PackWs& L, int32_t* counts, int64_t* tsum, hipStream_t s) {
  const dim3 grid((unsigned)L.NT), block(kPackThreads);
  if (L.cpl == 4)
    hipLaunchKernelGGL((k_pack_count<4, 8>), grid, block, 0, s, A, R, S, lda, mr, L.P, counts,
                       tsum);
  else if (L.cpl == 2)
    hipLaunchKernelGGL((k_pack_count<2, 16>), grid, block, 0, s, A, R, S, lda, mr, L.P, counts,
                       tsum);
  else if (L.rr == 8)
    hipLaunchKernelGGL((k_pack_count<1, 8>), grid, block, 0, s, A, R, S, lda, mr, L.P, counts,
                       tsum);
  else if (L.rr == 16)
    hipLaunchKernelGGL((k_pack_count<1, 16>), grid, block, 0, s, A, R, S, lda, mr, L.P, counts,
                       tsum);
  else
    hipLaunchKernelGGL((k_pack_count<1, 32>), grid, block, 0, s, A, R, S, lda, mr, L.P, counts,
                       tsum);
}

PackWs pack_ws_layout(int64_t R, int64_t S, int32_t mr, bool transpose) {
  PackWs L{};
  L.P = ceil_div(R, mr);
  L.cpl = pack_cols_per_lane(mr, L.P * S);
  L.rr = pack_rows_per_lane(mr, L.cpl);
  L.NT = ceil_div(L.P * S, (int64_t)kPackTile * L.cpl);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = (size_t)round_up(off + bytes, 256); return o; };
  L.counts = take(sizeof(int32_t) * (size_t)(L.P * S));
  L.tile_sums = take(sizeof(int64_t) * 3 * (size_t)L.NT);
  L.tile_offs = take(sizeof(int64_t) * 3 * (size_t)L.NT);
  L.totals = take(sizeof(int64_t) * 4);
  L.transposed = transpose ? take(sizeof(float) * (size_t)(R * S)) : 0;
  L.bytes = off;
  return L;
}

int32_t launch_pack_count_scan(const float* A, int64_t R, int64_t S, int64_t lda, int32_t mr,
                               void* ws, const PackWs& L, const rosko_packed* out,
                               hipStream_t s) {
  char* w = static_cast<char*>(ws);
  int32_t* counts = reinterpret_cast<int32_t*>(w + L.counts);
  int64_t* tsum = reinterpret_cast<int64_t*>(w + L.tile_sums);
  int64_t* toff = reinterpret_cast<int64_t*>(w + L.tile_offs);
  int64_t* totals = reinterpret_cast<int64_t*>(w + L.totals);
  if (L.NT > INT32_MAX) {
    set_error("matrix too large for the packing grid");
    return ROSKO_EUNSUPPORTED;
  }
  if (L.NT > 0) {
    launch_count(A, R, S, lda, mr, L, counts, tsum, s);
    ROSKO_LAUNCH_CHECK("k_pack_count");
  }
  hipLaunchKernelGGL(k_pack_scan, dim3(1), dim3(kScanThreads), 0, s, tsum, toff, L.NT, totals,
                     L.P, S,
                     out ? out->nnz_cap : INT64_MAX, out ? out->ncols_cap : INT64_MAX,
                     out ? out->nrec_cap : INT64_MAX,
                     out ? out->panel_nz_ptr : nullptr, out ? out->panel_col_ptr : nullptr,
                     out ? out->col_ptr : nullptr, out ? out->kblk_ptr : nullptr);
  ROSKO_LAUNCH_CHECK("k_pack_scan");
  return ROSKO_OK;
}

// Tag of a single-pass launch: distinct for every launch of the process (the
// first one drawn from the clock), so a word an earlier launch left in the
// workspace never carries the tag of a later one.
static std::atomic<uint32_t> g_pack_tag{0};
static std::atomic<int32_t> g_pack_mode{ROSKO_PACK_AUTO};

static uint32_t next_pack_tag() {
  uint32_t t = g_pack_tag.load(std::memory_order_relaxed);
  if (t == 0) {
    const uint32_t seed =
        (uint32_t)std::chrono::steady_clock::now().time_since_epoch().count() | 1u;
    g_pack_tag.compare_exchange_strong(t, seed, std::memory_order_relaxed);
  }
  return g_pack_tag.fetch_add(1, std::memory_order_relaxed);
}

int32_t set_pack_mode(int32_t mode) {
  if (mode != ROSKO_PACK_AUTO && mode != ROSKO_PACK_TWO_PASS && mode != ROSKO_PACK_RECOUNT) {
    set_error("unknown packing mode %d", mode);
    return ROSKO_EINVAL;
  }
  g_pack_mode.store(mode, std::memory_order_relaxed);
  return ROSKO_OK;
}

// The LDS instantiation whose panel-height bound RT covers mr: 8 with 4
// pairs per lane, 16 with 2, and with one pair per lane the rows per lane
// load (8 or 16 for small panels) or 32 / 64 (see pack_cols_per_lane); mr
// above kLdsMaxRows only with one pair per lane.
static int pack_rt(const PackWs& L, int32_t mr) {
  return L.cpl == 4   ? 8
         : L.cpl == 2 ? 16
         : L.rr < 32  ? L.rr
                      : (mr <= 32 ? 32 : kLdsMaxRows);
}

// Single pass (no count launch) for grids of up to kFusedMaxTiles tiles of
// panels of up to 32 rows, unless the stream is being captured into a
// graph: a replay would reuse the launch's tag, so captured packs take the
// two-pass form.
static int32_t single_pass_ok(const PackWs& L, int32_t mr, int rt, int32_t mode, hipStream_t s,
                              bool* ok) {
  *ok = false;
  if (mode != ROSKO_PACK_TWO_PASS && L.NT > 0 && L.NT <= kFusedMaxTiles && mr <= kLdsMaxRows &&
      rt <= 32) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    ROSKO_HIP_CHECK(hipStreamIsCapturing(s, &cap));
    *ok = cap == hipStreamCaptureStatusNone;
  }
  return ROSKO_OK;
}

// One matrix's entry in a single-pass grid, from tile tile0 on; its
// aggregate words live in its workspace where the tile sums would.
static PackJob make_job(const float* A, int64_t R, int64_t S, int64_t lda, int32_t mr, void* ws,
                        const PackWs& L, const rosko_packed* out, int64_t tile0) {
  char* w = static_cast<char*>(ws);
  PackJob j{};
  j.A = A;
  j.R = R;
  j.S = S;
  j.lda = lda;
  j.P = L.P;
  j.mr = mr;
  j.flags = reinterpret_cast<uint64_t*>(w + L.tile_sums);
  j.totals = reinterpret_cast<int64_t*>(w + L.totals);
  j.nnz_cap = out->nnz_cap;
  j.ncols_cap = out->ncols_cap;
  j.nrec_cap = out->nrec_cap;
  j.panel_nz_ptr = out->panel_nz_ptr;
  j.panel_col_ptr = out->panel_col_ptr;
  j.col_ind = out->col_ind;
  j.col_nnz = out->col_nnz;
  j.col_ptr = out->col_ptr;
  j.loc = out->loc;
  j.val = out->val;
  j.row_scale = out->row_scale;
  j.kblk_ptr = out->kblk_ptr;
  j.rec = out->rec;
  j.tile0 = tile0;
  j.ntiles = L.NT;
  return j;
}

// One single-pass launch over the jobs' tiles (`grid` of them in all), all of
// one value type and tile form (cpl, rt, record table), with a fresh tag.
static int32_t launch_single(const PackJobs& jobs, int64_t grid, int32_t val_dtype, int cpl,
                             int rt, bool table, int32_t mode, hipStream_t s) {
  if (grid <= 0) return ROSKO_OK;
  if (grid > INT32_MAX) {
    set_error("matrix too large for the packing grid");
    return ROSKO_EUNSUPPORTED;
  }
  const uint32_t tag = next_pack_tag();
  // the test mode publishes nothing, so every tile recounts every tile
  // before it; re-reads of a missing word before recounting it
  const int32_t publish = mode == ROSKO_PACK_RECOUNT ? 0 : 1;
  const int32_t spin = publish ? kFusedSpin : 1;
#define ROSKO_SINGLE_T(DT, TB)                                                                 \
  (cpl == 4    ? (k_pack_single<DT, 4, 8, TB>)                                                \
   : cpl == 2  ? (k_pack_single<DT, 2, 16, TB>)                                               \
   : rt == 8   ? (k_pack_single<DT, 1, 8, TB>)                                                \
   : rt == 16  ? (k_pack_single<DT, 1, 16, TB>)                                               \
               : (k_pack_single<DT, 1, 32, TB>))
  void (*k)(const PackJobs, uint32_t, int32_t, int32_t);
  if (val_dtype == ROSKO_F32)
    k = table ? ROSKO_SINGLE_T(ROSKO_F32, true) : ROSKO_SINGLE_T(ROSKO_F32, false);
  else if (val_dtype == ROSKO_BF16)
    k = table ? ROSKO_SINGLE_T(ROSKO_BF16, true) : ROSKO_SINGLE_T(ROSKO_BF16, false);
  else
    k = ROSKO_SINGLE_T(ROSKO_FP8_E4M3, true);   // FP8 packs through the record table
#undef ROSKO_SINGLE_T
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kPackThreads), 0, s, jobs, tag, spin,
                     publish);
  ROSKO_LAUNCH_CHECK("k_pack_single");
  return ROSKO_OK;
}

int32_t launch_pack(const float* A, int64_t R, int64_t S, int64_t lda, int32_t mr,
                    int32_t val_dtype, void* ws, const PackWs& L, const rosko_packed* out,
                    hipStream_t s) {
  char* w = static_cast<char*>(ws);
  int32_t* counts = reinterpret_cast<int32_t*>(w + L.counts);
  int64_t* tsum = reinterpret_cast<int64_t*>(w + L.tile_sums);
  int64_t* toff = reinterpret_cast<int64_t*>(w + L.tile_offs);
  int64_t* totals = reinterpret_cast<int64_t*>(w + L.totals);
  const bool lds = mr <= kLdsMaxRows;
  const int rt = pack_rt(L, mr);
  if (lds && mr > rt) {
    set_error("internal: panel height %d above the packing tile's %d rows", mr, rt);
    return ROSKO_EINTERNAL;
  }
  const int32_t mode = g_pack_mode.load(std::memory_order_relaxed);
  bool fused = false;
  int32_t st = single_pass_ok(L, mr, rt, mode, s, &fused);
  if (st) return st;
  const bool local = !fused && L.NT > 0 && L.NT <= kLocalPrefixTiles;
  if (fused) {
    // nothing before the write pass
  } else if (local) {
    launch_count(A, R, S, lda, mr, L, counts, tsum, s);
    ROSKO_LAUNCH_CHECK("k_pack_count");
  } else if ((st = launch_pack_count_scan(A, R, S, lda, mr, ws, L, out, s))) {
    return st;
  }
  if (L.NT == 0) return ROSKO_OK;
  if (!lds) {
#define ROSKO_WRITE_G(DT_, LOC)                                                                \
  hipLaunchKernelGGL((k_pack_write<DT_, LOC>), dim3((unsigned)L.NT), dim3(kPackThreads), 0, s, \
                     A, R, S, lda, mr, L.P, counts, toff, tsum, totals, out->nnz_cap,          \
                     out->ncols_cap, out->panel_nz_ptr, out->panel_col_ptr, out->col_ind,      \
                     out->col_nnz, out->col_ptr, out->loc, out->val, out->row_scale,           \
                     out->kblk_ptr, out->nrec_cap, out->rec)
    if (local) {
      if (val_dtype == ROSKO_F32) ROSKO_WRITE_G(ROSKO_F32, true);
      else if (val_dtype == ROSKO_BF16) ROSKO_WRITE_G(ROSKO_BF16, true);
      else ROSKO_WRITE_G(ROSKO_FP8_E4M3, true);
    } else {
      if (val_dtype == ROSKO_F32) ROSKO_WRITE_G(ROSKO_F32, false);
      else if (val_dtype == ROSKO_BF16) ROSKO_WRITE_G(ROSKO_BF16, false);
      else ROSKO_WRITE_G(ROSKO_FP8_E4M3, false);
    }
#undef ROSKO_WRITE_G
    ROSKO_LAUNCH_CHECK("k_pack_write");
    return ROSKO_OK;
  }
  if (fused) {
    PackJobs jobs{};
    jobs.n = 1;
    jobs.job[0] = make_job(A, R, S, lda, mr, ws, L, out, 0);
    return launch_single(jobs, L.NT, val_dtype, L.cpl, rt, L.NT > kImageMaxTiles, mode, s);
  }
  // record images staged whole for grids of up to kImageMaxTiles tiles (a
  // few per CU: each tile's own chain is the time), as a table above (the
  // smaller LDS footprint lets more workgroups share a CU)
  const bool table = L.NT > kImageMaxTiles;
#define ROSKO_KWRITE_T(DT, PF, TB)                                                             \
  (L.cpl == 4    ? (k_pack_write_lds<DT, PF, 4, 8, TB>)                                       \
   : L.cpl == 2  ? (k_pack_write_lds<DT, PF, 2, 16, TB>)                                      \
   : rt == 8     ? (k_pack_write_lds<DT, PF, 1, 8, TB>)                                       \
   : rt == 16    ? (k_pack_write_lds<DT, PF, 1, 16, TB>)                                      \
                 : (k_pack_write_lds<DT, PF, 1, 32, TB>))
#define ROSKO_KWRITE_T64(DT, PF, TB)                                                           \
  (rt == kLdsMaxRows ? (k_pack_write_lds<DT, PF, 1, kLdsMaxRows, TB>) : ROSKO_KWRITE_T(DT, PF, TB))
#define ROSKO_KWRITE(DT, PF)                                                                   \
  (table ? ROSKO_KWRITE_T64(DT, PF, true) : ROSKO_KWRITE_T64(DT, PF, false))
#define ROSKO_KWRITE_FP8(PF) ROSKO_KWRITE_T64(ROSKO_FP8_E4M3, PF, true)
#define ROSKO_WRITE(KERNEL)                                                                    \
  hipLaunchKernelGGL(KERNEL,                                                                  \
                     dim3((unsigned)L.NT), dim3(kPackThreads), 0, s,                         \
                     A, R, S, lda, mr, L.P, counts, toff, tsum, totals, out->nnz_cap,         \
                     out->ncols_cap, out->panel_nz_ptr, out->panel_col_ptr, out->col_ind,     \
                     out->col_nnz, out->col_ptr, out->loc, out->val, out->row_scale,          \
                     out->kblk_ptr, out->nrec_cap, out->rec)
  if (local) {
    if (val_dtype == ROSKO_F32) ROSKO_WRITE(ROSKO_KWRITE(ROSKO_F32, kPfxLocal));
    else if (val_dtype == ROSKO_BF16) ROSKO_WRITE(ROSKO_KWRITE(ROSKO_BF16, kPfxLocal));
    else ROSKO_WRITE(ROSKO_KWRITE_FP8(kPfxLocal));
  } else {
    if (val_dtype == ROSKO_F32) ROSKO_WRITE(ROSKO_KWRITE(ROSKO_F32, kPfxScan));
    else if (val_dtype == ROSKO_BF16) ROSKO_WRITE(ROSKO_KWRITE(ROSKO_BF16, kPfxScan));
    else ROSKO_WRITE(ROSKO_KWRITE_FP8(kPfxScan));
  }
#undef ROSKO_WRITE
#undef ROSKO_KWRITE
#undef ROSKO_KWRITE_FP8
#undef ROSKO_KWRITE_T
#undef ROSKO_KWRITE_T64
  ROSKO_LAUNCH_CHECK("k_pack_write");
  return ROSKO_OK;
}

int32_t launch_pack_batch(const PackTask* tasks, int32_t n, hipStream_t s) {
  if (n <= 0) return ROSKO_OK;
  if (n > kPackBatchMax) {
    set_error("internal: batch of %d packs above %d", n, kPackBatchMax);
    return ROSKO_EINTERNAL;
  }
  const int32_t mode = g_pack_mode.load(std::memory_order_relaxed);
  // the single-pass form of each task (-1: the task packs on its own)
  int32_t key[kPackBatchMax];
  for (int32_t i = 0; i < n; ++i) {
    const PackTask& t = tasks[i];
    const int rt = pack_rt(t.L, t.mr);
    bool fused = false;
    int32_t st = single_pass_ok(t.L, t.mr, rt, mode, s, &fused);
    if (st) return st;
    if (fused && t.mr > rt) {
      set_error("internal: panel height %d above the packing tile's %d rows", t.mr, rt);
      return ROSKO_EINTERNAL;
    }
    const bool table = t.L.NT > kImageMaxTiles || t.val_dtype == ROSKO_FP8_E4M3;
    key[i] = fused ? ((t.val_dtype * 8 + t.L.cpl) * 64 + rt) * 2 + (table ? 1 : 0) : -1;
    if (!fused) {
      if ((st = launch_pack(t.A, t.R, t.S, t.lda, t.mr, t.val_dtype, t.ws, t.L, t.out, s)))
        return st;
    }
  }
  // the single passes: each form's tasks in order, kPackJobs to a launch
  bool done[kPackBatchMax] = {};
  for (int32_t i = 0; i < n; ++i) {
    if (key[i] < 0 || done[i]) continue;
    PackJobs jobs{};
    int64_t grid = 0;
    for (int32_t j = i; j < n; ++j) {
      if (done[j] || key[j] != key[i]) continue;
      const PackTask& t = tasks[j];
      jobs.job[jobs.n++] = make_job(t.A, t.R, t.S, t.lda, t.mr, t.ws, t.L, t.out, grid);
      grid += t.L.NT;
      done[j] = true;
      if (jobs.n == kPackJobs) {
        int32_t st = launch_single(jobs, grid, tasks[i].val_dtype, tasks[i].L.cpl,
                                   pack_rt(tasks[i].L, tasks[i].mr),
                                   (key[i] & 1) != 0, mode, s);
        if (st) return st;
        jobs = PackJobs{};
        grid = 0;
      }
    }
    if (jobs.n > 0) {
      int32_t st = launch_single(jobs, grid, tasks[i].val_dtype, tasks[i].L.cpl,
                                 pack_rt(tasks[i].L, tasks[i].mr), (key[i] & 1) != 0, mode, s);
      if (st) return st;
    }
  }
  return ROSKO_OK;
}

int32_t launch_row_scale(const float* A, int64_t R, int64_t S, int64_t lda, float* scale,
                         hipStream_t s) {
  if (R == 0) return ROSKO_OK;
  const bool vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
  if (vec)
    hipLaunchKernelGGL(k_row_scale<true>, dim3((unsigned)ceil_div(R, 4)), dim3(256), 0, s, A, R,
                       S, lda, scale);
  else
    hipLaunchKernelGGL(k_row_scale<false>, dim3((unsigned)ceil_div(R, 4)), dim3(256), 0, s, A, R,
                       S, lda, scale);
  ROSKO_LAUNCH_CHECK("k_row_scale");
  return ROSKO_OK;
}

int32_t launch_transpose(const float* A, int64_t M, int64_t K, int64_t lda, float* At,
                         hipStream_t s) {
  if (M == 0 || K == 0) return ROSKO_OK;
  if (ceil_div(M, 32) > 65535 || ceil_div(K, 32) > INT32_MAX) {
    set_error("transpose of a %lld x %lld matrix exceeds the launch grid", (long long)M,
              (long long)K);
    return ROSKO_EUNSUPPORTED;
  }
  dim3 grid((unsigned)ceil_div(K, 32), (unsigned)ceil_div(M, 32));
  hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, A, M, K, lda, At);
  ROSKO_LAUNCH_CHECK("k_transpose");
  return ROSKO_OK;
}

}  // namespace rosko
