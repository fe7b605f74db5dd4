// Packing from compressed sparse rows (CSR), for matrices too large or too
// sparse to hand over densely (graph adjacency matrices: Sec. 5.5), with an
// optional row order chosen by an inspector (the row reordering of Sec. 6).
//
// The packed form is the one Alg. 1 gives for the matrix whose packed row i
// is CSR row perm[i] (row i without a permutation): in every panel the kept
// entries ordered by column, then by row inside the panel.  The panel's
// entries are the concatenation of its rows' CSR segments, in row order, so
// a stable sort of each panel's entries by column alone yields that order
// (entries of one column keep their row order).  The passes:
//   count   -- kept entries per packed row (one wavefront per row), input
//              checks (permutation, row pointers, column range),
//   scan    -- row offsets of the kept entries (panels are contiguous runs),
//   gather  -- per kept entry the key (its column) and the value (its FP32
//              bits and packed row), compacted in packed order,
//   sort    -- segmented stable radix sort by column, one segment per panel
//              (rocPRIM),
//   heads   -- entries whose column differs from the previous one, or that
//              open a panel, open a kept column; an inclusive scan of the
//              head flags numbers the kept columns,
//   columns -- col_ind / col_ptr / loc / val, then per column its count and
//              records, then the panel pointers and the K-block record
//              pointers (a binary search per block).
// Every index is an integer computed exactly, so the arrays are bit-identical
// to a sequential run of Alg. 1 over the permuted dense matrix.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include <algorithm>

#include "encode.h"
#include "internal.h"

namespace rosko {
namespace {

constexpr int kT = 256;           // threads per workgroup of the element-wise passes
constexpr int kRowsPerWg = 4;     // one wavefront per row in the row passes
constexpr int kRowChunks = 4;     // 64-entry chunks of a row loaded together

// bits of the "bad input" word (totals[kTotBad])
constexpr uint64_t kBadPerm = 1, kBadPermDup = 2, kBadRowPtr = 4, kBadCol = 8,
                   kBadDupEntry = 16;

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ void flag_bad(int64_t* totals, uint64_t bits) {
  if (bits) atomicOr(reinterpret_cast<unsigned long long*>(totals + kCsrTotBad),
                     (unsigned long long)bits);
}

// totals (and the permutation marks) to zero; a kernel, not a memset, so that
// the sequence can be captured in a graph.
__global__ void __launch_bounds__(kT)
k_csr_init(int64_t* __restrict__ totals, int32_t* __restrict__ seen, int64_t M) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < kCsrTotals) totals[i] = 0;
  if (seen != nullptr)
    for (int64_t m = i; m < M; m += (int64_t)gridDim.x * kT) seen[m] = 0;
}

// Source row of packed row i, or -1 (flagged) when the permutation is bad.
__device__ __forceinline__ int64_t source_row(const int32_t* __restrict__ perm, int64_t i,
                                              int64_t M, uint64_t* bad) {
  if (perm == nullptr) return i;
  const int64_t m = perm[i];
  if (m < 0 || m >= M) {
    *bad |= kBadPerm;
    return -1;
  }
  return m;
}

// One wavefront per packed row: kept entries (FP32 bits other than the sign
// not all zero, column in [0, K)) -> rowlen[i]; input checks.
__global__ void __launch_bounds__(kT)
k_csr_count(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
            const float* __restrict__ val, const int32_t* __restrict__ perm, int64_t M,
            int64_t K, int64_t nz_in, int64_t* __restrict__ rowlen, int32_t* __restrict__ seen,
            int64_t* __restrict__ totals) {
  const int64_t i = (int64_t)blockIdx.x * kRowsPerWg + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i == 0 && lane == 0) rowlen[M] = 0;   // the scan's last input
  if (i >= M) return;
  uint64_t bad = 0;
  const int64_t m = source_row(perm, i, M, &bad);
  if (m >= 0 && perm != nullptr && lane == 0 && atomicAdd(seen + m, 1) != 0) bad |= kBadPermDup;
  int64_t cnt = 0;
  if (m >= 0) {
    const int64_t b = row_ptr[m], e = row_ptr[m + 1];
    if (b < 0 || e < b || e > nz_in) {
      bad |= kBadRowPtr;
    } else {
      // kRowChunks chunks of 64 entries per pass, their loads issued
      // together from addresses clamped into the row (a hub row of
      // thousands of entries then takes a quarter of the round trips)
      for (int64_t j0 = b; j0 < e; j0 += 64 * kRowChunks) {
        int32_t cc[kRowChunks];
        float xx[kRowChunks];
#pragma unroll
        for (int u = 0; u < kRowChunks; ++u) {
          const int64_t j = std::min<int64_t>(j0 + 64 * u + lane, e - 1);
          cc[u] = col_idx[j];
          xx[u] = val[j];
        }
#pragma unroll
        for (int u = 0; u < kRowChunks; ++u) {
          const bool in = j0 + 64 * u + lane < e;
          const bool col_ok = cc[u] >= 0 && cc[u] < K;
          if (in && !col_ok) bad |= kBadCol;
          cnt += __popcll(__ballot(in && col_ok && kept(xx[u])));
        }
      }
    }
  }
  if (lane == 0) rowlen[i] = cnt;
  flag_bad(totals, bad);
}

// One wavefront per packed row: its kept entries at rowoff[i] onwards, in
// CSR order: key = column, value = (the entry's FP32 bits << 32) | packed row
// (the value travels with the sort, so no later pass gathers it from the
// CSR arrays).
__global__ void __launch_bounds__(kT)
k_csr_gather(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
             const float* __restrict__ val, const int32_t* __restrict__ perm, int64_t M,
             int64_t K, int64_t nz_in, const int64_t* __restrict__ rowoff,
             uint32_t* __restrict__ keys, uint64_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kRowsPerWg + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= M) return;
  uint64_t bad = 0;
  const int64_t m = source_row(perm, i, M, &bad);
  if (m < 0) return;
  const int64_t b = row_ptr[m], e = row_ptr[m + 1];
  if (b < 0 || e < b || e > nz_in) return;
  int64_t pos = rowoff[i];
  const int64_t end = rowoff[i + 1];
  for (int64_t j0 = b; j0 < e; j0 += 64 * kRowChunks) {
    int32_t cc[kRowChunks];
    float xx[kRowChunks];
#pragma unroll
    for (int u = 0; u < kRowChunks; ++u) {
      const int64_t j = std::min<int64_t>(j0 + 64 * u + lane, e - 1);
      cc[u] = col_idx[j];
      xx[u] = val[j];
    }
#pragma unroll
    for (int u = 0; u < kRowChunks; ++u) {
      const bool keep = j0 + 64 * u + lane < e && cc[u] >= 0 && cc[u] < K && kept(xx[u]);
      const uint64_t mask = __ballot(keep);
      const int64_t at = pos + lanes_below(mask);
      if (keep && at < end) {
        keys[at] = (uint32_t)cc[u];
        vals[at] = ((uint64_t)__float_as_uint(xx[u]) << 32) | (uint64_t)i;
      }
      pos += __popcll(mask);
    }
  }
}

// Segment (panel) offsets: pofs[p] = rowoff[min(p * mr, M)], p <= P.
__global__ void __launch_bounds__(kT)
k_csr_pofs(const int64_t* __restrict__ rowoff, int64_t M, int32_t mr, int64_t P,
           int64_t* __restrict__ pofs) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p <= P) pofs[p] = rowoff[std::min(p * mr, M)];
}

// hd[z] = 1 where the sorted key differs from the previous one (z < E), else 0.
__global__ void __launch_bounds__(kT)
k_csr_heads(const uint32_t* __restrict__ keys, const int64_t* __restrict__ rowoff, int64_t M,
            int64_t nz, int32_t* __restrict__ hd) {
  const int64_t z = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (z >= nz) return;
  const int64_t E = rowoff[M];
  hd[z] = (z < E && (z == 0 || keys[z] != keys[z - 1])) ? 1 : 0;
}

// Every non-empty panel opens a column at its first entry.
__global__ void __launch_bounds__(kT)
k_csr_panel_heads(const int64_t* __restrict__ pofs, int64_t P, int32_t* __restrict__ hd) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p < P && pofs[p] < pofs[p + 1]) hd[pofs[p]] = 1;
}

__device__ __forceinline__ int64_t csr_ncols(const int32_t* __restrict__ cid, int64_t E) {
  return E > 0 ? (int64_t)cid[E - 1] : 0;
}

// Per sorted entry z < E: column starts (col_ind, col_ptr and the workspace
// copies), loc and the stored value; duplicate (row, column) entries flagged.
template <int DT, bool WRITE>
__global__ void __launch_bounds__(kT)
k_csr_entries(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ vals,
              const int32_t* __restrict__ hd, const int32_t* __restrict__ cid,
              const int64_t* __restrict__ rowoff, int64_t M, int64_t nz, int32_t mr,
              int32_t* __restrict__ colstart,
              int32_t* __restrict__ colk, int64_t* __restrict__ totals, int32_t* col_ind,
              int64_t* col_ptr, uint8_t* loc, void* val, const float* row_scale,
              int64_t nnz_cap, int64_t ncols_cap) {
  const int64_t z = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (z >= nz) return;
  const int64_t E = rowoff[M];
  if (z >= E) return;
  const int64_t c = (int64_t)cid[z] - 1;
  const uint64_t v = vals[z];
  const int64_t row = (int64_t)(uint32_t)v;          // packed row
  if (hd[z]) {
    colstart[c] = (int32_t)z;
    colk[c] = (int32_t)keys[z];
    if (WRITE && c < ncols_cap) {
      col_ind[c] = (int32_t)keys[z];
      col_ptr[c] = z;
    }
  } else if ((uint32_t)vals[z - 1] == (uint32_t)v) {
    flag_bad(totals, kBadDupEntry);                   // same row and column twice
  }
  if (WRITE) {
    if (z == E - 1 && c + 1 <= ncols_cap) col_ptr[c + 1] = E;
    if (z < nnz_cap) {
      loc[z] = (uint8_t)(row % mr);
      const uint32_t xb = (uint32_t)(v >> 32);
      const float x = __uint_as_float(xb);
      if (DT == ROSKO_F32) reinterpret_cast<uint32_t*>(val)[z] = xb;
      else if (DT == ROSKO_BF16) reinterpret_cast<uint16_t*>(val)[z] = enc_bf16(x);
      else reinterpret_cast<uint8_t*>(val)[z] = enc_fp8(__fdiv_rn(x, row_scale[row]));
    }
  }
}

// Per kept column c < ncols: its count and record count; nr[c] = 0 for
// c >= ncols (c <= nz), so the record scan's total is nrec.
template <bool WRITE>
__global__ void __launch_bounds__(kT)
k_csr_colcnt(const int32_t* __restrict__ colstart, const int32_t* __restrict__ cid,
             const int64_t* __restrict__ rowoff, int64_t M, int64_t nz,
             int32_t* __restrict__ nr, int32_t* col_nnz, int64_t ncols_cap) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c > nz) return;
  const int64_t E = rowoff[M];
  const int64_t ncols = csr_ncols(cid, E);
  if (c >= ncols) {
    nr[c] = 0;
    return;
  }
  const int64_t cnt = ((c + 1 < ncols) ? (int64_t)colstart[c + 1] : E) - colstart[c];
  nr[c] = (int32_t)((cnt + kRecVals - 1) / kRecVals);
  if (WRITE && c < ncols_cap) col_nnz[c] = (int32_t)cnt;
}

// Per kept column: its records (header, row bytes, FP32 values of the stored
// codes, unused slots zero) from rptr[c], one lane per column.  The values
// come with the sorted entries, so each column's chain is its offsets, its
// entries and the stores.  (Four lanes per column, each storing one 16-byte
// part so that a wavefront's stores are contiguous, measured slower: a
// wavefront then covers 16 columns instead of 64 and the grid runs four
// times the dependent-load chains.)
template <int DT>
__global__ void __launch_bounds__(kT)
k_csr_records(const int32_t* __restrict__ colstart, const int32_t* __restrict__ colk,
              const int32_t* __restrict__ cid, const int64_t* __restrict__ rptr,
              const uint64_t* __restrict__ vals, const int64_t* __restrict__ rowoff, int64_t M,
              int64_t nz, int32_t mr, const float* __restrict__ row_scale,
              uint32_t* __restrict__ rec, int64_t nrec_cap) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c >= nz) return;
  // the column's own words are loaded together with the entry total (the
  // arrays hold nz entries, so every index here is in range); only the
  // entries wait for the column count
  const int64_t E = rowoff[M];
  const int64_t z0 = colstart[c];
  const int64_t z1 = colstart[std::min<int64_t>(c + 1, nz - 1)];
  const uint32_t k = (uint32_t)colk[c];
  int64_t r = rptr[c];
  const int64_t ncols = csr_ncols(cid, E);
  if (c >= ncols) return;
  const int64_t cnt = ((c + 1 < ncols) ? z1 : E) - z0;
  for (int64_t q = 0; q < cnt; q += kRecVals, ++r) {
    const int n = (int)std::min<int64_t>(kRecVals, cnt - q);
    uint32_t w[16];
    w[0] = (k << 8) | (uint32_t)n;
    w[1] = w[2] = w[3] = 0u;
#pragma unroll
    for (int u = 0; u < kRecVals; ++u) {
      uint32_t bits = 0u;
      if (u < n) {
        const uint64_t v = vals[z0 + q + u];
        const uint32_t row = (uint32_t)v;
        w[1 + u / 4] |= (row % (uint32_t)mr) << (8 * (u % 4));
        const uint32_t xb = (uint32_t)(v >> 32);
        if (DT == ROSKO_F32) bits = xb;
        else if (DT == ROSKO_BF16) bits = dec_bf16(enc_bf16(__uint_as_float(xb)));
        else bits = dec_fp8(enc_fp8(__fdiv_rn(__uint_as_float(xb), row_scale[row])));
      }
      w[4 + u] = bits;
    }
    if (r < nrec_cap) {
      uint4* d = reinterpret_cast<uint4*>(rec + r * 16);
      d[0] = make_uint4(w[0], w[1], w[2], w[3]);
      d[1] = make_uint4(w[4], w[5], w[6], w[7]);
      d[2] = make_uint4(w[8], w[9], w[10], w[11]);
      d[3] = make_uint4(w[12], w[13], w[14], w[15]);
    }
  }
}

// First kept column of panel p (p <= P): the heads before its first entry.
__device__ __forceinline__ int64_t panel_col(const int64_t* __restrict__ pofs,
                                             const int32_t* __restrict__ cid, int64_t p) {
  const int64_t z = pofs[p];
  return z == 0 ? 0 : (int64_t)cid[z - 1];
}

__global__ void __launch_bounds__(kT)
k_csr_panels(const int64_t* __restrict__ pofs, const int32_t* __restrict__ cid, int64_t P,
             int64_t* __restrict__ panel_nz_ptr, int64_t* __restrict__ panel_col_ptr) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p > P) return;
  panel_nz_ptr[p] = pofs[p];
  panel_col_ptr[p] = panel_col(pofs, cid, p);
}

// kblk_ptr[p * (nkb + 1) + j]: the first record of panel p whose column has
// k >= j * ROSKO_KSTEP (the panel's end for j = nkb or when there is none).
__global__ void __launch_bounds__(kT)
k_csr_kblk(const int64_t* __restrict__ pofs, const int32_t* __restrict__ cid,
           const int32_t* __restrict__ colk, const int64_t* __restrict__ rptr, int64_t P,
           int64_t nkb, int64_t* __restrict__ kblk_ptr) {
  const int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (idx >= P * (nkb + 1)) return;
  const int64_t p = idx / (nkb + 1), j = idx - p * (nkb + 1);
  const int64_t c0 = panel_col(pofs, cid, p), c1 = panel_col(pofs, cid, p + 1);
  int64_t lo = c0, hi = c1;           // first c in [c0, c1) with colk[c] >= j * KSTEP
  if (j < nkb) {
    const int64_t kmin = j * ROSKO_KSTEP;
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if ((int64_t)colk[mid] < kmin) lo = mid + 1;
      else hi = mid;
    }
  } else {
    lo = c1;
  }
  kblk_ptr[idx] = rptr[lo];
}

// Totals and the closing entries; one thread.
__global__ void k_csr_totals(const int64_t* __restrict__ rowoff, const int32_t* __restrict__ cid,
                             const int64_t* __restrict__ rptr, int64_t M,
                             int64_t* __restrict__ totals, int64_t* col_ptr, int64_t nnz_cap,
                             int64_t ncols_cap, int64_t nrec_cap) {
  const int64_t E = M > 0 ? rowoff[M] : 0;
  const int64_t ncols = M > 0 ? csr_ncols(cid, E) : 0;
  const int64_t nrec = M > 0 ? rptr[ncols] : 0;
  totals[kCsrTotNnz] = E;
  totals[kCsrTotNcols] = ncols;
  totals[kCsrTotNrec] = nrec;
  totals[kCsrTotOverflow] = (E > nnz_cap || ncols > ncols_cap || nrec > nrec_cap) ? 1 : 0;
  if (col_ptr != nullptr && E == 0) col_ptr[0] = 0;
}

// No rows: the panel pointers' single entries.
__global__ void k_csr_empty(int64_t* __restrict__ panel_nz_ptr,
                            int64_t* __restrict__ panel_col_ptr) {
  panel_nz_ptr[0] = 0;
  panel_col_ptr[0] = 0;
}

// One wavefront per packed row: s_i = max |x| / 448 over the stored entries
// of its source row (FP32, correctly rounded; NaN never wins), 1.0 when all
// are zero; the same rule the dense packer applies to a dense row.
__global__ void __launch_bounds__(kT)
k_csr_row_scale(const int64_t* __restrict__ row_ptr, const float* __restrict__ val,
                const int32_t* __restrict__ perm, int64_t M, int64_t nz_in,
                float* __restrict__ scale) {
  const int64_t i = (int64_t)blockIdx.x * kRowsPerWg + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= M) return;
  uint64_t bad = 0;
  const int64_t m = source_row(perm, i, M, &bad);
  float amax = 0.0f;
  if (m >= 0) {
    const int64_t b = row_ptr[m], e = row_ptr[m + 1];
    if (b >= 0 && e >= b && e <= nz_in)
      for (int64_t j = b + lane; j < e; j += 64) {
        const float v = fabsf(val[j]);
        if (v > amax) amax = v;
      }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const float o = __shfl_xor(amax, d, 64);
    if (o > amax) amax = o;
  }
  if (lane == 0) scale[i] = (amax == 0.0f) ? 1.0f : __fdiv_rn(amax, 448.0f);
}

// ----------------------------------------------------------- row order
// key[i] = 2^31 - 1 - (entries of row i): an ascending stable sort gives
// descending counts, ties by ascending row.
__global__ void __launch_bounds__(kT)
k_order_keys(const int64_t* __restrict__ row_ptr, int64_t M, uint32_t* __restrict__ keys,
             int32_t* __restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= M) return;
  const int64_t d = row_ptr[i + 1] - row_ptr[i];
  const int64_t dc = d < 0 ? 0 : (d > 0x7FFFFFFF ? 0x7FFFFFFF : d);
  keys[i] = (uint32_t)(0x7FFFFFFF - dc);
  ids[i] = (int32_t)i;
}

// Serpentine dealing of the count-sorted rows to panels: round q gives every
// panel that has a slot q (all but a short last panel beyond its rows) one
// row, panel order ascending in even rounds and descending in odd ones, so
// each panel gets one row from every band of the sorted order.
__global__ void __launch_bounds__(kT)
k_order_deal(const int32_t* __restrict__ sorted, int64_t M, int32_t mr,
             int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= M) return;
  const int64_t P = (M + mr - 1) / mr;
  const int64_t last = M - (P - 1) * mr;            // rows of the last panel
  const int64_t p = i / mr, q = i - p * mr;
  const int64_t before = q * P - (q > last ? q - last : 0);   // slots of rounds < q
  const int64_t np = q < last ? P : P - 1;                      // panels in round q
  const int64_t pos = (q & 1) ? np - 1 - p : p;
  perm[i] = sorted[before + pos];
}

}  // namespace

// ----------------------------------------------------------- host side
CsrWs csr_ws_layout(int64_t M, int64_t nz, int32_t mr) {
  CsrWs L{};
  L.P = (M + mr - 1) / mr;
  L.nz = nz;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (size_t)round_up((int64_t)(off + bytes), 256);
    return o;
  };
  L.totals = take(sizeof(int64_t) * kCsrTotals);
  L.rowlen = take(sizeof(int64_t) * (size_t)(M + 1));
  L.rowoff = take(sizeof(int64_t) * (size_t)(M + 1));
  L.seen = take(sizeof(int32_t) * (size_t)M);
  L.pofs = take(sizeof(int64_t) * (size_t)(L.P + 1));
  L.kin = take(sizeof(uint32_t) * (size_t)nz);
  L.kout = take(sizeof(uint32_t) * (size_t)nz);
  L.vin = take(sizeof(uint64_t) * (size_t)nz);
  L.vout = take(sizeof(uint64_t) * (size_t)nz);
  L.hd = take(sizeof(int32_t) * (size_t)nz);
  L.cid = take(sizeof(int32_t) * (size_t)nz);
  L.colstart = take(sizeof(int32_t) * (size_t)nz);
  L.colk = take(sizeof(int32_t) * (size_t)nz);
  L.nr = take(sizeof(int32_t) * (size_t)(nz + 1));
  L.rptr = take(sizeof(int64_t) * (size_t)(nz + 1));
  L.temp = off;
  L.bytes = off;
  return L;
}

static unsigned key_bits(int64_t K) {
  unsigned b = 1;
  while (b < 32 && ((int64_t)1 << b) < K) ++b;
  return b;
}

// Scratch bytes of the library scans and the sort (device-dependent: the
// library picks its configuration for the current device).
int32_t csr_temp_bytes(const CsrWs& L, int64_t M, int64_t K, size_t* bytes, hipStream_t s) {
  size_t t0 = 0, t1 = 0, t2 = 0, t3 = 0;
  hipError_t e = rocprim::exclusive_scan(nullptr, t0, (const int64_t*)nullptr,
                                         (int64_t*)nullptr, (int64_t)0, (size_t)(M + 1),
                                         rocprim::plus<int64_t>(), s);
  if (e == hipSuccess && L.nz > 0)
    e = rocprim::segmented_radix_sort_pairs(
        nullptr, t1, (const uint32_t*)nullptr, (uint32_t*)nullptr, (const uint64_t*)nullptr,
        (uint64_t*)nullptr, (unsigned)L.nz, (unsigned)L.P, (const int64_t*)nullptr,
        (const int64_t*)nullptr, 0u, key_bits(K), s);
  if (e == hipSuccess && L.nz > 0)
    e = rocprim::inclusive_scan(nullptr, t2, (const int32_t*)nullptr, (int32_t*)nullptr,
                                (size_t)L.nz, rocprim::plus<int32_t>(), s);
  if (e == hipSuccess)
    e = rocprim::exclusive_scan(nullptr, t3, (const int32_t*)nullptr, (int64_t*)nullptr,
                                (int64_t)0, (size_t)(L.nz + 1), rocprim::plus<int64_t>(), s);
  if (e != hipSuccess) {
    set_error("sizing the sort and scan scratch failed: %s", hipGetErrorString(e));
    return ROSKO_EHIP;
  }
  *bytes = std::max(std::max(t0, t1), std::max(t2, t3));
  return ROSKO_OK;
}

static unsigned grid_of(int64_t n, int64_t per) { return (unsigned)ceil_div(n, per); }

int32_t launch_pack_csr(const int64_t* row_ptr, const int32_t* col_idx, const float* val,
                        const int32_t* perm, int64_t M, int64_t K, int64_t nz_in, int32_t mr,
                        int32_t val_dtype, void* ws, size_t ws_bytes, const rosko_packed* out,
                        hipStream_t s) {
  const CsrWs L = csr_ws_layout(M, nz_in, mr);
  char* w = static_cast<char*>(ws);
  int64_t* totals = reinterpret_cast<int64_t*>(w + L.totals);
  int64_t* rowlen = reinterpret_cast<int64_t*>(w + L.rowlen);
  int64_t* rowoff = reinterpret_cast<int64_t*>(w + L.rowoff);
  int32_t* seen = perm ? reinterpret_cast<int32_t*>(w + L.seen) : nullptr;
  int64_t* pofs = reinterpret_cast<int64_t*>(w + L.pofs);
  uint32_t* kin = reinterpret_cast<uint32_t*>(w + L.kin);
  uint32_t* kout = reinterpret_cast<uint32_t*>(w + L.kout);
  uint64_t* vin = reinterpret_cast<uint64_t*>(w + L.vin);
  uint64_t* vout = reinterpret_cast<uint64_t*>(w + L.vout);
  int32_t* hd = reinterpret_cast<int32_t*>(w + L.hd);
  int32_t* cid = reinterpret_cast<int32_t*>(w + L.cid);
  int32_t* colstart = reinterpret_cast<int32_t*>(w + L.colstart);
  int32_t* colk = reinterpret_cast<int32_t*>(w + L.colk);
  int32_t* nr = reinterpret_cast<int32_t*>(w + L.nr);
  int64_t* rptr = reinterpret_cast<int64_t*>(w + L.rptr);
  void* temp = w + L.temp;
  size_t temp_bytes = ws_bytes - L.temp;
  const bool write = out != nullptr;

  hipLaunchKernelGGL(k_csr_init, dim3(std::max(1u, std::min(grid_of(M, kT), 4096u))), dim3(kT),
                     0, s, totals, seen, M);
  ROSKO_LAUNCH_CHECK("k_csr_init");
  if (M == 0) {
    hipLaunchKernelGGL(k_csr_totals, dim3(1), dim3(1), 0, s, rowoff, cid, rptr, M, totals,
                       write ? out->col_ptr : nullptr, write ? out->nnz_cap : 0,
                       write ? out->ncols_cap : 0, write ? out->nrec_cap : 0);
    ROSKO_LAUNCH_CHECK("k_csr_totals");
    if (write) {
      hipLaunchKernelGGL(k_csr_empty, dim3(1), dim3(1), 0, s, out->panel_nz_ptr,
                         out->panel_col_ptr);
      ROSKO_LAUNCH_CHECK("k_csr_empty");
    }
    return ROSKO_OK;
  }
  const unsigned g_rows = grid_of(M, kRowsPerWg);
  hipLaunchKernelGGL(k_csr_count, dim3(g_rows), dim3(kT), 0, s, row_ptr, col_idx, val, perm, M,
                     K, nz_in, rowlen, seen, totals);
  ROSKO_LAUNCH_CHECK("k_csr_count");
  hipError_t e = rocprim::exclusive_scan(temp, temp_bytes, rowlen, rowoff, (int64_t)0,
                                         (size_t)(M + 1), rocprim::plus<int64_t>(), s);
  if (e != hipSuccess) {
    set_error("row offset scan failed: %s", hipGetErrorString(e));
    return ROSKO_EHIP;
  }
  hipLaunchKernelGGL(k_csr_gather, dim3(g_rows), dim3(kT), 0, s, row_ptr, col_idx, val, perm,
                     M, K, nz_in, rowoff, kin, vin);
  ROSKO_LAUNCH_CHECK("k_csr_gather");
  hipLaunchKernelGGL(k_csr_pofs, dim3(grid_of(L.P + 1, kT)), dim3(kT), 0, s, rowoff, M, mr,
                     L.P, pofs);
  ROSKO_LAUNCH_CHECK("k_csr_pofs");
  if (write && val_dtype == ROSKO_FP8_E4M3) {
    hipLaunchKernelGGL(k_csr_row_scale, dim3(g_rows), dim3(kT), 0, s, row_ptr, val, perm, M,
                       nz_in, out->row_scale);
    ROSKO_LAUNCH_CHECK("k_csr_row_scale");
  }
  if (nz_in > 0) {
    e = rocprim::segmented_radix_sort_pairs(temp, temp_bytes, kin, kout, vin, vout,
                                            (unsigned)nz_in, (unsigned)L.P, pofs, pofs + 1, 0u,
                                            key_bits(K), s);
    if (e != hipSuccess) {
      set_error("segmented sort failed: %s", hipGetErrorString(e));
      return ROSKO_EHIP;
    }
    const unsigned g_nz = grid_of(nz_in, kT);
    hipLaunchKernelGGL(k_csr_heads, dim3(g_nz), dim3(kT), 0, s, kout, rowoff, M, nz_in, hd);
    ROSKO_LAUNCH_CHECK("k_csr_heads");
    hipLaunchKernelGGL(k_csr_panel_heads, dim3(grid_of(L.P, kT)), dim3(kT), 0, s, pofs, L.P,
                       hd);
    ROSKO_LAUNCH_CHECK("k_csr_panel_heads");
    e = rocprim::inclusive_scan(temp, temp_bytes, hd, cid, (size_t)nz_in,
                                rocprim::plus<int32_t>(), s);
    if (e != hipSuccess) {
      set_error("column numbering scan failed: %s", hipGetErrorString(e));
      return ROSKO_EHIP;
    }
#define RK_ENT(DT_, W_)                                                                      \
  hipLaunchKernelGGL((k_csr_entries<DT_, W_>), dim3(g_nz), dim3(kT), 0, s, kout, vout, hd,   \
                     cid, rowoff, M, nz_in, mr, colstart, colk, totals,                      \
                     write ? out->col_ind : nullptr, write ? out->col_ptr : nullptr,         \
                     write ? out->loc : nullptr, write ? out->val : nullptr,                 \
                     write ? out->row_scale : nullptr, write ? out->nnz_cap : 0,             \
                     write ? out->ncols_cap : 0)
    if (!write) RK_ENT(ROSKO_F32, false);
    else if (val_dtype == ROSKO_F32) RK_ENT(ROSKO_F32, true);
    else if (val_dtype == ROSKO_BF16) RK_ENT(ROSKO_BF16, true);
    else RK_ENT(ROSKO_FP8_E4M3, true);
#undef RK_ENT
    ROSKO_LAUNCH_CHECK("k_csr_entries");
  }
  if (write)
    hipLaunchKernelGGL(k_csr_colcnt<true>, dim3(grid_of(nz_in + 1, kT)), dim3(kT), 0, s,
                       colstart, cid, rowoff, M, nz_in, nr, out->col_nnz, out->ncols_cap);
  else
    hipLaunchKernelGGL(k_csr_colcnt<false>, dim3(grid_of(nz_in + 1, kT)), dim3(kT), 0, s,
                       colstart, cid, rowoff, M, nz_in, nr, nullptr, (int64_t)0);
  ROSKO_LAUNCH_CHECK("k_csr_colcnt");
  e = rocprim::exclusive_scan(temp, temp_bytes, nr, rptr, (int64_t)0, (size_t)(nz_in + 1),
                              rocprim::plus<int64_t>(), s);
  if (e != hipSuccess) {
    set_error("record offset scan failed: %s", hipGetErrorString(e));
    return ROSKO_EHIP;
  }
  if (write) {
    if (nz_in > 0) {
      const unsigned g_rec = grid_of(nz_in, kT);
#define RK_REC(DT_)                                                                          \
  hipLaunchKernelGGL((k_csr_records<DT_>), dim3(g_rec), dim3(kT), 0, s, colstart, colk, cid, \
                     rptr, vout, rowoff, M, nz_in, mr, out->row_scale, out->rec, out->nrec_cap)
      if (val_dtype == ROSKO_F32) RK_REC(ROSKO_F32);
      else if (val_dtype == ROSKO_BF16) RK_REC(ROSKO_BF16);
      else RK_REC(ROSKO_FP8_E4M3);
#undef RK_REC
      ROSKO_LAUNCH_CHECK("k_csr_records");
    }
    hipLaunchKernelGGL(k_csr_panels, dim3(grid_of(L.P + 1, kT)), dim3(kT), 0, s, pofs, cid,
                       L.P, out->panel_nz_ptr, out->panel_col_ptr);
    ROSKO_LAUNCH_CHECK("k_csr_panels");
    const int64_t nkb = ceil_div(K, ROSKO_KSTEP);
    hipLaunchKernelGGL(k_csr_kblk, dim3(grid_of(L.P * (nkb + 1), kT)), dim3(kT), 0, s, pofs,
                       cid, colk, rptr, L.P, nkb, out->kblk_ptr);
    ROSKO_LAUNCH_CHECK("k_csr_kblk");
  }
  hipLaunchKernelGGL(k_csr_totals, dim3(1), dim3(1), 0, s, rowoff, cid, rptr, M, totals,
                     write ? out->col_ptr : nullptr, write ? out->nnz_cap : 0,
                     write ? out->ncols_cap : 0, write ? out->nrec_cap : 0);
  ROSKO_LAUNCH_CHECK("k_csr_totals");
  return ROSKO_OK;
}

size_t order_ws_bytes_fixed(int64_t M) {
  // keys in/out (uint32), ids in/out (int32), 256-byte pieces
  return 4 * (size_t)round_up(sizeof(uint32_t) * (size_t)M, 256);
}

int32_t order_temp_bytes(int64_t M, size_t* bytes, hipStream_t s) {
  size_t t = 0;
  const hipError_t e = rocprim::radix_sort_pairs(
      nullptr, t, (const uint32_t*)nullptr, (uint32_t*)nullptr, (const int32_t*)nullptr,
      (int32_t*)nullptr, (size_t)M, 0u, 31u, s);
  if (e != hipSuccess) {
    set_error("sizing the row sort scratch failed: %s", hipGetErrorString(e));
    return ROSKO_EHIP;
  }
  *bytes = t;
  return ROSKO_OK;
}

int32_t launch_row_order(const int64_t* row_ptr, int64_t M, int32_t mr, int32_t mode,
                         void* ws, size_t ws_bytes, int32_t* perm, hipStream_t s) {
  if (M == 0) return ROSKO_OK;
  char* w = static_cast<char*>(ws);
  const size_t piece = (size_t)round_up(sizeof(uint32_t) * (size_t)M, 256);
  uint32_t* kin = reinterpret_cast<uint32_t*>(w);
  uint32_t* kout = reinterpret_cast<uint32_t*>(w + piece);
  int32_t* iin = reinterpret_cast<int32_t*>(w + 2 * piece);
  int32_t* iout = reinterpret_cast<int32_t*>(w + 3 * piece);
  hipLaunchKernelGGL(k_order_keys, dim3(grid_of(M, kT)), dim3(kT), 0, s, row_ptr, M, kin, iin);
  ROSKO_LAUNCH_CHECK("k_order_keys");
  size_t tb = ws_bytes - 4 * piece;
  int32_t* sorted = mode == ROSKO_ORDER_DEGREE ? perm : iout;
  const hipError_t e = rocprim::radix_sort_pairs(w + 4 * piece, tb, kin, kout, iin, sorted,
                                                 (size_t)M, 0u, 31u, s);
  if (e != hipSuccess) {
    set_error("row sort failed: %s", hipGetErrorString(e));
    return ROSKO_EHIP;
  }
  if (mode == ROSKO_ORDER_BALANCED) {
    hipLaunchKernelGGL(k_order_deal, dim3(grid_of(M, kT)), dim3(kT), 0, s, iout, M, mr, perm);
    ROSKO_LAUNCH_CHECK("k_order_deal");
  }
  return ROSKO_OK;
}

}  // namespace rosko
