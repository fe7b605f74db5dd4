// dA for C = A*B: the gradient of every kept entry (m, k) of A is the dot
// product of dC row m with B row k; pruned entries get none (an SDDMM on A's
// mask), and the result is written in A's packed order so it lines up with
// the packed values.
//
// Panels of up to 32 rows (the heights the training layers use) take the
// LDS kernel below, over column chunks of N.  The general kernel (any mr, N)
// gives a workgroup one panel; its wavefronts stride over the panel's kept
// columns.  For a column the wave keeps the selected B row in registers
// (lanes over N) and reuses it for every value of the column, which is the
// column-wise reuse the packed format exposes; each value's dot product is
// finished with a wave reduction.
#include <algorithm>

#include "internal.h"

namespace rosko {
namespace {

constexpr int kSdW = 8;        // waves per workgroup
constexpr int kSdMaxV = 32;    // B values held per lane (N <= 2048 in registers)

template <int VB>
__global__ void __launch_bounds__(64 * kSdW)
k_sddmm(const int64_t* __restrict__ panel_col_ptr, const int32_t* __restrict__ col_ind,
        const int32_t* __restrict__ col_nnz, const int64_t* __restrict__ col_ptr,
        const uint8_t* __restrict__ loc, int64_t M, int64_t K, int32_t mr,
        const int32_t* __restrict__ row_perm, const float* __restrict__ dC, int64_t lddc,
        const float* __restrict__ B, int64_t ldb, int64_t N, int64_t ncols_lim, int64_t nz_lim,
        float* __restrict__ dA) {
  const int64_t p = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rows = (int)min((int64_t)mr, M - p * mr);
  // the panel's column range and every index read from the packed arrays are
  // clamped into the caller's buffers, so no content of them can move an
  // access outside (a pack that overflowed its capacities, say)
  const int64_t c_hi = min(panel_col_ptr[p + 1], ncols_lim);
  const int64_t c_lo = min(max(panel_col_ptr[p], (int64_t)0), c_hi);
  for (int64_t c = c_lo + wid; c < c_hi; c += kSdW) {
    const int64_t k = min(max((int64_t)col_ind[c], (int64_t)0), K - 1);
    const int64_t z0 = max(col_ptr[c], (int64_t)0);
    const int n = (int)max((int64_t)0, min((int64_t)col_nnz[c], nz_lim - z0));
    const float* brow = B + k * ldb;
    float b[VB];
#pragma unroll
    for (int j = 0; j < VB; ++j) {
      const int64_t col = lane + 64 * j;
      b[j] = (col < N) ? brow[col] : 0.0f;
    }
    for (int t = 0; t < n; ++t) {
      const int64_t z = z0 + t;
      const int64_t m = p * mr + min((int)loc[z], rows - 1);
      const float* g = dC + perm_row(row_perm, m, M) * lddc;
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

// Sum of a float over the wavefront, in a fixed order, into lane 63: DPP
// row shifts by 1, 2, 4 and 8 inside each 16-lane row, then the row totals
// broadcast forward (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2
// and 3).
#define RK_DPPF(V, CTRL, RM, BM, BC) \
  __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(V), CTRL, RM, BM, BC))
__device__ __forceinline__ float wave_sum_f32(float x) {
  float v = x + RK_DPPF(x, 0x111, 0xf, 0xf, true);   // row_shr:1
  v += RK_DPPF(v, 0x112, 0xf, 0xf, true);            // row_shr:2: sums of 4
  v += RK_DPPF(v, 0x114, 0xf, 0xe, false);           // row_shr:4, lanes 4..15: sums of 8
  v += RK_DPPF(v, 0x118, 0xf, 0xc, false);           // row_shr:8, lanes 8..15: sums of 16
  v += RK_DPPF(v, 0x142, 0xa, 0xf, false);           // row_bcast:15
  v += RK_DPPF(v, 0x143, 0xc, 0xf, false);           // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
#undef RK_DPPF

// Panels of at most ROWS (8, 16 or 32) rows, one chunk of RW = 256 * VQ <= 1024
// columns of dC and B per workgroup.  The workgroup puts its panel's dC rows
// (that column chunk) in LDS once; each of its wavefronts takes a contiguous
// range of the panel's kept columns (the panel's columns are also split over
// kSdLdsG workgroups).  The column metadata and in-panel rows (packed as
// bytes) come in 64 columns at a time, one column per lane.  Lane l holds
// B columns 4l..4l+3 (+256 v) of the chunk as float4s; the B rows of the next
// kSdDepth columns are in flight while a column is computed.  For each of a
// column's values the wave forms the dot product with the LDS row over the
// chunk and reduces it across the wavefront.  With one chunk (N <= RW) the
// result is dA; with several, each chunk writes its partial dot products to
// out + chunk * nz_lim and k_sddmm_sum adds them in chunk order.
constexpr int kSdLdsG = 4;       // workgroups per panel
constexpr int kSdDepth = 4;      // B rows in flight per wavefront
constexpr int kSdChunk = 1024;   // widest column chunk (VQ = 4)
// Column chunk of the LDS kernel by panel height: 1024 columns for panels
// of up to 8 rows (32 KB of dC rows), 512 for up to 16 rows and 256 for up
// to 32 rows (also 32 KB, so as many workgroups share a CU).
inline int64_t sddmm_chunk(int32_t mr) {
  return mr <= 8 ? kSdChunk : (mr <= 16 ? kSdChunk / 2 : kSdChunk / 4);
}
constexpr int32_t kSdLdsMaxRows = 32;

template <int ROWS, int VQ>
__global__ void __launch_bounds__(64 * kSdW)
k_sddmm_lds(const int64_t* __restrict__ panel_col_ptr, const int32_t* __restrict__ col_ind,
            const int32_t* __restrict__ col_nnz, const int64_t* __restrict__ col_ptr,
            const uint8_t* __restrict__ loc, int64_t M, int64_t K, int32_t mr, int32_t n_panels,
            const int32_t* __restrict__ row_perm, const float* __restrict__ dC, int64_t lddc,
            const float* __restrict__ B,
            int64_t ldb, int64_t N, bool vec, int64_t ncols_lim, int64_t nz_lim,
            float* __restrict__ out) {
  constexpr int RW = 256 * VQ;                    // LDS row width (floats)
  constexpr int RWD = ROWS / 4;                   // dwords of row bytes per column
  static_assert(ROWS == 8 || ROWS == 16 || ROWS == 32, "panels of 8, 16 or 32 rows");
  __shared__ float4 sdc4[ROWS * RW / 4];
  float* sdc = reinterpret_cast<float*>(sdc4);
  const int64_t chunk = blockIdx.y;
  const int64_t p = blockIdx.x / kSdLdsG;
  const int g = (int)(blockIdx.x % kSdLdsG);
  const int64_t n0 = chunk * RW;
  float* dst = out + chunk * nz_lim;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = p * mr;
  const int rows = (int)min((int64_t)mr, M - r0);
  // the panel's dC rows (this chunk) into LDS: a thread's loads are all
  // issued before any of its LDS stores, so the fill costs one round trip
  constexpr int PER = ROWS * RW / (64 * kSdW);    // floats per thread
  static_assert(PER * 64 * kSdW == ROWS * RW, "the workgroup covers the LDS rows exactly");
  {
    float v[PER];
    if (rows > 0 && n0 < N) {
      // every load unconditional, from an address inside dC (out-of-range
      // elements re-read the chunk's first element of the panel's first row
      // and keep zero), so the compiler issues them back to back
      int64_t prow[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int r = (threadIdx.x + i * 64 * kSdW) / RW;
        prow[i] = perm_row(row_perm, r0 + (r < rows ? r : rows - 1), M);
      }
      const int64_t base = perm_row(row_perm, r0, M) * lddc + n0;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int idx = threadIdx.x + i * 64 * kSdW;
        const int r = idx / RW, n = idx - r * RW;
        const bool ok = r < rows && n0 + n < N;
        const float x = dC[ok ? prow[i] * lddc + n0 + n : base];
        v[i] = ok ? x : 0.0f;
      }
    } else {
#pragma unroll
      for (int i = 0; i < PER; ++i) v[i] = 0.0f;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) sdc[threadIdx.x + i * 64 * kSdW] = v[i];
  }
  __syncthreads();
  // clamped as in k_sddmm
  const int64_t c_hi = min(panel_col_ptr[p + 1], ncols_lim);
  const int64_t c_lo = min(max(panel_col_ptr[p], (int64_t)0), c_hi);
  const int64_t parts = (int64_t)kSdLdsG * kSdW, part = (int64_t)g * kSdW + w;
  const int64_t a = c_lo + (c_hi - c_lo) * part / parts;
  const int64_t e = c_lo + (c_hi - c_lo) * (part + 1) / parts;
  // B row k at this lane's columns of the chunk; vec: aligned float4 loads,
  // else element loads (columns past N read as 0 and meet zero LDS entries).
  // The chunk's start is folded into the base pointer once, so the loads'
  // addresses carry no per-load offset arithmetic.
  const float* Bn = B + n0;
  const int64_t n_rem = N - n0;
  auto load_b = [&](int64_t k, float4* b) {
    const float* row = Bn + k * ldb;
#pragma unroll
    for (int v = 0; v < VQ; ++v) {
      const int col = 4 * lane + 256 * v;
      if (vec && col < n_rem) {
        b[v] = *reinterpret_cast<const float4*>(row + col);
      } else {
        b[v] = make_float4(col < n_rem ? row[col] : 0.0f, col + 1 < n_rem ? row[col + 1] : 0.0f,
                           col + 2 < n_rem ? row[col + 2] : 0.0f,
                           col + 3 < n_rem ? row[col + 3] : 0.0f);
      }
    }
  };
  for (int64_t cb = a; cb < e; cb += 64) {
    const int64_t c = cb + lane;
    const bool valid = c < e;
    // the three column words, loaded together from an index inside [cb, e)
    // (lanes past the range re-read column e - 1 and keep nothing of it)
    const int64_t cc = valid ? c : e - 1;
    const int32_t ci = col_ind[cc], cn = col_nnz[cc];
    const int64_t cp = col_ptr[cc];
    const int kk = valid ? (int)min(max((int64_t)ci, (int64_t)0), K - 1) : 0;
    const int64_t zz = valid ? max(cp, (int64_t)0) : 0;
    const int nn = valid ? (int)max((int64_t)0, min((int64_t)min(cn, ROWS), nz_lim - zz)) : 0;
    // in-panel rows of the column as bytes: the loads (only the column's own
    // entries) all issued before they are combined
    uint32_t lb[ROWS];
    if (nz_lim > 0) {
      // unconditional byte loads inside [0, nz_lim): the column's own
      // entries, lanes without one re-read entry 0 and keep nothing
#pragma unroll
      for (int t = 0; t < ROWS; ++t) {
        const uint32_t b = loc[nn > 0 ? zz + (t < nn ? t : nn - 1) : 0];
        lb[t] = t < nn ? b : 0u;
      }
    } else {
#pragma unroll
      for (int t = 0; t < ROWS; ++t) lb[t] = 0u;
    }
    uint32_t rw[RWD];
#pragma unroll
    for (int q = 0; q < RWD; ++q) rw[q] = 0u;
#pragma unroll
    for (int t = 0; t < ROWS; ++t) rw[t / 4] |= lb[t] << (8 * (t % 4));
    const int cnt = (int)min<int64_t>(64, e - cb);
    float4 bq[kSdDepth][VQ];
#pragma unroll
    for (int d = 0; d < kSdDepth; ++d)
      load_b(__builtin_amdgcn_readlane(kk, d < cnt ? d : 0), bq[d]);
    for (int j0 = 0; j0 < cnt; j0 += kSdDepth) {
#pragma unroll
      for (int d = 0; d < kSdDepth; ++d) {
        const int j = j0 + d;
        if (j < cnt) {
          const int n = __builtin_amdgcn_readlane(nn, j);
          const int64_t z = ((int64_t)__builtin_amdgcn_readlane((int)(zz >> 32), j) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane((int)zz, j);
          uint32_t rj[RWD];
#pragma unroll
          for (int q = 0; q < RWD; ++q) rj[q] = __builtin_amdgcn_readlane(rw[q], j);
          for (int t = 0; t < n; ++t) {
            uint32_t word;
            if constexpr (RWD == 2) {
              word = t < 4 ? rj[0] : rj[1];
            } else if constexpr (RWD == 4) {
              word = t < 4 ? rj[0] : (t < 8 ? rj[1] : (t < 12 ? rj[2] : rj[3]));
            } else {
              word = rj[0];
#pragma unroll
              for (int q = 1; q < RWD; ++q)
                if ((t >> 2) == q) word = rj[q];
            }
            const int r = (int)((word >> (8 * (t & 3))) & (uint32_t)(ROWS - 1));
            const float4* row = sdc4 + (r * RW) / 4 + lane;
            float acc = 0.0f;
#pragma unroll
            for (int v = 0; v < VQ; ++v) {
              const float4 x = row[64 * v], y = bq[d][v];
              acc = fmaf(x.x, y.x, acc);
              acc = fmaf(x.y, y.y, acc);
              acc = fmaf(x.z, y.z, acc);
              acc = fmaf(x.w, y.w, acc);
            }
            const float sum = wave_sum_f32(acc);
            if (lane == 0) dst[z + t] = sum;
          }
          // this slot's next column, kSdDepth ahead
          const int jn = j + kSdDepth;
          if (jn < cnt) load_b(__builtin_amdgcn_readlane(kk, jn), bq[d]);
        }
      }
    }
  }
}

// dA[z] = sum over chunks c (ascending) of part[c * stride + z], z < nz.
__global__ void __launch_bounds__(256)
k_sddmm_sum(const float* __restrict__ part, int32_t n_chunks, int64_t stride, int64_t nz,
            float* __restrict__ dA) {
  for (int64_t z = (int64_t)blockIdx.x * 256 + threadIdx.x; z < nz;
       z += (int64_t)gridDim.x * 256) {
    float acc = part[z];
    for (int32_t c = 1; c < n_chunks; ++c) acc += part[c * stride + z];
    dA[z] = acc;
  }
}

}  // namespace

size_t sddmm_ws_bytes(const rosko_packed* A, int64_t N) {
  if (A == nullptr || A->mr > kSdLdsMaxRows || N <= sddmm_chunk(A->mr)) return 0;
  return sizeof(float) * (size_t)ceil_div(N, sddmm_chunk(A->mr)) * (size_t)A->nnz_cap;
}

int32_t launch_sddmm(const rosko_packed* A, const float* dC, int64_t lddc, const float* B,
                     int64_t ldb, int64_t N, float* dA_val, int64_t dA_cap, float* ws,
                     size_t ws_bytes, hipStream_t s) {
  if (A->n_panels == 0 || A->K == 0) return ROSKO_OK;
  const int64_t ncols_lim = A->ncols_cap;
  const int64_t nz_lim = std::min(A->nnz_cap, dA_cap);
  if (A->mr <= kSdLdsMaxRows) {
    // LDS path: panels of up to 32 rows, N in chunks of 256 to 1024 columns
    const int64_t chunk = sddmm_chunk(A->mr);
    const int64_t n_chunks = ceil_div(std::max<int64_t>(N, 1), chunk);
    float* out = dA_val;
    if (n_chunks > 1) {
      const size_t need = sizeof(float) * (size_t)n_chunks * (size_t)A->nnz_cap;
      if (ws == nullptr || ws_bytes < need) {
        set_error("backward workspace %zu bytes < %zu (dA partials of %lld column chunks)",
                  ws_bytes, need, (long long)n_chunks);
        return ROSKO_ESMALLBUF;
      }
      out = ws;
    }
    const int64_t nb = (int64_t)A->n_panels * kSdLdsG;
    if (nb > INT32_MAX || n_chunks > 65535) {
      set_error("SDDMM grid too large");
      return ROSKO_EUNSUPPORTED;
    }
    const dim3 grid((unsigned)nb, (unsigned)n_chunks);
    const bool vec = (N % 4 == 0) && (ldb % 4 == 0) && ((uintptr_t)B % 16 == 0);
    const int64_t nz_out = n_chunks > 1 ? A->nnz_cap : nz_lim;
#define RK_SDL(R_, VQ_)                                                                      \
  hipLaunchKernelGGL((k_sddmm_lds<R_, VQ_>), grid, dim3(64 * kSdW), 0, s, A->panel_col_ptr,  \
                     A->col_ind, A->col_nnz, A->col_ptr, A->loc, A->M, A->K, A->mr,          \
                     A->n_panels, A->row_perm, dC, lddc, B, ldb, N, vec, ncols_lim, nz_out,  \
                     out)
    const int64_t nc = n_chunks > 1 ? chunk : N;   // columns of a chunk
    if (A->mr <= 8) {
      if (nc <= 256) RK_SDL(8, 1);
      else if (nc <= 512) RK_SDL(8, 2);
      else RK_SDL(8, 4);
    } else if (A->mr <= 16) {
      if (nc <= 256) RK_SDL(16, 1);
      else RK_SDL(16, 2);
    } else {
      RK_SDL(32, 1);
    }
#undef RK_SDL
    ROSKO_LAUNCH_CHECK("k_sddmm_lds");
    if (n_chunks > 1) {
      const int64_t blocks = std::min<int64_t>(ceil_div(std::max<int64_t>(nz_lim, 1), 256), 65536);
      hipLaunchKernelGGL(k_sddmm_sum, dim3((unsigned)blocks), dim3(256), 0, s, ws,
                         (int32_t)n_chunks, A->nnz_cap, nz_lim, dA_val);
      ROSKO_LAUNCH_CHECK("k_sddmm_sum");
    }
    return ROSKO_OK;
  }
  const int64_t vb = ceil_div(N, 64);
#define RK_SD(VB_)                                                                          \
  hipLaunchKernelGGL(k_sddmm<VB_>, dim3((unsigned)A->n_panels), dim3(64 * kSdW), 0, s,       \
                     A->panel_col_ptr, A->col_ind, A->col_nnz, A->col_ptr, A->loc, A->M,     \
                     A->K, A->mr, A->row_perm, dC, lddc, B, ldb, N, ncols_lim, nz_lim, dA_val)
  if (vb <= 1) RK_SD(1);
  else if (vb <= 4) RK_SD(4);
  else if (vb <= 16) RK_SD(16);
  else RK_SD(kSdMaxV);
#undef RK_SD
  ROSKO_LAUNCH_CHECK("k_sddmm");
  return ROSKO_OK;
}

}  // namespace rosko

// ------------------------------------------------------------------ scatter
// out[row(p*mr + loc[z])][col_ind[c]] = vals[z] for every stored entry z of A
// (row() the optional row order), in
// packed order: the inverse of packing for a dense M x K gradient (the
// weight gradient of the training decomposition is dA on the mask, zero
// elsewhere; the caller zero-fills out).  A panel's kept columns are dealt
// to the threads of several workgroups; indices clamped as in the SDDMM.
namespace rosko {
namespace {
__global__ void __launch_bounds__(256)
k_scatter_dense(const int64_t* __restrict__ panel_col_ptr, const int32_t* __restrict__ col_ind,
                const int32_t* __restrict__ col_nnz, const int64_t* __restrict__ col_ptr,
                const uint8_t* __restrict__ loc, int64_t M, int64_t K, int32_t mr,
                const int32_t* __restrict__ row_perm, int64_t ncols_lim, int64_t nz_lim,
                const float* __restrict__ vals, float* __restrict__ out, int64_t ldo) {
  const int64_t p = blockIdx.x;
  const int rows = (int)min((int64_t)mr, M - p * mr);
  const int64_t c_hi = min(panel_col_ptr[p + 1], ncols_lim);
  const int64_t c_lo = min(max(panel_col_ptr[p], (int64_t)0), c_hi);
  for (int64_t c = c_lo + (int64_t)blockIdx.y * 256 + threadIdx.x; c < c_hi;
       c += (int64_t)gridDim.y * 256) {
    const int64_t k = col_ind[c];
    if (k < 0 || k >= K) continue;
    const int64_t z0 = max(col_ptr[c], (int64_t)0);
    const int64_t n = max((int64_t)0, min((int64_t)col_nnz[c], nz_lim - z0));
    for (int64_t t = 0; t < n; ++t) {
      const int r = loc[z0 + t];
      if (r < rows) out[perm_row(row_perm, p * mr + r, M) * ldo + k] = vals[z0 + t];
    }
  }
}
}  // namespace

int32_t launch_scatter_dense(const rosko_packed* A, const float* vals, int64_t n_vals,
                             float* out, int64_t ldo, hipStream_t s) {
  if (A->n_panels == 0 || A->K == 0) return ROSKO_OK;
  // the panel's kept columns are split over kScatterG workgroups
  constexpr unsigned kScatterG = 16;
  hipLaunchKernelGGL(k_scatter_dense, dim3((unsigned)A->n_panels, kScatterG), dim3(256), 0, s,
                     A->panel_col_ptr, A->col_ind, A->col_nnz, A->col_ptr, A->loc, A->M, A->K,
                     A->mr, A->row_perm, A->ncols_cap, std::min(A->nnz_cap, n_vals), vals, out,
                     ldo);
  ROSKO_LAUNCH_CHECK("k_scatter_dense");
  return ROSKO_OK;
}

}  // namespace rosko
