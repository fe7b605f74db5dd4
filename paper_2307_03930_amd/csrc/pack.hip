// Rosko packing on gfx950 (Alg. 1, Sec. 4.1), as three passes:
//   count  -- values per (panel, column) and per-tile sums,
//   scan   -- exclusive prefix over tiles (one workgroup, exact integers),
//   write  -- per (panel, column): col_ind / col_nnz / col_ptr at its slot and
//             the column's values and in-panel rows at its value offset.
// The flattened index f = p*S + k walks panels, then columns, which is the
// packed order, so the prefix of the counts at f is exactly the value offset
// (and the prefix of "count > 0" the column slot) that Alg. 1's running
// indices reach there.  All arithmetic on offsets is integer, hence the
// packed arrays are bit-identical to a sequential run of Alg. 1.
#include "internal.h"

namespace rosko {

namespace {

// Kept-entry test on the FP32 bits: every bit except the sign.
__device__ __forceinline__ int kept(float x) {
  return (__float_as_uint(x) & 0x7fffffffu) != 0u;
}

// BF16 round-to-nearest-even by integer carry; NaN -> 0x7FC0.
__device__ __forceinline__ uint16_t enc_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7FC0u;
  uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

// OCP E4M3FN, nearest-even, saturating at 448, NaN -> 0x7F.  Normal range
// rounds the FP32 mantissa to 3 bits with a carry into the exponent;
// magnitudes below 2^-6 are scaled by 2^9 (exact) and rounded to an integer
// number of subnormal steps with rintf (nearest-even).
__device__ __forceinline__ uint8_t enc_fp8(float y) {
  uint32_t u = __float_as_uint(y);
  uint32_t sign = (u >> 24) & 0x80u;
  uint32_t a = u & 0x7fffffffu;
  if (a > 0x7f800000u) return (uint8_t)0x7Fu;
  if (a >= 0x43E00000u) return (uint8_t)(sign | 0x7Eu);        // >= 448
  if (a >= 0x3C800000u) {                                       // >= 2^-6
    uint32_t e = (a >> 23) - 127u + 7u;                         // 1..8+7
    uint32_t m = (a >> 20) & 7u;
    uint32_t rest = a & 0xFFFFFu;
    uint32_t code = (e << 3) | m;
    if (rest > 0x80000u || (rest == 0x80000u && (m & 1u))) code += 1u;
    return (uint8_t)(sign | code);
  }
  float q = __uint_as_float(a) * 512.0f;                        // units of 2^-9
  uint32_t code = (uint32_t)rintf(q);                           // 0..8
  return (uint8_t)(sign | code);
}

// Values, kept columns and column records of a range of (panel, column)
// pairs; the scans below carry all three.
struct Tri { int64_t a, b, c; };

// Rows i0 .. i0+31 of a column into registers: 32 independent loads in
// flight at once (addresses clamped to the panel's last row; the caller
// masks entries at or past `rows`).
__device__ __forceinline__ void load_rows32(const float* __restrict__ col, int64_t lda, int i0,
                                            int rows, float* x) {
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const int i = (i0 + j < rows) ? i0 + j : rows - 1;
    x[j] = col[(int64_t)i * lda];
  }
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

// FP32 value of a packed value (FP8: the code's value, unscaled), as bits.
__device__ __forceinline__ uint32_t dec_bf16(uint16_t h) { return (uint32_t)h << 16; }
__device__ __forceinline__ uint32_t dec_fp8(uint8_t c) {
  const uint32_t e = (c >> 3) & 15u, m = c & 7u, s = (uint32_t)(c & 0x80u) << 24;
  if (e == 15 && m == 7) return 0x7FC00000u;
  if (e == 0) return s | __float_as_uint((float)m * 0.001953125f);     // m * 2^-9
  return s | ((e + 120u) << 23) | (m << 20);                            // (1+m/8) 2^(e-7)
}

// ------------------------------------------------------------------ count
// Tile t covers flattened indices [t*256, t*256+256); thread x handles
// f = t*256 + x (adjacent threads -> adjacent columns, so the row loads are
// coalesced), with all rows of its column loaded in batches of 32.
__global__ void __launch_bounds__(kPackThreads)
k_pack_count(const float* __restrict__ A, int64_t R, int64_t S, int64_t lda, int32_t mr,
             int64_t P, int32_t* __restrict__ counts, int64_t* __restrict__ tile_sums) {
  const int64_t total = P * S;
  const int64_t f0 = (int64_t)blockIdx.x * kPackTile;
  int64_t my_nnz = 0, my_cols = 0, my_recs = 0;
#pragma unroll
  for (int j = 0; j < kPackTile / kPackThreads; ++j) {
    const int64_t f = f0 + threadIdx.x + (int64_t)kPackThreads * j;
    if (f < total) {
      const int64_t p = f / S, k = f - p * S;
      const int64_t r0 = p * mr;
      const int rows = (int)((R - r0) < mr ? (R - r0) : mr);
      const float* col = A + r0 * lda + k;
      int c = 0;
      for (int i0 = 0; i0 < rows; i0 += 32) {
        float x[32];
        load_rows32(col, lda, i0, rows, x);
#pragma unroll
        for (int j = 0; j < 32; ++j) c += (i0 + j < rows) & kept(x[j]);
      }
      counts[f] = c;
      my_nnz += c;
      my_cols += (c != 0);
      my_recs += n_records(c);
    }
  }
  Tri tot;
  (void)block_excl_scan(Tri{my_nnz, my_cols, my_recs}, &tot);
  if (threadIdx.x == 0) {
    tile_sums[3 * blockIdx.x] = tot.a;
    tile_sums[3 * blockIdx.x + 1] = tot.b;
    tile_sums[3 * blockIdx.x + 2] = tot.c;
  }
}

// ------------------------------------------------------------------- scan
// One workgroup: exclusive prefix over the tile sums, totals, the overflow
// flag, and the closing entries of the pointer arrays.
__global__ void __launch_bounds__(1024)
k_pack_scan(const int64_t* __restrict__ tile_sums, int64_t* __restrict__ tile_offs, int64_t NT,
            int64_t* __restrict__ totals, int64_t P, int64_t S, int64_t nnz_cap,
            int64_t ncols_cap, int64_t nrec_cap, int64_t* __restrict__ panel_nz_ptr,
            int64_t* __restrict__ panel_col_ptr, int64_t* __restrict__ col_ptr,
            int64_t* __restrict__ kblk_ptr) {
  Tri carry{0, 0, 0};
  for (int64_t base = 0; base < NT; base += 1024) {
    const int64_t i = base + threadIdx.x;
    Tri v{0, 0, 0};
    if (i < NT) v = Tri{tile_sums[3 * i], tile_sums[3 * i + 1], tile_sums[3 * i + 2]};
    Tri tot;
    Tri e = block_excl_scan(v, &tot);
    if (i < NT) {
      tile_offs[3 * i] = carry.a + e.a;
      tile_offs[3 * i + 1] = carry.b + e.b;
      tile_offs[3 * i + 2] = carry.c + e.c;
    }
    carry.a += tot.a;
    carry.b += tot.b;
    carry.c += tot.c;
  }
  const int64_t nkb = (S + ROSKO_KSTEP - 1) / ROSKO_KSTEP;
  if (threadIdx.x == 0) {
    totals[0] = carry.a;
    totals[1] = carry.b;
    totals[2] = (carry.a > nnz_cap || carry.b > ncols_cap || carry.c > nrec_cap) ? 1 : 0;
    totals[3] = carry.c;
    if (panel_nz_ptr) {
      panel_nz_ptr[P] = carry.a;
      panel_col_ptr[P] = carry.b;
      if (carry.b <= ncols_cap) col_ptr[carry.b] = carry.a;
      if (P > 0) kblk_ptr[(P - 1) * (nkb + 1) + nkb] = carry.c;   // end of the last panel
    }
  }
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

// ------------------------------------------------------------------ write
template <int DT>
__global__ void __launch_bounds__(kPackThreads)
k_pack_write(const float* __restrict__ A, int64_t R, int64_t S, int64_t lda, int32_t mr,
             int64_t P, const int32_t* __restrict__ counts, const int64_t* __restrict__ tile_offs,
             int64_t nnz_cap, int64_t ncols_cap, int64_t* __restrict__ panel_nz_ptr,
             int64_t* __restrict__ panel_col_ptr, int32_t* __restrict__ col_ind,
             int32_t* __restrict__ col_nnz, int64_t* __restrict__ col_ptr,
             uint8_t* __restrict__ loc, void* __restrict__ val,
             const float* __restrict__ row_scale, int64_t* __restrict__ kblk_ptr,
             int64_t nrec_cap, uint32_t* __restrict__ rec) {
  const int64_t total = P * S;
  const int64_t nkb = (S + ROSKO_KSTEP - 1) / ROSKO_KSTEP;
  const int64_t f0 = (int64_t)blockIdx.x * kPackTile;
  Tri carry{tile_offs[3 * blockIdx.x], tile_offs[3 * blockIdx.x + 1],
            tile_offs[3 * blockIdx.x + 2]};
  // The tile is visited as four rows of 256 flattened indices; within a row
  // thread x holds f0 + 256*j + x, so a block scan per row plus the carry of
  // the rows before gives the exclusive prefix in flattened order.
#pragma unroll 1
  for (int j = 0; j < kPackTile / kPackThreads; ++j) {
    const int64_t f = f0 + (int64_t)kPackThreads * j + threadIdx.x;
    const int c = (f < total) ? counts[f] : 0;
    Tri tot;
    Tri e = block_excl_scan(Tri{c, c != 0, n_records(c)}, &tot);
    const int64_t nz_off = carry.a + e.a;
    const int64_t col_slot = carry.b + e.b;
    const int64_t rec_off = carry.c + e.c;
    carry.a += tot.a;
    carry.b += tot.b;
    carry.c += tot.c;
    if (f >= total) continue;
    const int64_t p = f / S, k = f - p * S;
    if (k == 0) {
      panel_nz_ptr[p] = nz_off;
      panel_col_ptr[p] = col_slot;
    }
    // the exclusive record prefix at a block start is the first record of
    // the panel with k >= that start (or the panel's end); at k = 0 it is
    // also the end of the previous panel
    if (k % ROSKO_KSTEP == 0) kblk_ptr[p * (nkb + 1) + k / ROSKO_KSTEP] = rec_off;
    if (k == 0 && p > 0) kblk_ptr[(p - 1) * (nkb + 1) + nkb] = rec_off;
    if (c == 0) continue;
    if (col_slot < ncols_cap) {
      col_ind[col_slot] = (int32_t)k;
      col_nnz[col_slot] = c;
      col_ptr[col_slot] = nz_off;
    }
    const int64_t r0 = p * mr;
    const int rows = (int)((R - r0) < mr ? (R - r0) : mr);
    const float* col = A + r0 * lda + k;
    int64_t z = nz_off;
    // column records: header, row bytes, FP32 values (unused slots zero)
    int in_rec = 0;
    int64_t r = rec_off;
    uint32_t lw0 = 0u, lw1 = 0u, lw2 = 0u;     // row bytes of the open record
    auto flush = [&](int cnt) {
      if (r < nrec_cap) {
        uint32_t* d = rec + r * 16;
        *reinterpret_cast<uint4*>(d) = make_uint4(((uint32_t)k << 8) | (uint32_t)cnt, lw0, lw1,
                                                  lw2);
        for (int t = cnt; t < kRecVals; ++t) d[4 + t] = 0u;
      }
      lw0 = lw1 = lw2 = 0u;
      ++r;
    };
    for (int i0 = 0; i0 < rows; i0 += 32) {
      float xs[32];
      load_rows32(col, lda, i0, rows, xs);
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
}

// -------------------------------------------------------------- row scale
// One wave per row: s_m = max |A[m][k]| / 448 (FP32, correctly rounded),
// 1.0 for an all-zero row; NaN entries never win the comparison.
__global__ void __launch_bounds__(256)
k_row_scale(const float* __restrict__ A, int64_t R, int64_t S, int64_t lda,
            float* __restrict__ scale) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= R) return;
  const float* a = A + row * lda;
  float amax = 0.0f;
  for (int64_t k = lane; k < S; k += 64) {
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

PackWs pack_ws_layout(int64_t R, int64_t S, int32_t mr, bool transpose) {
  PackWs L{};
  L.P = ceil_div(R, mr);
  L.NT = ceil_div(L.P * S, kPackTile);
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
    hipLaunchKernelGGL(k_pack_count, dim3((unsigned)L.NT), dim3(kPackThreads), 0, s, A, R, S,
                       lda, mr, L.P, counts, tsum);
    ROSKO_LAUNCH_CHECK("k_pack_count");
  }
  hipLaunchKernelGGL(k_pack_scan, dim3(1), dim3(1024), 0, s, tsum, toff, L.NT, totals, L.P, S,
                     out ? out->nnz_cap : INT64_MAX, out ? out->ncols_cap : INT64_MAX,
                     out ? out->nrec_cap : INT64_MAX,
                     out ? out->panel_nz_ptr : nullptr, out ? out->panel_col_ptr : nullptr,
                     out ? out->col_ptr : nullptr, out ? out->kblk_ptr : nullptr);
  ROSKO_LAUNCH_CHECK("k_pack_scan");
  return ROSKO_OK;
}

int32_t launch_pack_write(const float* A, int64_t R, int64_t S, int64_t lda, int32_t mr,
                          int32_t val_dtype, void* ws, const PackWs& L, const rosko_packed* out,
                          hipStream_t s) {
  if (L.NT == 0) return ROSKO_OK;
  char* w = static_cast<char*>(ws);
  const int32_t* counts = reinterpret_cast<const int32_t*>(w + L.counts);
  const int64_t* toff = reinterpret_cast<const int64_t*>(w + L.tile_offs);
#define ROSKO_WRITE(DT)                                                                      \
  hipLaunchKernelGGL(k_pack_write<DT>, dim3((unsigned)L.NT), dim3(kPackThreads), 0, s, A, R, \
                     S, lda, mr, L.P, counts, toff, out->nnz_cap, out->ncols_cap,            \
                     out->panel_nz_ptr, out->panel_col_ptr, out->col_ind, out->col_nnz,      \
                     out->col_ptr, out->loc, out->val, out->row_scale, out->kblk_ptr,       \
                     out->nrec_cap, out->rec)
  if (val_dtype == ROSKO_F32) ROSKO_WRITE(ROSKO_F32);
  else if (val_dtype == ROSKO_BF16) ROSKO_WRITE(ROSKO_BF16);
  else ROSKO_WRITE(ROSKO_FP8_E4M3);
#undef ROSKO_WRITE
  ROSKO_LAUNCH_CHECK("k_pack_write");
  return ROSKO_OK;
}

int32_t launch_row_scale(const float* A, int64_t R, int64_t S, int64_t lda, float* scale,
                         hipStream_t s) {
  if (R == 0) return ROSKO_OK;
  hipLaunchKernelGGL(k_row_scale, dim3((unsigned)ceil_div(R, 4)), dim3(256), 0, s, A, R, S, lda,
                     scale);
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
