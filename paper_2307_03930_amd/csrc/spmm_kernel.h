// Kernel template of the row-skipping SpMM; included by the per-dtype
// translation units spmm_<values>_<B>.hip.  See spmm.hip for the design.
#pragma once
#include "internal.h"

namespace rosko {
namespace {

typedef float f32x32 __attribute__((ext_vector_type(32)));

// ---------------------------------------------------------------- tile
template <int NT>
struct Tile { f32x32 t[NT]; };

#define RK_STR2(x) #x
#define RK_STR(x) RK_STR2(x)
#define RK_FMA(REG, BOP) "v_fma_f32 v" RK_STR(REG) ", %[a], %[" BOP "], v" RK_STR(REG) "\n\t"
#define RK_ON "s_set_gpr_idx_on %[r], gpr_idx(SRC2,DST)\n\t"
#define RK_OFF "s_set_gpr_idx_off"
#define RK_OUT1(T) "+{v[64:95]}"(T.t[0])
#define RK_OUT2(T) "+{v[64:95]}"(T.t[0]), "+{v[96:127]}"(T.t[1])
#define RK_OUT4(T) \
  "+{v[64:95]}"(T.t[0]), "+{v[96:127]}"(T.t[1]), "+{v[128:159]}"(T.t[2]), "+{v[160:191]}"(T.t[3])

// acc(row r, column j) += a * b[j] for j < V; r already masked to MR-1.
template <int MR, int V> struct Fma;

#define RK_DEF_FMA4(MR_, NT_, R0, R1, R2, R3)                                            \
  template <> struct Fma<MR_, 4> {                                                      \
    static __device__ __forceinline__ void run(Tile<NT_>& T, uint32_t r, float a,       \
                                               const float* b) {                       \
      asm volatile(RK_ON RK_FMA(R0, "b0") RK_FMA(R1, "b1") RK_FMA(R2, "b2")             \
                       RK_FMA(R3, "b3") RK_OFF                                          \
                   : RK_OUT##NT_(T)                                                     \
                   : [r] "s"(r), [a] "s"(a), [b0] "v"(b[0]), [b1] "v"(b[1]),            \
                     [b2] "v"(b[2]), [b3] "v"(b[3])                                     \
                   : "m0");                                                             \
    }                                                                                   \
  };
#define RK_DEF_FMA2(MR_, NT_, R0, R1)                                                    \
  template <> struct Fma<MR_, 2> {                                                      \
    static __device__ __forceinline__ void run(Tile<NT_>& T, uint32_t r, float a,       \
                                               const float* b) {                       \
      asm volatile(RK_ON RK_FMA(R0, "b0") RK_FMA(R1, "b1") RK_OFF                       \
                   : RK_OUT##NT_(T)                                                     \
                   : [r] "s"(r), [a] "s"(a), [b0] "v"(b[0]), [b1] "v"(b[1])             \
                   : "m0");                                                             \
    }                                                                                   \
  };
#define RK_DEF_FMA1(MR_, NT_)                                                            \
  template <> struct Fma<MR_, 1> {                                                      \
    static __device__ __forceinline__ void run(Tile<NT_>& T, uint32_t r, float a,       \
                                               const float* b) {                       \
      asm volatile(RK_ON RK_FMA(64, "b0") RK_OFF                                         \
                   : RK_OUT##NT_(T)                                                     \
                   : [r] "s"(r), [a] "s"(a), [b0] "v"(b[0])                             \
                   : "m0");                                                             \
    }                                                                                   \
  };

RK_DEF_FMA4(8, 1, 64, 72, 80, 88)
RK_DEF_FMA4(16, 2, 64, 80, 96, 112)
RK_DEF_FMA4(32, 4, 64, 96, 128, 160)
RK_DEF_FMA2(16, 1, 64, 80)
RK_DEF_FMA2(32, 2, 64, 96)
RK_DEF_FMA2(64, 4, 64, 128)
RK_DEF_FMA1(32, 1)
RK_DEF_FMA1(64, 2)
RK_DEF_FMA1(128, 4)

template <int MR, int V> constexpr int tile_nt() { return (MR * V) / 32; }

// The packed arrays are read-only for the whole kernel, so they are read
// through the constant address space: wave-uniform indices then become
// scalar loads into SGPRs instead of vector loads plus v_readfirstlane.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const void* p) {
  return (cptr<T>)(p);
}

// ----------------------------------------------------------- value decode
// Packed value z as FP32 (FP8: the code's value; the row scale is applied
// to the finished sums).  All arguments are wave-uniform, so these become
// scalar loads and scalar bit operations.
template <int TA> __device__ __forceinline__ float load_a(const void* val, int64_t z);
template <> __device__ __forceinline__ float load_a<ROSKO_F32>(const void* val, int64_t z) {
  return as_const<float>(val)[z];
}
template <> __device__ __forceinline__ float load_a<ROSKO_BF16>(const void* val, int64_t z) {
  const uint32_t w = as_const<uint32_t>(val)[z >> 1];
  return __uint_as_float((z & 1) ? (w & 0xFFFF0000u) : (w << 16));
}
template <> __device__ __forceinline__ float load_a<ROSKO_FP8_E4M3>(const void* val, int64_t z) {
  const uint32_t w = as_const<uint32_t>(val)[z >> 2];
  const uint32_t c = (w >> (8 * (uint32_t)(z & 3))) & 0xFFu;
  const uint32_t e = (c >> 3) & 15u, m = c & 7u, s = (c & 0x80u) << 24;
  uint32_t bits;
  if (e == 0) bits = __float_as_uint((float)m * 0.001953125f);        // m * 2^-9
  else if (e == 15 && m == 7) bits = 0x7FC00000u;                      // NaN
  else bits = ((e + 120u) << 23) | (m << 20);                          // (1+m/8) 2^(e-7)
  return __uint_as_float(bits | s);
}

// Rows within the panel (one byte each) of packed values z .. z+7, masked
// to MR-1: two dword pairs cover the 8 bytes wherever z falls in a dword.
template <int MR>
__device__ __forceinline__ void load_loc8(const uint8_t* loc, int64_t z, uint32_t* r) {
  cptr<uint32_t> lw = as_const<uint32_t>(loc);
  const int64_t q = z >> 2;
  const uint32_t sh = 8u * (uint32_t)(z & 3);
  const uint64_t lo = (uint64_t)lw[q] | ((uint64_t)lw[q + 1] << 32);
  const uint64_t hi = (uint64_t)lw[q + 1] | ((uint64_t)lw[q + 2] << 32);
  const uint32_t L0 = (uint32_t)(lo >> sh), L1 = (uint32_t)(hi >> sh);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    r[t] = (L0 >> (8 * t)) & (uint32_t)(MR - 1);
    r[t + 4] = (L1 >> (8 * t)) & (uint32_t)(MR - 1);
  }
}

// ----------------------------------------------------------- B / C access
// The same 8 row bytes, split in two steps so the scalar loads can be in
// flight while other work runs: load_locw fetches the dwords that hold bytes
// z .. z+7, loc_from_words extracts them (after the loads have landed).
struct LocWords { uint32_t w0, w1, w2, sh; };
__device__ __forceinline__ LocWords load_locw(const uint8_t* loc, int64_t z) {
  cptr<uint32_t> lw = as_const<uint32_t>(loc);
  const int64_t q = z >> 2;
  return LocWords{lw[q], lw[q + 1], lw[q + 2], 8u * (uint32_t)(z & 3)};
}
template <int MR>
__device__ __forceinline__ void loc_from_words(const LocWords& w, uint32_t* r) {
  const uint64_t lo = (uint64_t)w.w0 | ((uint64_t)w.w1 << 32);
  const uint64_t hi = (uint64_t)w.w1 | ((uint64_t)w.w2 << 32);
  const uint32_t L0 = (uint32_t)(lo >> w.sh), L1 = (uint32_t)(hi >> w.sh);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    r[t] = (L0 >> (8 * t)) & (uint32_t)(MR - 1);
    r[t + 4] = (L1 >> (8 * t)) & (uint32_t)(MR - 1);
  }
}

// ------------------------------------------------------------ B staging
// B rows of the current K block are staged in LDS as [row][unit], one unit
// = the V consecutive elements a lane multiplies (64 units per row), in B's
// own element type.
template <int TB> struct BElem;
template <> struct BElem<ROSKO_F32> { using T = float; };
template <> struct BElem<ROSKO_BF16> { using T = uint16_t; };

template <int TB, int V> struct Unit;    // raw storage of one unit
template <> struct Unit<ROSKO_F32, 4> { using T = float4; };
template <> struct Unit<ROSKO_F32, 2> { using T = float2; };
template <> struct Unit<ROSKO_F32, 1> { using T = float; };
template <> struct Unit<ROSKO_BF16, 4> { using T = uint2; };
template <> struct Unit<ROSKO_BF16, 2> { using T = uint32_t; };
template <> struct Unit<ROSKO_BF16, 1> { using T = uint16_t; };

// Issue the load of unit `u` of B row `row` (columns col0 .. col0+V-1)
// without consuming it: out-of-range addresses are clamped to B's first
// element, and `ok` (one bit per element) records which elements are real.
// The zero fill is applied only when the unit is written to LDS, after the
// current block's compute, so the loads of a block overlap each other and
// that compute instead of each waiting for the previous one.
template <int TB, int V, bool VEC>
__device__ __forceinline__ void issue_unit(const void* __restrict__ B, int64_t ldb, int64_t row,
                                           bool row_ok, int64_t col0, int64_t N,
                                           typename Unit<TB, V>::T* dst, uint32_t* ok) {
  using E = typename BElem<TB>::T;
  using U = typename Unit<TB, V>::T;
  const E* base = reinterpret_cast<const E*>(B);
  if constexpr (VEC) {
    const bool in = row_ok && col0 < N;
    *dst = *reinterpret_cast<const U*>(base + (in ? row * ldb + col0 : 0));
    *ok = in ? ((1u << V) - 1u) : 0u;
  } else {
    E* e = reinterpret_cast<E*>(dst);
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const bool in = row_ok && col0 + j < N;
      e[j] = base[in ? row * ldb + col0 + j : 0];
      m |= in ? (1u << j) : 0u;
    }
    *ok = m;
  }
}

// The unit with its out-of-range elements replaced by zero.
template <int TB, int V>
__device__ __forceinline__ typename Unit<TB, V>::T masked_unit(typename Unit<TB, V>::T u,
                                                               uint32_t ok) {
  using E = typename BElem<TB>::T;
  E* e = reinterpret_cast<E*>(&u);
#pragma unroll
  for (int j = 0; j < V; ++j) e[j] = ((ok >> j) & 1u) ? e[j] : E(0);
  return u;
}

template <int TB, int V>
__device__ __forceinline__ void unit_to_float(typename Unit<TB, V>::T u, float* b) {
  if constexpr (TB == ROSKO_F32) {
    const float* f = reinterpret_cast<const float*>(&u);
#pragma unroll
    for (int j = 0; j < V; ++j) b[j] = f[j];
  } else {
    const uint16_t* h = reinterpret_cast<const uint16_t*>(&u);
#pragma unroll
    for (int j = 0; j < V; ++j) b[j] = __uint_as_float((uint32_t)h[j] << 16);
  }
}

template <int V>
__device__ __forceinline__ void store_c(float* __restrict__ C, int64_t off, int64_t n0, int64_t N,
                                        bool VEC, const float* v, int beta) {
  float* p = C + off + n0;
  if (VEC) {
    if (n0 >= N) return;
    if (V == 4) {
      float4 x = make_float4(v[0], v[1], v[2], v[3]);
      if (beta) { float4 o = *reinterpret_cast<const float4*>(p); x.x += o.x; x.y += o.y; x.z += o.z; x.w += o.w; }
      *reinterpret_cast<float4*>(p) = x;
    } else if (V == 2) {
      float2 x = make_float2(v[0], v[1]);
      if (beta) { float2 o = *reinterpret_cast<const float2*>(p); x.x += o.x; x.y += o.y; }
      *reinterpret_cast<float2*>(p) = x;
    } else {
      p[0] = beta ? p[0] + v[0] : v[0];
    }
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j)
      if (n0 + j < N) p[j] = beta ? p[j] + v[j] : v[j];
  }
}

// Blocks are dealt to the 8 XCDs round-robin; remap so that consecutive
// tile ids (which share B rows) run on the same XCD and hit its L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, rem = nb & 7, x = b & 7, pos = b >> 3;
  const int64_t start = (x < rem) ? x * (q + 1) : rem * (q + 1) + (x - rem) * q;
  return start + pos;
}

// Rows per staged K block: at most 8 units per thread, at most 64 rows, and
// a divisor of ROSKO_KSTEP so K ranges never split a block.
template <int V, int G> constexpr int stage_rows() {
  constexpr int r = 8 * G;           // units per row = 64; threads = 64*G
  return r > 64 ? 64 : r;
}

constexpr int kChunk = 8;   // values fetched per scalar batch

// Per-column state of the pipelined column walk: the column's metadata and
// its first batch of values and row bytes.
struct ColState {
  int32_t k, n;
  float a[kChunk];
  LocWords w;
};

// One workgroup: panels [pg*G, pg*G+G) (one wavefront each), columns
// [chunk*64V, chunk*64V + 64V), K range of split s.
template <int MR, int V, int G, int TA, int TB, bool VEC>
__global__ void __launch_bounds__(64 * G)
k_spmm_sparse(SpmmArgs g) {
  constexpr int NT = tile_nt<MR, V>();
  constexpr int KB = stage_rows<V, G>();
  constexpr int NL = KB * 64 / (64 * G);               // units per thread per block
  using U = typename Unit<TB, V>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  U* stage = reinterpret_cast<U*>(smem);                // [2][KB][64]

  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t n_pg = (g.n_panels + G - 1) / G;
  const int64_t pg = tile % n_pg;
  const int64_t cs = tile / n_pg;
  const int64_t chunk = cs % g.n_chunks;
  const int64_t s = cs / g.n_chunks;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t p = pg * G + wid;
  const bool active = p < g.n_panels;
  constexpr bool vec = VEC;
  const int64_t col_base = chunk * (64 * V);
  const int64_t n0 = col_base + (int64_t)lane * V;

  // K range of this split, on ROSKO_KSTEP boundaries
  const int64_t nkb = (g.K + ROSKO_KSTEP - 1) / ROSKO_KSTEP;
  const int64_t blo = (nkb * s) / g.k_split, bhi = (nkb * (s + 1)) / g.k_split;
  const int64_t k_lo = blo * ROSKO_KSTEP;
  const int64_t k_hi = min(g.K, bhi * ROSKO_KSTEP);

  cptr<int64_t> panel_col_ptr = as_const<int64_t>(g.panel_col_ptr);
  cptr<int32_t> col_ind = as_const<int32_t>(g.col_ind);
  cptr<int32_t> col_nnz = as_const<int32_t>(g.col_nnz);
  cptr<int64_t> col_ptr = as_const<int64_t>(g.col_ptr);
  cptr<int64_t> kblk = as_const<int64_t>(g.kblk_ptr);

  // Column walk, carried across K blocks, software pipelined so that each
  // column waits once, for loads issued one column earlier: the metadata
  // (k, count) of the column after next, the first batch of values and row
  // bytes of the next column, and the B row of the next column (read from
  // LDS at the end of the current one).  Two state slots swap roles from
  // column to column (the loop body is unrolled twice), so no register that
  // a load is still filling is touched before that wait.
  int64_t c = 0, c_end = 0, z = 0;
  ColState SA, SB;
  SA.k = SB.k = INT32_MAX;
  SA.n = SB.n = 0;
  if (active && k_lo < k_hi) {
    c = kblk[p * nkb + blo];
    c_end = (bhi < nkb) ? kblk[p * nkb + bhi] : panel_col_ptr[p + 1];
    z = col_ptr[c];
    if (c < c_end) { SA.k = col_ind[c]; SA.n = col_nnz[c]; }
    if (c + 1 < c_end) { SB.k = col_ind[c + 1]; SB.n = col_nnz[c + 1]; }
#pragma unroll
    for (int t = 0; t < kChunk; ++t) SA.a[t] = load_a<TA>(g.val, z + t);
    SA.w = load_locw(g.loc, z);
  }

  Tile<NT> acc;
#pragma unroll
  for (int q = 0; q < NT; ++q) acc.t[q] = (f32x32)(0.0f);

  const int64_t nblk = (k_hi > k_lo) ? (k_hi - k_lo + KB - 1) / KB : 0;
  U regs[NL];
  uint32_t okbits[NL];
  auto fetch = [&](int64_t kb0) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int u = threadIdx.x + i * 64 * G;          // unit index in the block
      const int r = u >> 6, uc = u & 63;
      const int64_t row = kb0 + r;
      issue_unit<TB, V, VEC>(g.B, g.ldb, row, row < k_hi, col_base + (int64_t)uc * V, g.N,
                             &regs[i], &okbits[i]);
    }
  };

  float b[V];
  // One column: X holds the current column, Y.k/Y.n the next column's
  // metadata.  Returns false when the next column is past this K block or
  // past the panel's range (its state is then in Y).
  auto column = [&](ColState& X, ColState& Y, const U* buf, int64_t kb0, int64_t kb1) -> bool {
    // Everything this column needs (its B row, metadata, first values) was
    // requested one column ago: wait here, so the prefetch issued next stays
    // in flight during the FMAs (scalar loads retire out of order, so any
    // later wait would be a full lgkmcnt(0) draining the prefetch too).
    // 0xC07F: lgkmcnt 0, vmcnt and expcnt unrestricted.
    __builtin_amdgcn_s_waitcnt(0xC07F);
    const int32_t ncur = X.n;
    uint32_t rv[kChunk];
    loc_from_words<MR>(X.w, rv);
    // prefetch: first values of column c+1, metadata of column c+2
#pragma unroll
    for (int t = 0; t < kChunk; ++t) Y.a[t] = load_a<TA>(g.val, z + ncur + t);
    Y.w = load_locw(g.loc, z + ncur);
    if (c + 2 < c_end) { X.k = col_ind[c + 2]; X.n = col_nnz[c + 2]; }
    else { X.k = INT32_MAX; X.n = 0; }
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      if (t < ncur) {
        const uint32_t r = __builtin_amdgcn_readfirstlane(rv[t]);
        const float a = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(X.a[t])));
        Fma<MR, V>::run(acc, r, a, b);
      }
    }
    for (int base = kChunk; base < ncur; base += kChunk) {
      float ax[kChunk];
      uint32_t rx[kChunk];
#pragma unroll
      for (int t = 0; t < kChunk; ++t) ax[t] = load_a<TA>(g.val, z + base + t);
      loc_from_words<MR>(load_locw(g.loc, z + base), rx);
      const int rem = ncur - base;
#pragma unroll
      for (int t = 0; t < kChunk; ++t) {
        if (t < rem) {
          const uint32_t r = __builtin_amdgcn_readfirstlane(rx[t]);
          const float a = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(ax[t])));
          Fma<MR, V>::run(acc, r, a, b);
        }
      }
    }
    z += ncur;
    ++c;
    if (c >= c_end || Y.k >= kb1) return false;
    unit_to_float<TB, V>(buf[(Y.k - kb0) * 64 + lane], b);
    return true;
  };

  if (nblk > 0) fetch(k_lo);
  for (int64_t ib = 0; ib < nblk; ++ib) {
    U* buf = stage + (ib & 1) * (KB * 64);
#pragma unroll
    for (int i = 0; i < NL; ++i) buf[threadIdx.x + i * 64 * G] = masked_unit<TB, V>(regs[i], okbits[i]);
    __syncthreads();
    const int64_t kb0 = k_lo + ib * KB;
    if (ib + 1 < nblk) fetch(kb0 + KB);                // next block in flight
    const int64_t kb1 = min(kb0 + KB, k_hi);
    if (active && c < c_end && SA.k < kb1) {
      unit_to_float<TB, V>(buf[(SA.k - kb0) * 64 + lane], b);
      while (true) {
        // after a stop in the first half the current column lives in SB and
        // the next column's metadata in SA: swap so the walk resumes from SA
        if (!column(SA, SB, buf, kb0, kb1)) { ColState t = SA; SA = SB; SB = t; break; }
        if (!column(SB, SA, buf, kb0, kb1)) break;
      }
    }
  }

  if (!active) return;
  // ---- epilogue: one split -> C (row scale, beta); several -> partials
  const int rows = (int)min((int64_t)g.mr, g.M - p * g.mr);
  cptr<float> row_scale = as_const<float>(g.row_scale);
#pragma unroll
  for (int r = 0; r < MR; ++r) {
    if (r < rows) {
      const int64_t row = p * g.mr + r;
      float v[V];
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const int idx = j * MR + r;
        v[j] = acc.t[idx >> 5][idx & 31];
      }
      if (g.k_split == 1) {
        if (TA == ROSKO_FP8_E4M3) {
          const float sc = row_scale[row];
#pragma unroll
          for (int j = 0; j < V; ++j) v[j] *= sc;
        }
        store_c<V>(g.C, row * g.ldc, n0, g.N, vec, v, g.beta);
      } else {
        store_c<V>(g.ws, (s * g.M + row) * g.N, n0, g.N, g.ws_vec != 0, v, 0);
      }
    }
  }
}

template <int MR, int V, int G, int TA, int TB>
int32_t launch_one(const SpmmArgs& g, hipStream_t st) {
  const int64_t n_pg = (g.n_panels + G - 1) / G;
  const int64_t nb = n_pg * g.n_chunks * g.k_split;
  if (nb == 0) return ROSKO_OK;
  if (nb > INT32_MAX) {
    set_error("spmm grid too large (%lld workgroups)", (long long)nb);
    return ROSKO_EUNSUPPORTED;
  }
  constexpr int KB = stage_rows<V, G>();
  const size_t lds = 2 * (size_t)KB * 64 * sizeof(typename Unit<TB, V>::T);
  if (g.vec)
    hipLaunchKernelGGL((k_spmm_sparse<MR, V, G, TA, TB, true>), dim3((unsigned)nb), dim3(64 * G),
                       lds, st, g);
  else
    hipLaunchKernelGGL((k_spmm_sparse<MR, V, G, TA, TB, false>), dim3((unsigned)nb),
                       dim3(64 * G), lds, st, g);
  ROSKO_LAUNCH_CHECK("k_spmm_sparse");
  return ROSKO_OK;
}

template <int MR, int V, int TA, int TB>
int32_t dispatch_g(const SpmmArgs& g, int G, hipStream_t s) {
  switch (G) {
    case 1: return launch_one<MR, V, 1, TA, TB>(g, s);
    case 2: return launch_one<MR, V, 2, TA, TB>(g, s);
    case 4: return launch_one<MR, V, 4, TA, TB>(g, s);
    case 8: return launch_one<MR, V, 8, TA, TB>(g, s);
    default: break;
  }
  set_error("unsupported panels per workgroup %d (1, 2, 4 or 8)", G);
  return ROSKO_EUNSUPPORTED;
}

// Supported (tile height, columns per lane) pairs keep the register tile at
// 32, 64 or 128 VGPRs.
template <int TA, int TB>
int32_t dispatch_tile(const SpmmArgs& g, int H, int V, int G, hipStream_t s) {
  if (H == 8 && V == 4) return dispatch_g<8, 4, TA, TB>(g, G, s);
  if (H == 16 && V == 4) return dispatch_g<16, 4, TA, TB>(g, G, s);
  if (H == 32 && V == 4) return dispatch_g<32, 4, TA, TB>(g, G, s);
  if (H == 32 && V == 2) return dispatch_g<32, 2, TA, TB>(g, G, s);
  if (H == 64 && V == 2) return dispatch_g<64, 2, TA, TB>(g, G, s);
  if (H == 128 && V == 1) return dispatch_g<128, 1, TA, TB>(g, G, s);
  set_error("unsupported register tile: height %d with %d columns per lane", H, V);
  return ROSKO_EUNSUPPORTED;
}

}  // namespace
}  // namespace rosko
