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
// acc(row M0, column j) += a * b_j, with relative addressing of the addend
// and the result; REG is the VGPR holding row 0 of column j.
#define RK_FMA(REG, A, B) "v_fma_f32 v" RK_STR(REG) ", %[" A "], %[" B "], v" RK_STR(REG) "\n\t"
#define RK_OFF "s_set_gpr_idx_off"
#define RK_OUT1(T) "+{v[64:95]}"(T.t[0])
#define RK_OUT2(T) "+{v[64:95]}"(T.t[0]), "+{v[96:127]}"(T.t[1])
#define RK_OUT4(T) \
  "+{v[64:95]}"(T.t[0]), "+{v[96:127]}"(T.t[1]), "+{v[128:159]}"(T.t[2]), "+{v[160:191]}"(T.t[3])
#define RK_IN4 [b0] "v"(b[0]), [b1] "v"(b[1]), [b2] "v"(b[2]), [b3] "v"(b[3])
#define RK_IN2 [b0] "v"(b[0]), [b1] "v"(b[1])
#define RK_IN1 [b0] "v"(b[0])

// Rec<MR, V>::run applies all values (1..12) of one column record to the
// register tile in a single asm block: the record's three row words w1..w3
// (bytes already masked to MR-1) feed s_set_gpr_idx_on one byte at a time,
// and the block ends early, through its own branch, after `cnt` values.
// One asm site per record keeps the tile in its pinned registers (several
// sites in different branches made the allocator shuttle the tile around).
// Index mode is off again at the end of the block.
template <int MR, int V> struct Rec;

#define RK_ON1 "s_set_gpr_idx_on %[w1], gpr_idx(SRC2,DST)\n\t"
#define RK_ON2 "s_set_gpr_idx_on %[w2], gpr_idx(SRC2,DST)\n\t"
#define RK_ON3 "s_set_gpr_idx_on %[w3], gpr_idx(SRC2,DST)\n\t"
#define RK_SH(W) "s_lshr_b32 %[" W "], %[" W "], 8\n\t"
#define RK_IF(N) "s_cmp_lt_u32 %[cnt], " #N "\n\ts_cbranch_scc1 .Lrk_end%=\n\t"
#define RK_BODY(FL)                                                                   \
  RK_ON1 FL("a0") RK_IF(2) RK_SH("w1") RK_ON1 FL("a1") RK_IF(3) RK_SH("w1") RK_ON1  \
  FL("a2") RK_IF(4) RK_SH("w1") RK_ON1 FL("a3")                                     \
  RK_IF(5) RK_ON2 FL("a4") RK_IF(6) RK_SH("w2") RK_ON2 FL("a5") RK_IF(7) RK_SH("w2") \
  RK_ON2 FL("a6") RK_IF(8) RK_SH("w2") RK_ON2 FL("a7")                              \
  RK_IF(9) RK_ON3 FL("a8") RK_IF(10) RK_SH("w3") RK_ON3 FL("a9") RK_IF(11)           \
  RK_SH("w3") RK_ON3 FL("a10") RK_IF(12) RK_SH("w3") RK_ON3 FL("a11")               \
  ".Lrk_end%=:\n\t" RK_OFF

#define RK_REC(MR_, V_, NT_, FL, IN)                                                      \
  template <> struct Rec<MR_, V_> {                                                      \
    static __device__ __forceinline__ void run(Tile<NT_>& T, uint32_t cnt, uint32_t w1,  \
                                               uint32_t w2, uint32_t w3, const float* a, \
                                               const float* b) {                         \
      asm volatile(RK_BODY(FL)                                                           \
                   : RK_OUT##NT_(T), [w1] "+s"(w1), [w2] "+s"(w2), [w3] "+s"(w3)          \
                   : [cnt] "s"(cnt), [a0] "s"(a[0]), [a1] "s"(a[1]), [a2] "s"(a[2]),      \
                     [a3] "s"(a[3]), [a4] "s"(a[4]), [a5] "s"(a[5]), [a6] "s"(a[6]),      \
                     [a7] "s"(a[7]), [a8] "s"(a[8]), [a9] "s"(a[9]), [a10] "s"(a[10]),    \
                     [a11] "s"(a[11]), IN                                                \
                   : "m0", "scc");                                                       \
    }                                                                                    \
  };

#define RK_FL_8x4(A) RK_FMA(64, A, "b0") RK_FMA(72, A, "b1") RK_FMA(80, A, "b2") RK_FMA(88, A, "b3")
#define RK_FL_16x4(A) RK_FMA(64, A, "b0") RK_FMA(80, A, "b1") RK_FMA(96, A, "b2") RK_FMA(112, A, "b3")
#define RK_FL_32x4(A) RK_FMA(64, A, "b0") RK_FMA(96, A, "b1") RK_FMA(128, A, "b2") RK_FMA(160, A, "b3")
#define RK_FL_32x2(A) RK_FMA(64, A, "b0") RK_FMA(96, A, "b1")
#define RK_FL_64x2(A) RK_FMA(64, A, "b0") RK_FMA(128, A, "b1")
#define RK_FL_128x1(A) RK_FMA(64, A, "b0")

RK_REC(8, 4, 1, RK_FL_8x4, RK_IN4)
RK_REC(16, 4, 2, RK_FL_16x4, RK_IN4)
RK_REC(32, 4, 4, RK_FL_32x4, RK_IN4)
RK_REC(32, 2, 2, RK_FL_32x2, RK_IN2)
RK_REC(64, 2, 4, RK_FL_64x2, RK_IN2)
RK_REC(128, 1, 4, RK_FL_128x1, RK_IN1)

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

// Element j of a unit, by value (no address taken, so no private memory).
template <int TB, int V>
__device__ __forceinline__ void set_elem(typename Unit<TB, V>::T& u, int j,
                                         typename BElem<TB>::T x) {
  if constexpr (TB == ROSKO_F32) {
    if constexpr (V == 4) { if (j == 0) u.x = x; else if (j == 1) u.y = x; else if (j == 2) u.z = x; else u.w = x; }
    else if constexpr (V == 2) { if (j == 0) u.x = x; else u.y = x; }
    else u = x;
  } else {
    if constexpr (V == 4) {
      if (j == 0) u.x = (u.x & 0xFFFF0000u) | x;
      else if (j == 1) u.x = (u.x & 0x0000FFFFu) | ((uint32_t)x << 16);
      else if (j == 2) u.y = (u.y & 0xFFFF0000u) | x;
      else u.y = (u.y & 0x0000FFFFu) | ((uint32_t)x << 16);
    } else if constexpr (V == 2) {
      if (j == 0) u = (u & 0xFFFF0000u) | x;
      else u = (u & 0x0000FFFFu) | ((uint32_t)x << 16);
    } else {
      u = x;
    }
  }
}

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
    uint32_t m = 0;
    U u;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const bool in = row_ok && col0 + j < N;
      set_elem<TB, V>(u, j, base[in ? row * ldb + col0 + j : 0]);
      m |= in ? (1u << j) : 0u;
    }
    *dst = u;
    *ok = m;
  }
}

// The unit with its out-of-range elements replaced by zero.
template <int TB, int V>
__device__ __forceinline__ typename Unit<TB, V>::T masked_unit(typename Unit<TB, V>::T u,
                                                               uint32_t ok) {
  if constexpr (TB == ROSKO_F32) {
    if constexpr (V == 4) {
      u.x = (ok & 1u) ? u.x : 0.0f; u.y = (ok & 2u) ? u.y : 0.0f;
      u.z = (ok & 4u) ? u.z : 0.0f; u.w = (ok & 8u) ? u.w : 0.0f;
    } else if constexpr (V == 2) {
      u.x = (ok & 1u) ? u.x : 0.0f; u.y = (ok & 2u) ? u.y : 0.0f;
    } else {
      u = (ok & 1u) ? u : 0.0f;
    }
  } else {
    if constexpr (V == 4) {
      u.x &= ((ok & 1u) ? 0x0000FFFFu : 0u) | ((ok & 2u) ? 0xFFFF0000u : 0u);
      u.y &= ((ok & 4u) ? 0x0000FFFFu : 0u) | ((ok & 8u) ? 0xFFFF0000u : 0u);
    } else if constexpr (V == 2) {
      u &= ((ok & 1u) ? 0x0000FFFFu : 0u) | ((ok & 2u) ? 0xFFFF0000u : 0u);
    } else {
      u = (ok & 1u) ? u : (uint16_t)0;
    }
  }
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

typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));

// Byte-wise mask keeping every row byte of a record word below MR.
template <int MR> constexpr uint32_t row_mask() { return (uint32_t)(MR - 1) * 0x01010101u; }

// All values (1..12) of a column record.
template <int MR, int V, int NT>
__device__ __forceinline__ void apply_record(Tile<NT>& acc, const u32x16& R, uint32_t cnt,
                                             const float* b) {
  constexpr uint32_t m = row_mask<MR>();
  float a[12];
#pragma unroll
  for (int t = 0; t < 12; ++t) a[t] = __uint_as_float(R[4 + t]);
  Rec<MR, V>::run(acc, cnt, R[1] & m, R[2] & m, R[3] & m, a, b);
}

// One workgroup: panels [pg*G, pg*G+G) (one wavefront each), columns
// [chunk*64V, chunk*64V + 64V), K range of split s.
template <int MR, int V, int G, int TB, bool VEC>
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
  const int64_t col_base = chunk * (64 * V);
  const int64_t n0 = col_base + (int64_t)lane * V;

  // K range of this split, on ROSKO_KSTEP boundaries
  const int64_t nkb = (g.K + ROSKO_KSTEP - 1) / ROSKO_KSTEP;
  const int64_t blo = (nkb * s) / g.k_split, bhi = (nkb * (s + 1)) / g.k_split;
  const int64_t k_lo = blo * ROSKO_KSTEP;
  const int64_t k_hi = min(g.K, bhi * ROSKO_KSTEP);

  // this panel's records whose column lies in [k_lo, k_hi)
  // (32-bit record cursor relative to the panel's first record, so the walk
  // needs no 64-bit scalar arithmetic or VALU compares)
  cptr<int64_t> kblk = as_const<int64_t>(g.kblk_ptr);
  cptr<u32x16> recs = as_const<u32x16>(g.rec);
  uint32_t r = 0, r_end = 0;
  if (active && k_lo < k_hi) {
    const int64_t r0 = kblk[p * (nkb + 1)];
    recs = recs + r0;
    r = (uint32_t)(kblk[p * (nkb + 1) + blo] - r0);
    r_end = (uint32_t)(kblk[p * (nkb + 1) + bhi] - r0);
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
      const int rr = u >> 6, uc = u & 63;
      const int64_t row = kb0 + rr;
      issue_unit<TB, V, VEC>(g.B, g.ldb, row, row < k_hi, col_base + (int64_t)uc * V, g.N,
                             &regs[i], &okbits[i]);
    }
  };

  // Record walk.  The record of the current column was requested one column
  // earlier (two slots swap roles from column to column, so no register a
  // load is still filling is touched early): wait for it, read the B row its
  // column selects from LDS, request the next record, apply the values.
  // Returns false when the walk leaves this K block or the panel's range;
  // the current record then stays in X.
  float b[V];
  auto column = [&](u32x16& X, u32x16& Y, const U* buf, int32_t kb0, int32_t kb1) -> bool {
    __builtin_amdgcn_s_waitcnt(0xC07F);                 // lgkmcnt(0): X has landed
    const uint32_t hdr = X[0];
    const int32_t k = (int32_t)(hdr >> 8);
    const uint32_t cnt = hdr & 0xFFu;
    if (k >= kb1) return false;
    unit_to_float<TB, V>(buf[(k - kb0) * 64 + lane], b);
    __builtin_amdgcn_s_waitcnt(0xC07F);                 // the B row (no load pending)
    if (r + 1 < r_end) Y = recs[r + 1];                 // in flight during the FMAs
    apply_record<MR, V>(acc, X, cnt, b);
    ++r;
    return r < r_end;
  };

  u32x16 RA, RB;
  if (r < r_end) RA = recs[r];
  if (nblk > 0) fetch(k_lo);
  for (int64_t ib = 0; ib < nblk; ++ib) {
    U* buf = stage + (ib & 1) * (KB * 64);
#pragma unroll
    for (int i = 0; i < NL; ++i) buf[threadIdx.x + i * 64 * G] = masked_unit<TB, V>(regs[i], okbits[i]);
    __syncthreads();
    const int64_t kb0 = k_lo + ib * KB;
    if (ib + 1 < nblk) fetch(kb0 + KB);                // next block in flight
    const int32_t kb0_32 = (int32_t)kb0;
    const int32_t kb1 = (int32_t)min(kb0 + KB, k_hi);
    if (active && r < r_end) {
      while (true) {
        if (!column(RA, RB, buf, kb0_32, kb1)) break;
        if (!column(RB, RA, buf, kb0_32, kb1)) { RA = RB; break; }
      }
    }
  }

  if (!active) return;
  // ---- epilogue: one split -> C (row scale, beta); several -> partials
  const int rows = (int)min((int64_t)g.mr, g.M - p * g.mr);
  cptr<float> row_scale = as_const<float>(g.row_scale);
  const bool scaled = g.row_scale != nullptr;
#pragma unroll
  for (int q = 0; q < MR; ++q) {
    if (q < rows) {
      const int64_t row = p * g.mr + q;
      float v[V];
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const int idx = j * MR + q;
        v[j] = acc.t[idx >> 5][idx & 31];
      }
      if (g.k_split == 1) {
        if (scaled) {
          const float sc = row_scale[row];
#pragma unroll
          for (int j = 0; j < V; ++j) v[j] *= sc;
        }
        store_c<V>(g.C, row * g.ldc, n0, g.N, VEC, v, g.beta);
      } else {
        store_c<V>(g.ws, (s * g.M + row) * g.N, n0, g.N, g.ws_vec != 0, v, 0);
      }
    }
  }
}

template <int MR, int V, int G, int TB>
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
    hipLaunchKernelGGL((k_spmm_sparse<MR, V, G, TB, true>), dim3((unsigned)nb), dim3(64 * G), lds,
                       st, g);
  else
    hipLaunchKernelGGL((k_spmm_sparse<MR, V, G, TB, false>), dim3((unsigned)nb), dim3(64 * G),
                       lds, st, g);
  ROSKO_LAUNCH_CHECK("k_spmm_sparse");
  return ROSKO_OK;
}

template <int MR, int V, int TB>
int32_t dispatch_g(const SpmmArgs& g, int G, hipStream_t s) {
  switch (G) {
    case 1: return launch_one<MR, V, 1, TB>(g, s);
    case 2: return launch_one<MR, V, 2, TB>(g, s);
    case 4: return launch_one<MR, V, 4, TB>(g, s);
    case 8: return launch_one<MR, V, 8, TB>(g, s);
    default: break;
  }
  set_error("unsupported panels per workgroup %d (1, 2, 4 or 8)", G);
  return ROSKO_EUNSUPPORTED;
}

// Supported (tile height, columns per lane) pairs keep the register tile at
// 32, 64 or 128 VGPRs.
template <int TB>
int32_t dispatch_tile(const SpmmArgs& g, int H, int V, int G, hipStream_t s) {
  if (H == 8 && V == 4) return dispatch_g<8, 4, TB>(g, G, s);
  if (H == 16 && V == 4) return dispatch_g<16, 4, TB>(g, G, s);
  if (H == 32 && V == 4) return dispatch_g<32, 4, TB>(g, G, s);
  if (H == 32 && V == 2) return dispatch_g<32, 2, TB>(g, G, s);
  if (H == 64 && V == 2) return dispatch_g<64, 2, TB>(g, G, s);
  if (H == 128 && V == 1) return dispatch_g<128, 1, TB>(g, G, s);
  set_error("unsupported register tile: height %d with %d columns per lane", H, V);
  return ROSKO_EUNSUPPORTED;
}

}  // namespace
}  // namespace rosko
