// Kernel template of the row-skipping SpMM (Alg. 2); included by the
// per-B-dtype translation units spmm_b<dtype>.hip.  See spmm.hip for the
// host side and the design notes.
#pragma once
#include "internal.h"

namespace rosko {
namespace {

typedef float f32x32 __attribute__((ext_vector_type(32)));

// ---------------------------------------------------------------- tile
// The C tile of one wavefront: MR rows x V columns per lane, column j of row
// r in VGPR base + j*MR + r, pinned by asm constraints so that a row index
// can select the register at run time.  In the record loop (spmm_loop.inc)
// the base is the first multiple of 8 after the loop's record and B
// registers (v24 for the 128-register tiles at depth 4: 158 VGPRs in all);
// the element-load path below pins it at v40 (128-register tiles) or v32.
template <int NT>
struct Tile { f32x32 t[NT]; };

#define RK_STR2(x) #x
#define RK_STR(x) RK_STR2(x)
// acc(row, column j) += value * b_j.  The value is lane SLOT of each 16-lane
// row of the record register, broadcast by DPP; the accumulator register is
// relative (index mode on SRC2 and DST); REG is the VGPR of row 0 of column j.
#define RK_FMA(REG, SLOT, B)                                                         \
  "v_fmac_f32_dpp v" RK_STR(REG) ", %[vr], %[" B "] row_newbcast:" RK_STR(SLOT)      \
  " row_mask:0xf bank_mask:0xf\n\t"
#define RK_OUT1(T) "+{v[32:63]}"(T.t[0])
#define RK_OUT2(T) "+{v[32:63]}"(T.t[0]), "+{v[64:95]}"(T.t[1])
#define RK_OUT4(T) \
  "+{v[40:71]}"(T.t[0]), "+{v[72:103]}"(T.t[1]), "+{v[104:135]}"(T.t[2]), "+{v[136:167]}"(T.t[3])
#define RK_IN4 [b0] "v"(b[0]), [b1] "v"(b[1]), [b2] "v"(b[2]), [b3] "v"(b[3])
#define RK_IN2 [b0] "v"(b[0]), [b1] "v"(b[1])
#define RK_IN1 [b0] "v"(b[0])

// Rec<MR, V>::run applies the 1..12 values of one column record to the
// register tile in a single asm block.  The record sits in one VGPR, lane l
// holding dword (l & 15): dword 0 the header, dwords 1..3 the row bytes,
// dwords 4..15 the values.  A row word is read into an SGPR (v_readlane,
// index mode off), masked to MR-1 per byte, and fed to s_set_gpr_idx_on one
// byte at a time; the block leaves through its own branch after `cnt`
// values.  The leading s_nop gives the DPP reads the two wait states they
// need after any VALU write of their operands.
template <int MR, int V> struct Rec;

#define RK_ON "s_set_gpr_idx_on %[w], gpr_idx(SRC2,DST)\n\t"
#define RK_SH "s_lshr_b32 %[w], %[w], 8\n\t"
#define RK_IF(N) "s_cmp_lt_u32 %[cnt], " #N "\n\ts_cbranch_scc1 .Lrk_end%=\n\t"
#define RK_WORD(LANE, MASK)                                          \
  "s_set_gpr_idx_off\n\tv_readlane_b32 %[w], %[vr], " #LANE "\n\t" \
  "s_and_b32 %[w], %[w], " MASK "\n\t"
#define RK_BODY(FL, MASK)                                                                \
  "s_nop 1\n\tv_readlane_b32 %[w], %[vr], 1\n\ts_and_b32 %[w], %[w], " MASK "\n\t"      \
  RK_ON FL(4) RK_IF(2) RK_SH RK_ON FL(5) RK_IF(3) RK_SH RK_ON FL(6) RK_IF(4) RK_SH RK_ON \
  FL(7) RK_IF(5) RK_WORD(2, MASK) RK_ON FL(8) RK_IF(6) RK_SH RK_ON FL(9) RK_IF(7) RK_SH  \
  RK_ON FL(10) RK_IF(8) RK_SH RK_ON FL(11) RK_IF(9) RK_WORD(3, MASK) RK_ON FL(12)        \
  RK_IF(10) RK_SH RK_ON FL(13) RK_IF(11) RK_SH RK_ON FL(14) RK_IF(12) RK_SH RK_ON FL(15) \
  ".Lrk_end%=:\n\ts_set_gpr_idx_off"

#define RK_REC(MR_, V_, NT_, FL, IN, MASK)                                                \
  template <> struct Rec<MR_, V_> {                                                      \
    static __device__ __forceinline__ void run(Tile<NT_>& T, uint32_t vr, uint32_t cnt,  \
                                               const float* b) {                         \
      uint32_t w;                                                                        \
      asm volatile(RK_BODY(FL, MASK)                                                     \
                   : RK_OUT##NT_(T), [w] "=&s"(w)                                        \
                   : [vr] "v"(vr), [cnt] "s"(cnt), IN                                    \
                   : "m0", "scc");                                                       \
    }                                                                                    \
  };

#define RK_FL_8x4(S) RK_FMA(32, S, "b0") RK_FMA(40, S, "b1") RK_FMA(48, S, "b2") RK_FMA(56, S, "b3")
#define RK_FL_16x4(S) RK_FMA(32, S, "b0") RK_FMA(48, S, "b1") RK_FMA(64, S, "b2") RK_FMA(80, S, "b3")
#define RK_FL_32x2(S) RK_FMA(32, S, "b0") RK_FMA(64, S, "b1")
#define RK_FL_32x4(S) RK_FMA(40, S, "b0") RK_FMA(72, S, "b1") RK_FMA(104, S, "b2") RK_FMA(136, S, "b3")
#define RK_FL_64x2(S) RK_FMA(40, S, "b0") RK_FMA(104, S, "b1")
#define RK_FL_128x1(S) RK_FMA(40, S, "b0")

RK_REC(8, 4, 1, RK_FL_8x4, RK_IN4, "0x07070707")
RK_REC(16, 4, 2, RK_FL_16x4, RK_IN4, "0x0f0f0f0f")
RK_REC(32, 2, 2, RK_FL_32x2, RK_IN2, "0x1f1f1f1f")
RK_REC(32, 4, 4, RK_FL_32x4, RK_IN4, "0x1f1f1f1f")
RK_REC(64, 2, 4, RK_FL_64x2, RK_IN2, "0x3f3f3f3f")
RK_REC(128, 1, 4, RK_FL_128x1, RK_IN1, "0x7f7f7f7f")

template <int MR, int V> constexpr int tile_nt() { return (MR * V) / 32; }

template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const void* p) {
  return (cptr<T>)(p);
}

// ------------------------------------------------------------ B access
// One lane reads V consecutive elements of a B row ("unit"), in B's own
// element type, and widens them to FP32 when the record is applied.
template <int TB, int V> struct Unit;
template <> struct Unit<ROSKO_F32, 4> { using T = float4; };
template <> struct Unit<ROSKO_F32, 2> { using T = float2; };
template <> struct Unit<ROSKO_F32, 1> { using T = float; };
template <> struct Unit<ROSKO_BF16, 4> { using T = uint2; };
template <> struct Unit<ROSKO_BF16, 2> { using T = uint32_t; };
template <> struct Unit<ROSKO_BF16, 1> { using T = uint16_t; };

template <int TB> struct BElem;
template <> struct BElem<ROSKO_F32> { using T = float; };
template <> struct BElem<ROSKO_BF16> { using T = uint16_t; };

// Unit of row k at this lane's columns.  VEC: one aligned vector load at a
// column clamped into [0, N-V]; otherwise V element loads, each clamped into
// [0, N-1].  Clamped lanes read valid memory; their C columns are never stored.
template <int TB, int V, bool VEC>
__device__ __forceinline__ typename Unit<TB, V>::T load_unit(const void* __restrict__ B,
                                                             int64_t ldb, uint32_t k,
                                                             int64_t col, int64_t N) {
  using E = typename BElem<TB>::T;
  using U = typename Unit<TB, V>::T;
  const E* row = reinterpret_cast<const E*>(B) + (int64_t)k * ldb;
  if constexpr (VEC) {
    const int64_t c = col < N - V ? col : N - V;
    return *reinterpret_cast<const U*>(row + c);
  } else {
    E e[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int64_t c = col + j < N ? col + j : N - 1;
      e[j] = row[c];
    }
    U u;
    if constexpr (TB == ROSKO_F32) {
      if constexpr (V == 4) u = make_float4(e[0], e[1], e[2], e[3]);
      else if constexpr (V == 2) u = make_float2(e[0], e[1]);
      else u = e[0];
    } else {
      if constexpr (V == 4)
        u = make_uint2((uint32_t)e[0] | ((uint32_t)e[1] << 16),
                       (uint32_t)e[2] | ((uint32_t)e[3] << 16));
      else if constexpr (V == 2) u = (uint32_t)e[0] | ((uint32_t)e[1] << 16);
      else u = e[0];
    }
    return u;
  }
}

template <int TB, int V>
__device__ __forceinline__ void unit_to_float(typename Unit<TB, V>::T u, float* b) {
  if constexpr (TB == ROSKO_F32) {
    if constexpr (V == 4) { b[0] = u.x; b[1] = u.y; b[2] = u.z; b[3] = u.w; }
    else if constexpr (V == 2) { b[0] = u.x; b[1] = u.y; }
    else b[0] = u;
  } else {
    if constexpr (V == 4) {
      b[0] = __uint_as_float(u.x << 16); b[1] = __uint_as_float(u.x & 0xFFFF0000u);
      b[2] = __uint_as_float(u.y << 16); b[3] = __uint_as_float(u.y & 0xFFFF0000u);
    } else if constexpr (V == 2) {
      b[0] = __uint_as_float(u << 16); b[1] = __uint_as_float(u & 0xFFFF0000u);
    } else {
      b[0] = __uint_as_float((uint32_t)u << 16);
    }
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

// Workgroups are dealt to the 8 XCDs round-robin; remap so that consecutive
// ids (the panels of one column chunk and K part, which read the same B
// rows) run on the same XCD and share its L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, rem = nb & 7, x = b & 7, pos = b >> 3;
  const int64_t start = (x < rem) ? x * (q + 1) : rem * (q + 1) + (x - rem) * q;
  return start + pos;
}

// Tile element (row q, column j) of a lane, for the epilogue (constant
// indices after unrolling).
template <int MR, int NT>
__device__ __forceinline__ float tile_at(const Tile<NT>& acc, int q, int j) {
  const int idx = j * MR + q;
  return acc.t[idx >> 5][idx & 31];
}
// LDS image of one tile: row q, lane l, column j at (q*64 + l)*V + j, so a
// wavefront moves a row as 64 consecutive V-vectors.
template <int MR, int V, int NT>
__device__ __forceinline__ void tile_to_lds(const Tile<NT>& acc, float* buf, int lane) {
#pragma unroll
  for (int q = 0; q < MR; ++q)
#pragma unroll
    for (int j = 0; j < V; ++j) buf[(q * 64 + lane) * V + j] = tile_at<MR>(acc, q, j);
}
// buf += tile, element by element (each lane touches only its own slots).
template <int MR, int V, int NT>
__device__ __forceinline__ void tile_accumulate_lds(const Tile<NT>& acc, float* buf, int lane) {
#pragma unroll
  for (int q = 0; q < MR; ++q)
#pragma unroll
    for (int j = 0; j < V; ++j) buf[(q * 64 + lane) * V + j] += tile_at<MR>(acc, q, j);
}

// B rows in flight per wavefront in the element-load path (the vector
// path's depth is a template parameter: 4 or 8).
constexpr int kDepth = 4;

#include "spmm_loop.inc"

// One workgroup: H wavefronts on one (panel, column chunk) tile; split s of
// k_split.  The panel's records are cut into k_split*H equal runs (by record
// count, so the waves get the same work); wavefront w takes run s*H + w,
// keeps its partial tile in VGPRs, and the H tiles are added through LDS in a
// fixed order.  Each wavefront streams its records and the B rows they name
// with vector loads, kDepth records ahead of the FMAs, so no step waits on a
// single load round trip.
template <int MR, int V, int H, int TB, bool VEC, int DV>
__global__ void __launch_bounds__(64 * H)
k_spmm_rows(SpmmArgs g) {
  constexpr int NT = tile_nt<MR, V>();
  constexpr int D = kDepth;
  using U = typename Unit<TB, V>::T;
  extern __shared__ __align__(16) float red[];

  const int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t p = bid % g.n_panels;
  const int64_t rest = bid / g.n_panels;
  const int64_t s = rest % g.k_split;
  const int64_t chunk = rest / g.k_split;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t n0 = chunk * (64 * V) + (int64_t)lane * V;

  // this wavefront's run of the panel's records
  const int64_t nkb = (g.K + ROSKO_KSTEP - 1) / ROSKO_KSTEP;
  cptr<int64_t> kblk = as_const<int64_t>(g.kblk_ptr);
  // the panel's record range, clamped into [0, rec_bound] so that no content of
  // the packed arrays can move a record address outside the record array
  const int64_t r0 = min(max(kblk[p * (nkb + 1)], (int64_t)0), g.rec_bound);
  const int64_t r1 = min(max(kblk[p * (nkb + 1) + nkb], r0), g.rec_bound);
  const int64_t parts = (int64_t)g.k_split * H, part = s * H + w;
  const int64_t a = r0 + (r1 - r0) * part / parts;
  const int64_t e = r0 + (r1 - r0) * (part + 1) / parts;
  const int32_t n = (int32_t)(e - a);
  const uint32_t* rp = g.rec + a * 16 + (lane & 15);

  Tile<NT> acc;
#pragma unroll
  for (int q = 0; q < NT; ++q) acc.t[q] = (f32x32)(0.0f);

  if (n > 0) {
    if constexpr (VEC) {
      // the record loop in one asm block (spmm_loop.inc); buffer loads with
      // 32-bit offsets from this run's first record and from B.  Each buffer
      // is sized exactly (the records from this run's first to the array's
      // end; K rows of ldb elements), so the hardware returns zero for any
      // load outside it instead of touching other memory
      constexpr uint32_t esz = TB == ROSKO_F32 ? 4 : 2;
      const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(g.rec + a * 16), 0, (int)(uint32_t)((g.rec_bound - a) * 64), 0x00020000);
      const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
          (void*)g.B, 0, (int)(uint32_t)(g.K * g.ldb * esz), 0x00020000);
      const int64_t cl = n0 < g.N - V ? n0 : g.N - V;
      RkLoop<MR, V, TB, DV>::run(acc, (uint32_t)n, rr, rb, (uint32_t)(g.ldb * esz),
                             (uint32_t)(g.K - 1), (uint32_t)(lane & 15) * 4u,
                             (uint32_t)(cl * esz));
    } else {
      auto rec_load = [&](int32_t i) -> uint32_t {
        return rp[16 * (int64_t)(i < n ? i : n - 1)];
      };
      const uint32_t km1 = (uint32_t)(g.K - 1);   // as in the asm loop: B rows stay in bounds
      uint32_t RV[2 * D];
      uint32_t HD[D];
      U BV[D];
#pragma unroll
      for (int j = 0; j < D; ++j) RV[j] = rec_load(j);
#pragma unroll
      for (int j = 0; j < D; ++j) {
        HD[j] = __builtin_amdgcn_readfirstlane(RV[j]);
        BV[j] = load_unit<TB, V, false>(g.B, g.ldb, min(HD[j] >> 8, km1), n0, g.N);
        RV[D + j] = rec_load(D + j);
      }
      for (int32_t base = 0; base < n; base += 2 * D) {
#pragma unroll
        for (int u = 0; u < 2 * D; ++u) {
          const int32_t i = base + u;
          if (i >= n) break;
          float b[V];
          unit_to_float<TB, V>(BV[u % D], b);
          Rec<MR, V>::run(acc, RV[u], HD[u % D] & 0xFFu, b);
          const uint32_t h2 = __builtin_amdgcn_readfirstlane(RV[(u + D) % (2 * D)]);
          HD[u % D] = h2;
          BV[u % D] = load_unit<TB, V, false>(g.B, g.ldb, min(h2 >> 8, km1), n0, g.N);
          RV[u] = rec_load(i + 2 * D);
        }
      }
    }
  }

  // ---- add the H partial tiles in a fixed order: t0 + t1 for H = 2,
  // (t0 + t2) + (t1 + t3) for H = 4.  The register tile is only read here,
  // so it needs no second copy.
  constexpr int TS = MR * 64 * V;  // floats per tile image
  if constexpr (H == 4) {
    if (w >= 2) tile_to_lds<MR, V>(acc, red + (w - 2) * TS, lane);
    __syncthreads();
    if (w < 2) tile_accumulate_lds<MR, V>(acc, red + w * TS, lane);
    __syncthreads();
  } else if constexpr (H == 2) {
    if (w == 1) tile_to_lds<MR, V>(acc, red, lane);
    __syncthreads();
  }
  if (w != 0) return;

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
        const int o = (q * 64 + lane) * V + j;
        if constexpr (H == 4) v[j] = red[o] + red[TS + o];
        else if constexpr (H == 2) v[j] = tile_at<MR>(acc, q, j) + red[o];
        else v[j] = tile_at<MR>(acc, q, j);
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

template <int MR, int V, int H, int TB>
int32_t launch_one(const SpmmArgs& g, int depth, hipStream_t st) {
  const int64_t nb = (int64_t)g.n_panels * g.n_chunks * g.k_split;
  if (nb == 0) return ROSKO_OK;
  if (nb > INT32_MAX) {
    set_error("spmm grid too large (%lld workgroups)", (long long)nb);
    return ROSKO_EUNSUPPORTED;
  }
  const size_t lds = (H == 4 ? 2 : (H == 2 ? 1 : 0)) * (size_t)MR * 64 * V * sizeof(float);
  if (!g.vec)
    hipLaunchKernelGGL((k_spmm_rows<MR, V, H, TB, false, 4>), dim3((unsigned)nb), dim3(64 * H),
                       lds, st, g);
  else if (depth == 8)
    hipLaunchKernelGGL((k_spmm_rows<MR, V, H, TB, true, 8>), dim3((unsigned)nb), dim3(64 * H),
                       lds, st, g);
  else
    hipLaunchKernelGGL((k_spmm_rows<MR, V, H, TB, true, 4>), dim3((unsigned)nb), dim3(64 * H),
                       lds, st, g);
  ROSKO_LAUNCH_CHECK("k_spmm_rows");
  return ROSKO_OK;
}

template <int MR, int V, int TB>
int32_t dispatch_h(const SpmmArgs& g, int H, int depth, hipStream_t s) {
  switch (H) {
    case 1: return launch_one<MR, V, 1, TB>(g, depth, s);
    case 2: return launch_one<MR, V, 2, TB>(g, depth, s);
    case 4: return launch_one<MR, V, 4, TB>(g, depth, s);
    default: break;
  }
  set_error("unsupported waves per tile %d (1, 2 or 4)", H);
  return ROSKO_EUNSUPPORTED;
}

// Supported (tile height, columns per lane) pairs keep the register tile at
// 32, 64 or 128 VGPRs.
template <int TB>
int32_t dispatch_tile(const SpmmArgs& g, int MRt, int V, int H, int depth, hipStream_t s) {
  if (MRt == 8 && V == 4) return dispatch_h<8, 4, TB>(g, H, depth, s);
  if (MRt == 16 && V == 4) return dispatch_h<16, 4, TB>(g, H, depth, s);
  if (MRt == 32 && V == 4) return dispatch_h<32, 4, TB>(g, H, depth, s);
  if (MRt == 32 && V == 2) return dispatch_h<32, 2, TB>(g, H, depth, s);
  if (MRt == 64 && V == 2) return dispatch_h<64, 2, TB>(g, H, depth, s);
  if (MRt == 128 && V == 1) return dispatch_h<128, 1, TB>(g, H, depth, s);
  set_error("unsupported register tile: height %d with %d columns per lane", MRt, V);
  return ROSKO_EUNSUPPORTED;
}

}  // namespace
}  // namespace rosko
