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
// registers (v24 for the 128-register tiles at depth 4: 158 VGPRs in all).
template <int NT>
struct Tile { f32x32 t[NT]; };

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

#include "spmm_loop.inc"

// One workgroup: H wavefronts on one (panel, column chunk) tile; split s of
// k_split.  The panel's records are cut into k_split*H equal runs (by record
// count, so the waves get the same work); wavefront w takes run s*H + w,
// keeps its partial tile in VGPRs, and the H tiles are added through LDS in a
// fixed order.  Each wavefront streams its records and the B rows they name
// with vector loads, DV records ahead of the FMAs, so no step waits on a
// single load round trip.  B and C rows are accessed V elements at a time
// (the host checks their alignment).
template <int MR, int V, int H, int TB, int DV>
__global__ void __launch_bounds__(64 * H)
k_spmm_rows(SpmmArgs g) {
  constexpr int NT = tile_nt<MR, V>();
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

  Tile<NT> acc;
#pragma unroll
  for (int q = 0; q < NT; ++q) acc.t[q] = (f32x32)(0.0f);

  if (n > 0) {
    {
      // the record loop in one asm block (spmm_loop.inc); buffer loads with
      // 32-bit offsets from this run's first record and from B.  Each buffer
      // is sized exactly (the records from this run's first to the array's
      // end, capped below 4 GiB -- a run is far shorter; K rows of ldb
      // elements; b_rows of them for a flat B), so the hardware returns zero
      // for any load outside it instead of touching other memory
      constexpr uint32_t esz = TB == ROSKO_F32 ? 4 : 2;
      const int64_t rbytes = min((g.rec_bound - a) * 64, (int64_t)0xFFFFFFC0);
      const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(g.rec + a * 16), 0, (int)(uint32_t)rbytes, 0x00020000);
      const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
          (void*)g.B, 0, (int)(uint32_t)(g.b_rows * g.ldb * esz), 0x00020000);
      const int64_t cl = n0 < g.N - V ? n0 : g.N - V;
      RkLoop<MR, V, TB, DV>::run(acc, (uint32_t)n, rr, rb, (uint32_t)(g.ldb * esz),
                             (uint32_t)(g.b_rows - 1), (uint32_t)(lane & 15) * 4u,
                             (uint32_t)(cl * esz));
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
        store_c<V>(g.C, perm_row(g.row_perm, row, g.M) * g.ldc, n0, g.N, true, v, g.beta);
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
  if (depth == 8)
    hipLaunchKernelGGL((k_spmm_rows<MR, V, H, TB, 8>), dim3((unsigned)nb), dim3(64 * H),
                       lds, st, g);
  else
    hipLaunchKernelGGL((k_spmm_rows<MR, V, H, TB, 4>), dim3((unsigned)nb), dim3(64 * H),
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
