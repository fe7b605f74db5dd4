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
// Lane's V columns [n0, n0+V) of B row `row_off`.  Branch-free, so every
// lane issues the load (keeping the memory counters in order for the
// one-column-ahead prefetch): out-of-range columns read column 0 of the row
// and are replaced by zero.  With vec, N is a multiple of V, so a lane's
// columns are all in range or all out.
template <int TB, int V>
__device__ __forceinline__ void load_b(const void* __restrict__ B, int64_t row_off, int64_t n0,
                                       int64_t N, bool VEC, float* b) {
  if (TB == ROSKO_F32) {
    const float* p = reinterpret_cast<const float*>(B) + row_off;
    if (VEC) {
      const bool in = n0 < N;
      const float* q = p + (in ? n0 : 0);
      float x[V];
      if (V == 4) { float4 y = *reinterpret_cast<const float4*>(q); x[0] = y.x; x[1] = y.y; x[2] = y.z; x[3] = y.w; }
      else if (V == 2) { float2 y = *reinterpret_cast<const float2*>(q); x[0] = y.x; x[1] = y.y; }
      else x[0] = q[0];
#pragma unroll
      for (int j = 0; j < V; ++j) b[j] = in ? x[j] : 0.0f;
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const bool in = n0 + j < N;
        const float x = p[in ? n0 + j : 0];
        b[j] = in ? x : 0.0f;
      }
    }
  } else {
    const uint16_t* p = reinterpret_cast<const uint16_t*>(B) + row_off;
    if (VEC) {
      const bool in = n0 < N;
      const uint16_t* q = p + (in ? n0 : 0);
      float x[V];
      if (V == 4) {
        uint2 y = *reinterpret_cast<const uint2*>(q);
        x[0] = __uint_as_float(y.x << 16); x[1] = __uint_as_float(y.x & 0xFFFF0000u);
        x[2] = __uint_as_float(y.y << 16); x[3] = __uint_as_float(y.y & 0xFFFF0000u);
      } else if (V == 2) {
        uint32_t y = *reinterpret_cast<const uint32_t*>(q);
        x[0] = __uint_as_float(y << 16); x[1] = __uint_as_float(y & 0xFFFF0000u);
      } else {
        x[0] = __uint_as_float((uint32_t)q[0] << 16);
      }
#pragma unroll
      for (int j = 0; j < V; ++j) b[j] = in ? x[j] : 0.0f;
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const bool in = n0 + j < N;
        const float x = __uint_as_float((uint32_t)p[in ? n0 + j : 0] << 16);
        b[j] = in ? x : 0.0f;
      }
    }
  }
}

template <int V>
__device__ __forceinline__ void store_c(float* __restrict__ C, int64_t off, int64_t n0, int64_t N,
                                        bool VEC, const float* v, int beta) {
  float* p = C + off + n0;
  if (VEC && n0 + V <= N) {
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
// tile ids (which share B columns) run on the same XCD and hit its L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, rem = nb & 7, x = b & 7, pos = b >> 3;
  const int64_t start = (x < rem) ? x * (q + 1) : rem * (q + 1) + (x - rem) * q;
  return start + pos;
}


constexpr int kChunk = 8;   // values fetched per scalar batch

template <int MR, int V, int W, int TA, int TB>
__global__ void __launch_bounds__(64 * W)
k_spmm_sparse(SpmmArgs g) {
  constexpr int NT = tile_nt<MR, V>();
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t chunk = tile / g.n_panels, p = tile - chunk * g.n_panels;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t n0 = chunk * (64 * V) + (int64_t)lane * V;
  const bool vec = g.vec != 0;

  Tile<NT> acc;
#pragma unroll
  for (int q = 0; q < NT; ++q) acc.t[q] = (f32x32)(0.0f);

  cptr<int64_t> panel_col_ptr = as_const<int64_t>(g.panel_col_ptr);
  cptr<int32_t> col_ind = as_const<int32_t>(g.col_ind);
  cptr<int32_t> col_nnz = as_const<int32_t>(g.col_nnz);
  cptr<int64_t> col_ptr = as_const<int64_t>(g.col_ptr);
  const int64_t c_lo = panel_col_ptr[p], c_hi = panel_col_ptr[p + 1];
  const int64_t ncp = c_hi - c_lo;
  const int64_t cw0 = c_lo + (ncp * wid) / W, cw1 = c_lo + (ncp * (wid + 1)) / W;

  if (cw0 < cw1) {
    int64_t z = col_ptr[cw0];
    int32_t kc = col_ind[cw0], nc = col_nnz[cw0];
    float b[V];
    load_b<TB, V>(g.B, (int64_t)kc * g.ldb, n0, g.N, vec, b);
    for (int64_t c = cw0; c < cw1; ++c) {
      // next column's B row is requested before this column's values run
      int32_t kn = 0, nn = 0;
      float bn[V];
#pragma unroll
      for (int j = 0; j < V; ++j) bn[j] = 0.0f;
      if (c + 1 < cw1) {
        kn = col_ind[c + 1];
        nn = col_nnz[c + 1];
        load_b<TB, V>(g.B, (int64_t)kn * g.ldb, n0, g.N, vec, bn);
      }
      for (int base = 0; base < nc; base += kChunk) {
        float av[kChunk];
        uint32_t rv[kChunk];
#pragma unroll
        for (int t = 0; t < kChunk; ++t) av[t] = load_a<TA>(g.val, z + base + t);
        load_loc8<MR>(g.loc, z + base, rv);
        const int rem = nc - base;
#pragma unroll
        for (int t = 0; t < kChunk; ++t) {
          if (t < rem) {
            const uint32_t r = __builtin_amdgcn_readfirstlane(rv[t]);
            const float a = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(av[t])));
            Fma<MR, V>::run(acc, r, a, b);
          }
        }
      }
      z += nc;
      kc = kn;
      nc = nn;
#pragma unroll
      for (int j = 0; j < V; ++j) b[j] = bn[j];
    }
  }

  // ---- epilogue.  W = 1: the wave stores its tile from registers.  W > 1:
  // every wave writes its partial tile to LDS, then all threads of the
  // workgroup add the W partials in wave order (fixed, so the sum does not
  // depend on timing) and store C row by row with coalesced accesses.
  const int rows = (int)min((int64_t)g.mr, g.M - p * g.mr);
  cptr<float> row_scale = as_const<float>(g.row_scale);
  if constexpr (W == 1) {
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
        if (TA == ROSKO_FP8_E4M3) {
          const float sc = row_scale[row];
#pragma unroll
          for (int j = 0; j < V; ++j) v[j] *= sc;
        }
        store_c<V>(g.C, row * g.ldc, n0, g.N, vec, v, g.beta);
      }
    }
  } else {
    extern __shared__ float red[];   // W * MR * 64 * V floats, [w][r][lane*V + j]
    float* dst = red + (int64_t)wid * MR * 64 * V;
#pragma unroll
    for (int r = 0; r < MR; ++r) {
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const int idx = j * MR + r;
        dst[(r * 64 + lane) * V + j] = acc.t[idx >> 5][idx & 31];
      }
    }
    __syncthreads();
    const int64_t col0 = chunk * (64 * V);
    for (int e = threadIdx.x; e < rows * 64 * V; e += 64 * W) {
      const int r = e / (64 * V), cc = e - r * (64 * V);
      const int64_t col = col0 + cc;
      if (col >= g.N) continue;
      float sum = red[e];
      for (int w = 1; w < W; ++w) sum += red[(int64_t)w * MR * 64 * V + e];
      const int64_t row = p * g.mr + r;
      if (TA == ROSKO_FP8_E4M3) sum *= row_scale[row];
      float* cp = g.C + row * g.ldc + col;
      *cp = g.beta ? *cp + sum : sum;
    }
  }
}

template <int MR, int V, int W, int TA, int TB>
int32_t launch_one(const SpmmArgs& g, hipStream_t s) {
  const int64_t chunks = ceil_div(g.N, 64 * V);
  const int64_t nb = chunks * g.n_panels;
  if (nb == 0) return ROSKO_OK;
  if (nb > INT32_MAX) {
    set_error("spmm grid too large (%lld workgroups)", (long long)nb);
    return ROSKO_EUNSUPPORTED;
  }
  const size_t lds = (W > 1) ? sizeof(float) * (size_t)W * MR * 64 * V : 0;
  hipLaunchKernelGGL((k_spmm_sparse<MR, V, W, TA, TB>), dim3((unsigned)nb), dim3(64 * W), lds,
                     s, g);
  ROSKO_LAUNCH_CHECK("k_spmm_sparse");
  return ROSKO_OK;
}

template <int MR, int V, int TA, int TB>
int32_t dispatch_waves(const SpmmArgs& g, int waves, hipStream_t s) {
  switch (waves) {
    case 1: return launch_one<MR, V, 1, TA, TB>(g, s);
    case 2: return launch_one<MR, V, 2, TA, TB>(g, s);
    case 4: return launch_one<MR, V, 4, TA, TB>(g, s);
    default: break;
  }
  set_error("unsupported waves per workgroup %d (1, 2 or 4)", waves);
  return ROSKO_EUNSUPPORTED;
}

// Supported (tile height, columns per lane) pairs keep the register tile at
// 32, 64 or 128 VGPRs.
template <int TA, int TB>
int32_t dispatch_tile(const SpmmArgs& g, int H, int V, int W, hipStream_t s) {
  if (H == 8 && V == 4) return dispatch_waves<8, 4, TA, TB>(g, W, s);
  if (H == 16 && V == 4) return dispatch_waves<16, 4, TA, TB>(g, W, s);
  if (H == 32 && V == 4) return dispatch_waves<32, 4, TA, TB>(g, W, s);
  if (H == 32 && V == 2) return dispatch_waves<32, 2, TA, TB>(g, W, s);
  if (H == 64 && V == 2) return dispatch_waves<64, 2, TA, TB>(g, W, s);
  if (H == 128 && V == 1) return dispatch_waves<128, 1, TA, TB>(g, W, s);
  set_error("unsupported register tile: height %d with %d columns per lane", H, V);
  return ROSKO_EUNSUPPORTED;
}

}  // namespace
}  // namespace rosko
