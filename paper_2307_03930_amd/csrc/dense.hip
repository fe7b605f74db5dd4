// Dense-MFMA panel path (plan path ROSKO_PATH_DENSE).
//
// Row skipping pays while a column of a panel holds few nonzeros; once the
// panels are dense enough the matrix cores win, because they run zeros at a
// multiple of the vector rate (the method itself beats dense multiplication
// only above about 75% sparsity, Sec. 5.3, and hands lower sparsities to a
// dense library in Sec. 5.4).  This path computes every panel
// densely from the packed form:
//   1. k_densify_*:   the column records are scattered into a zero-filled
//                     dense copy Ad (M_pad x K_pad) -- exact, since the
//                     records hold the values packing stored;
//   2. k_transpose_b: B (K x N) becomes Bt (N_pad x K_pad) so that both MFMA
//                     operands are contiguous along k;
//   3. k_dense_mfma:  C = Ad * Bt^T on 128 x 128 tiles, four wavefronts of
//                     2 x 2 MFMA 32x32 blocks each, A and B tiles staged
//                     through LDS with the next K step's loads in flight,
//                     epilogue with the FP8 row scale and beta.
// Operand type: BF16 MFMA (v_mfma_f32_32x32x16_bf16) when both A's values
// and B are exactly BF16 (BF16 or FP8 values, BF16 B); FP32 MFMA
// (v_mfma_f32_32x32x2_f32) otherwise.  Accumulation is FP32 either way.
#include <algorithm>

#include "internal.h"

namespace rosko {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128, BN = 128;
constexpr int KALIGN = 32;   // K is padded to this (a multiple of both BKs)

// BK: K step of one staged tile; PAD: LDS row padding against bank conflicts
template <bool BF> struct DT;
template <> struct DT<true> {
  using T = uint16_t;
  static constexpr int BK = 32, PAD = 8;
};
template <> struct DT<false> {
  using T = float;
  static constexpr int BK = 16, PAD = 1;
};

__device__ __forceinline__ uint16_t f32_to_bf16_exact(float x) {
  // only called on values that are exactly BF16 (BF16 / FP8 codes)
  return (uint16_t)(__float_as_uint(x) >> 16);
}

template <bool BF>
__global__ void __launch_bounds__(256)
k_densify_zero(typename DT<BF>::T* __restrict__ Ad, int64_t count) {
  using T = typename DT<BF>::T;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256)
    Ad[i] = (T)0;
}

// One workgroup per panel: its threads stride over the panel's column
// records and write each record's values at (row, k) of Ad.
template <bool BF>
__global__ void __launch_bounds__(256)
k_densify_scatter(const uint32_t* __restrict__ rec, const int64_t* __restrict__ kblk, int64_t nkb,
                  int32_t mr, typename DT<BF>::T* __restrict__ Ad, int64_t Kp) {
  const int64_t p = blockIdx.x;
  const int64_t r0 = kblk[p * (nkb + 1)], r1 = kblk[p * (nkb + 1) + nkb];
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
    const uint32_t* R = rec + r * 16;
    const uint32_t hdr = R[0];
    const int64_t k = hdr >> 8;
    const int cnt = (int)(hdr & 0xFFu);
    if (k >= Kp || cnt > 12) continue;           // never true for a packed matrix
    for (int t = 0; t < cnt; ++t) {
      const int row = (int)((R[1 + t / 4] >> (8 * (t % 4))) & 0xFFu);
      if (row >= mr) continue;                    // never true for a packed matrix
      const float v = __uint_as_float(R[4 + t]);
      const int64_t off = (p * mr + row) * Kp + k;
      if constexpr (BF) Ad[off] = f32_to_bf16_exact(v);
      else Ad[off] = v;
    }
  }
}

// Bt[n][k] = B[k][n] for n < N, k < K; zero in the padding.  32 x 32 tiles
// through LDS (one extra column against bank conflicts).
template <int TB, bool BF>
__global__ void __launch_bounds__(256)
k_transpose_b(const void* __restrict__ B, int64_t K, int64_t N, int64_t ldb,
              typename DT<BF>::T* __restrict__ Bt, int64_t Kp) {
  using T = typename DT<BF>::T;
  __shared__ float tile[32][33];
  const int64_t k0 = (int64_t)blockIdx.y * 32, n0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int i = ty; i < 32; i += 8) {
    const int64_t k = k0 + i, n = n0 + tx;
    float x = 0.0f;
    if (k < K && n < N) {
      if constexpr (TB == ROSKO_F32) x = reinterpret_cast<const float*>(B)[k * ldb + n];
      else x = __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(B)[k * ldb + n] << 16);
    }
    tile[i][tx] = x;
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int64_t n = n0 + i, k = k0 + tx;
    const float x = tile[tx][i];
    if constexpr (BF) Bt[n * Kp + k] = f32_to_bf16_exact(x);
    else Bt[n * Kp + k] = x;
  }
}

__device__ __forceinline__ int64_t xcd_remap2(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, rem = nb & 7, x = b & 7, pos = b >> 3;
  const int64_t start = (x < rem) ? x * (q + 1) : rem * (q + 1) + (x - rem) * q;
  return start + pos;
}

// C[m][n] = scale_m * sum_k Ad[m][k] Bt[n][k] (+ C[m][n] when beta).
// Workgroup tile 128 x 128, wavefront w owns rows 64*(w>>1).., columns
// 64*(w&1).. as 2 x 2 blocks of 32 x 32.  MFMA 32x32 output layout: lane l,
// accumulator r hold row 8*(r/4) + 4*(l/32) + r%4, column l%32.
template <bool BF>
__global__ void __launch_bounds__(256)
k_dense_mfma(const typename DT<BF>::T* __restrict__ Ad, const typename DT<BF>::T* __restrict__ Bt,
             int64_t Kp, int64_t M, int64_t N, int64_t n_tiles_n, float* __restrict__ C,
             int64_t ldc, const float* __restrict__ row_scale, int32_t beta) {
  using T = typename DT<BF>::T;
  constexpr int BK = DT<BF>::BK, PAD = DT<BF>::PAD;
  constexpr int LD = BK + PAD;                          // LDS row length (elements)
  __shared__ __align__(16) T As[2][BM * LD];
  __shared__ __align__(16) T Bs[2][BN * LD];

  const int64_t tile = xcd_remap2(blockIdx.x, gridDim.x);
  const int64_t bm = tile / n_tiles_n, bn = tile % n_tiles_n;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const T* Ag = Ad + bm * BM * Kp;
  const T* Bg = Bt + bn * BN * Kp;

  // global -> registers: a tile is 128 rows x BK elements; each thread moves
  // 16-byte chunks (4 per row, 2 per thread per tile)
  constexpr int EPC = 16 / sizeof(T);                   // elements per chunk
  constexpr int CPR = BK / EPC;                         // chunks per row
  constexpr int NCH = BM * CPR / 256;                   // chunks per thread
  uint4 ra[NCH], rb[NCH];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int id = t + c * 256, row = id / CPR, ch = id % CPR;
      ra[c] = *reinterpret_cast<const uint4*>(Ag + row * Kp + k0 + ch * EPC);
      rb[c] = *reinterpret_cast<const uint4*>(Bg + row * Kp + k0 + ch * EPC);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int id = t + c * 256, row = id / CPR, ch = id % CPR;
      if constexpr (BF) {
        *reinterpret_cast<uint4*>(&As[buf][row * LD + ch * EPC]) = ra[c];
        *reinterpret_cast<uint4*>(&Bs[buf][row * LD + ch * EPC]) = rb[c];
      } else {   // rows of 17 floats are not 16-byte aligned: four dword stores
        float* a = reinterpret_cast<float*>(&As[buf][row * LD + ch * EPC]);
        float* b = reinterpret_cast<float*>(&Bs[buf][row * LD + ch * EPC]);
        a[0] = __uint_as_float(ra[c].x); a[1] = __uint_as_float(ra[c].y);
        a[2] = __uint_as_float(ra[c].z); a[3] = __uint_as_float(ra[c].w);
        b[0] = __uint_as_float(rb[c].x); b[1] = __uint_as_float(rb[c].y);
        b[2] = __uint_as_float(rb[c].z); b[3] = __uint_as_float(rb[c].w);
      }
    }
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f32x16)(0.0f);

  const int64_t nk = Kp / BK;   // Kp is a multiple of KALIGN, hence of BK
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t ks = 0; ks < nk; ++ks) {
    const int buf = (int)(ks & 1);
    if (ks + 1 < nk) gload((ks + 1) * BK);
    const T* as = As[buf];
    const T* bs = Bs[buf];
    if constexpr (BF) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 16) {
        const int kof = kk + 8 * (lane >> 5);
        bf16x8 av[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int r = wm * 64 + i * 32 + (lane & 31);
          av[i] = *reinterpret_cast<const bf16x8*>(&as[r * LD + kof]);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int c = wn * 64 + j * 32 + (lane & 31);
          bv[j] = *reinterpret_cast<const bf16x8*>(&bs[c * LD + kof]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        const int kof = kk + (lane >> 5);
        float av[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) av[i] = as[(wm * 64 + i * 32 + (lane & 31)) * LD + kof];
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j] = bs[(wn * 64 + j * 32 + (lane & 31)) * LD + kof];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
    }
    if (ks + 1 < nk) {
      sstore(buf ^ 1);
    }
    __syncthreads();
  }

  // epilogue
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = bm * BM + wm * 64 + i * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r & 3);
        const int64_t col = bn * BN + wn * 64 + j * 32 + (lane & 31);
        if (row < M && col < N) {
          float v = acc[i][j][r];
          if (row_scale) v *= row_scale[row];
          float* c = C + row * ldc + col;
          *c = beta ? *c + v : v;
        }
      }
}

bool use_bf16_mfma(const rosko_packed* A, int32_t b_dtype) {
  return A->val_dtype != ROSKO_F32 && b_dtype == ROSKO_BF16;
}

struct DenseWs {
  size_t ad, bt, bytes;
  int64_t Mp, Kp, Np;
};
DenseWs dense_ws_layout(const rosko_packed* A, int64_t N, bool bf) {
  DenseWs L{};
  const size_t es = bf ? 2 : 4;
  L.Mp = round_up(std::max<int64_t>(1, (int64_t)A->n_panels * A->mr), BM);
  L.Kp = round_up(std::max<int64_t>(1, A->K), KALIGN);
  L.Np = round_up(std::max<int64_t>(1, N), BN);
  L.ad = 0;
  L.bt = (size_t)round_up((int64_t)(es * L.Mp * L.Kp), 256);
  L.bytes = L.bt + (size_t)round_up((int64_t)(es * L.Np * L.Kp), 256);
  return L;
}

template <bool BF>
int32_t run_dense(const rosko_packed* A, const void* B, int32_t b_dtype, int64_t N, int64_t ldb,
                  float* C, int64_t ldc, int32_t beta, void* ws, const DenseWs& L,
                  hipStream_t s) {
  using T = typename DT<BF>::T;
  T* Ad = reinterpret_cast<T*>(static_cast<char*>(ws) + L.ad);
  T* Bt = reinterpret_cast<T*>(static_cast<char*>(ws) + L.bt);
  const int64_t nkb = (A->K + ROSKO_KSTEP - 1) / ROSKO_KSTEP;
  const int64_t nad = L.Mp * L.Kp;
  hipLaunchKernelGGL(k_densify_zero<BF>, dim3((unsigned)std::min<int64_t>(ceil_div(nad, 256), 8192)),
                     dim3(256), 0, s, Ad, nad);
  ROSKO_LAUNCH_CHECK("k_densify_zero");
  if (A->n_panels > 0) {
    hipLaunchKernelGGL(k_densify_scatter<BF>, dim3((unsigned)A->n_panels), dim3(256), 0, s,
                       A->rec, A->kblk_ptr, nkb, A->mr, Ad, L.Kp);
    ROSKO_LAUNCH_CHECK("k_densify_scatter");
  }
  const dim3 tg((unsigned)(L.Np / 32), (unsigned)(L.Kp / 32));
  if (b_dtype == ROSKO_F32)
    hipLaunchKernelGGL((k_transpose_b<ROSKO_F32, BF>), tg, dim3(256), 0, s, B, A->K, N, ldb, Bt, L.Kp);
  else
    hipLaunchKernelGGL((k_transpose_b<ROSKO_BF16, BF>), tg, dim3(256), 0, s, B, A->K, N, ldb, Bt, L.Kp);
  ROSKO_LAUNCH_CHECK("k_transpose_b");
  const int64_t tm = ceil_div(A->M, BM), tn = L.Np / BN;
  const float* rs = A->val_dtype == ROSKO_FP8_E4M3 ? A->row_scale : nullptr;
  hipLaunchKernelGGL(k_dense_mfma<BF>, dim3((unsigned)(tm * tn)), dim3(256), 0, s, Ad, Bt, L.Kp,
                     A->M, N, tn, C, ldc, rs, beta);
  ROSKO_LAUNCH_CHECK("k_dense_mfma");
  return ROSKO_OK;
}

}  // namespace

size_t dense_ws_bytes(const rosko_packed* A, int64_t N, int32_t b_dtype) {
  return dense_ws_layout(A, N, use_bf16_mfma(A, b_dtype)).bytes;
}

int32_t launch_spmm_dense(const rosko_packed* A, const void* B, int32_t b_dtype, int64_t N,
                          int64_t ldb, float* C, int64_t ldc, int32_t beta, void* ws,
                          size_t ws_bytes, hipStream_t s) {
  const bool bf = use_bf16_mfma(A, b_dtype);
  const DenseWs L = dense_ws_layout(A, N, bf);
  if (ws == nullptr || ws_bytes < L.bytes) {
    set_error("dense path workspace %zu bytes < %zu", ws_bytes, L.bytes);
    return ROSKO_ESMALLBUF;
  }
  if ((uintptr_t)ws % 256 != 0) {
    set_error("dense path workspace must be 256-byte aligned");
    return ROSKO_EINVAL;
  }
  return bf ? run_dense<true>(A, B, b_dtype, N, ldb, C, ldc, beta, ws, L, s)
            : run_dense<false>(A, B, b_dtype, N, ldb, C, ldc, beta, ws, L, s);
}

}  // namespace rosko
