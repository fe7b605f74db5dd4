// Dense-MFMA path (plan path ROSKO_PATH_DENSE).
//
// Row skipping pays while a panel column holds few nonzeros; once the
// panels are dense enough the matrix cores win, because they run zeros at a
// multiple of the vector rate (the method beats dense multiplication only
// above about 75% sparsity, Sec. 5.3, and training hands lower sparsities to
// a dense library, Sec. 5.4).  This path multiplies every panel densely,
// starting from the packed form (A itself is not an argument of rosko_spmm):
//   1. k_densify_lds: (panels of up to 64 rows) one workgroup per (panel,
//                     256-column block) builds its block of the dense copy
//                     Ad (Mp x Kp) in LDS from the column records -- exact,
//                     since the records hold the values packing stored --
//                     and writes it out as whole rows; k_densify (taller
//                     panels) zero-fills the block in Ad and scatters into it;
//   2. k_transpose_b: Bt (Np x Kp) = B^T, so both MFMA operands run along k;
//   3. k_dense_gemm:  C = s_m * Ad Bt^T (+ C) on 128 x 128 tiles, four
//                     wavefronts of 2 x 2 blocks of 32 x 32, K steps staged
//                     through LDS with the next step's global loads in flight.
// Operands: BF16 MFMA (v_mfma_f32_32x32x16_bf16) when A's values and B are
// exactly BF16 (BF16 or FP8 values, BF16 B), else FP32 MFMA
// (v_mfma_f32_32x32x2f32); FP32 accumulation either way.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace rosko {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTile = 128;       // rows and columns of a GEMM tile
constexpr int kKAlign = 64;      // Kp: K rounded up to this (a multiple of both K steps)

template <bool BF> struct Op;
template <> struct Op<true> {    // BF16 operands
  using T = uint16_t;
  static constexpr int BK = 64, LDK = 72, EPC = 8;  // K step, LDS row, elements per 16 B
};
template <> struct Op<false> {   // FP32 operands
  using T = float;
  static constexpr int BK = 32, LDK = 36, EPC = 4;
};

__device__ __forceinline__ int64_t ceil_div_dev(int64_t x, int64_t a) { return (x + a - 1) / a; }

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, rem = nb & 7, x = b & 7, pos = b >> 3;
  const int64_t start = (x < rem) ? x * (q + 1) : rem * (q + 1) + (x - rem) * q;
  return start + pos;
}

// Workgroup (p, q): rows [p*mr, p*mr + rows_p) of Ad (and, for the last
// panel, the padding rows up to Mp), columns [q*kDensifyK, (q+1)*kDensifyK)
// of Kp, are zero-filled, then the panel's records with k in that range
// (found through the K-block index) are scattered into them.  Records whose
// column or row is out of range (never written by packing) are skipped.
constexpr int kDensifyK = 512;   // a multiple of ROSKO_KSTEP and of kKAlign
template <bool BF>
__global__ void __launch_bounds__(256)
k_densify(const uint32_t* __restrict__ rec, const int64_t* __restrict__ kblk, int64_t nkb,
          int64_t rec_bound, int32_t mr, int32_t n_panels, int64_t M, int64_t K, int64_t Mp,
          int64_t Kp, typename Op<BF>::T* __restrict__ Ad) {
  using T = typename Op<BF>::T;
  constexpr int EPC = 16 / sizeof(T);             // elements per 16-byte store
  const int64_t p = blockIdx.x;
  const int64_t k_lo = (int64_t)blockIdx.y * kDensifyK;
  const int64_t k_hi = min(k_lo + kDensifyK, Kp);
  const int64_t r0 = p * mr;
  const int rows = (int)min((int64_t)mr, M - r0);
  const int64_t r_end = (p == n_panels - 1) ? Mp : r0 + rows;
  // zero fill: (r_end - r0) rows of (k_hi - k_lo) elements, 16 bytes a store
  const int64_t per_row = (k_hi - k_lo) / EPC;
  const int64_t nz = (r_end - r0) * per_row;
  for (int64_t i = threadIdx.x; i < nz; i += 256) {
    const int64_t r = i / per_row, c = i - r * per_row;
    *reinterpret_cast<uint4*>(Ad + (r0 + r) * Kp + k_lo + c * EPC) = make_uint4(0u, 0u, 0u, 0u);
  }
  __threadfence_block();
  __syncthreads();
  const int64_t jb = k_lo / ROSKO_KSTEP, je = min(ceil_div_dev(k_hi, ROSKO_KSTEP), nkb);
  const int64_t a = min(max(kblk[p * (nkb + 1) + min(jb, nkb)], (int64_t)0), rec_bound);
  const int64_t e = min(max(kblk[p * (nkb + 1) + je], a), rec_bound);
  for (int64_t r = a + threadIdx.x; r < e; r += 256) {
    const uint32_t* R = rec + r * 16;
    const uint32_t hdr = R[0];
    const int64_t k = hdr >> 8;
    const int cnt = (int)(hdr & 0xFFu);
    if (k < k_lo || k >= k_hi || k >= K || cnt > 12) continue;
    for (int t = 0; t < cnt; ++t) {
      const int row = (int)((R[1 + t / 4] >> (8 * (t % 4))) & 0xFFu);
      if (row >= rows) continue;
      const uint32_t bits = R[4 + t];
      T* dst = Ad + (r0 + row) * Kp + k;
      if constexpr (BF) *dst = (uint16_t)(bits >> 16);   // values exactly BF16 here
      else *dst = __uint_as_float(bits);
    }
  }
}

// Panels of at most MAXR rows: workgroup (p, q) builds the block of rows
// [p*mr, p*mr + rows_p) and columns [q*kDenseLdsK, ...) of Ad in LDS -- zero
// it, scatter the panel's records with k in the block into it -- and writes
// it out as whole rows with 16-byte stores, so Ad's lines are written once
// and completely; the last panel's workgroups also zero the padding rows up
// to Mp.  Same record range and skips as k_densify.
constexpr int kDenseLdsK = 256;  // a multiple of ROSKO_KSTEP and of kKAlign
constexpr int kDenseLdsRows = 64;
template <bool BF>
__global__ void __launch_bounds__(256)
k_densify_lds(const uint32_t* __restrict__ rec, const int64_t* __restrict__ kblk, int64_t nkb,
              int64_t rec_bound, int32_t mr, int32_t n_panels, int64_t M, int64_t K,
              int64_t Mp, int64_t Kp, typename Op<BF>::T* __restrict__ Ad) {
  using T = typename Op<BF>::T;
  constexpr int EPC = 16 / sizeof(T);             // elements per 16 bytes
  constexpr int RQ = kDenseLdsK / EPC;            // 16-byte pieces per LDS row
  __shared__ uint4 tile4[kDenseLdsRows * RQ];
  T* tile = reinterpret_cast<T*>(tile4);
  const int64_t p = blockIdx.x;
  const int64_t k_lo = (int64_t)blockIdx.y * kDenseLdsK;
  const int64_t k_hi = min(k_lo + kDenseLdsK, Kp);
  const int64_t r0 = p * mr;
  const int rows = (int)min((int64_t)min(mr, kDenseLdsRows), M - r0);
  for (int i = threadIdx.x; i < rows * RQ; i += 256) tile4[i] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  const int64_t jb = k_lo / ROSKO_KSTEP, je = min(ceil_div_dev(k_hi, ROSKO_KSTEP), nkb);
  const int64_t a = min(max(kblk[p * (nkb + 1) + min(jb, nkb)], (int64_t)0), rec_bound);
  const int64_t e = min(max(kblk[p * (nkb + 1) + je], a), rec_bound);
  // a record as four 16-byte loads: header and row words, then the values
  const uint4* rec4 = reinterpret_cast<const uint4*>(rec);
  for (int64_t r = a + threadIdx.x; r < e; r += 256) {
    const uint4 h = rec4[r * 4];
    const int64_t k = h.x >> 8;
    const int cnt = (int)(h.x & 0xFFu);
    if (k < k_lo || k >= k_hi || k >= K || cnt > 12) continue;
    const uint4 v0 = rec4[r * 4 + 1], v1 = rec4[r * 4 + 2], v2 = rec4[r * 4 + 3];
    const uint32_t rw[3] = {h.y, h.z, h.w};
    const uint32_t vb[12] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w,
                             v2.x, v2.y, v2.z, v2.w};
    const int kk = (int)(k - k_lo);
#pragma unroll
    for (int t = 0; t < 12; ++t) {
      const int row = (int)((rw[t / 4] >> (8 * (t % 4))) & 0xFFu);
      if (t >= cnt || row >= rows) continue;
      if constexpr (BF) tile[row * kDenseLdsK + kk] = (uint16_t)(vb[t] >> 16);   // exact BF16
      else tile[row * kDenseLdsK + kk] = __uint_as_float(vb[t]);
    }
  }
  __syncthreads();
  const int per_row = (int)((k_hi - k_lo) / EPC);
  for (int i = threadIdx.x; i < rows * per_row; i += 256) {
    const int r = i / per_row, c = i - r * per_row;
    *reinterpret_cast<uint4*>(Ad + (r0 + r) * Kp + k_lo + c * EPC) = tile4[r * RQ + c];
  }
  if (p == n_panels - 1) {
    const int pad = (int)(Mp - (r0 + rows));
    for (int i = threadIdx.x; i < pad * per_row; i += 256) {
      const int r = i / per_row, c = i - r * per_row;
      *reinterpret_cast<uint4*>(Ad + (r0 + rows + r) * Kp + k_lo + c * EPC) =
          make_uint4(0u, 0u, 0u, 0u);
    }
  }
}

// Bt[n][k] = B[k][n] for n < N, k < K, zero elsewhere in Np x Kp, through
// 64 x 64 tiles in LDS (held as FP32, one extra column against bank
// conflicts).  VEC (B 16-byte aligned, ldb a multiple of the elements per 16
// bytes): a thread loads 16-byte pieces of B's rows (elements past N or K
// read as zero), and every thread stores 16-byte pieces of Bt's rows (Bt is
// 256-byte aligned and Kp a multiple of 64).  Otherwise the loads are per
// element.
constexpr int kTrT = 64;
template <int TB, bool BF, bool VEC>
__global__ void __launch_bounds__(256)
k_transpose_b(const void* __restrict__ B, int64_t K, int64_t N, int64_t ldb,
              typename Op<BF>::T* __restrict__ Bt, int64_t Kp) {
  using T = typename Op<BF>::T;
  using TI = typename std::conditional<TB == ROSKO_F32, float, uint16_t>::type;
  constexpr int EI = 16 / sizeof(TI), EO = 16 / sizeof(T);   // elements per 16 bytes
  __shared__ float tile[kTrT][kTrT + 1];
  const int64_t k0 = (int64_t)blockIdx.y * kTrT, n0 = (int64_t)blockIdx.x * kTrT;
  const TI* Bi = reinterpret_cast<const TI*>(B);
  auto widen = [](TI x) -> float {
    if constexpr (TB == ROSKO_F32) return x;
    else return __uint_as_float((uint32_t)x << 16);
  };
  // loads: kTrT / EI pieces per row, 256 / (kTrT / EI) rows per pass
  constexpr int PR = kTrT / EI, RP = 256 / PR;
  const int lr = threadIdx.x / PR, lp = threadIdx.x % PR;
#pragma unroll
  for (int i = 0; i < kTrT / RP; ++i) {
    const int kl = lr + i * RP;
    const int64_t k = k0 + kl, n = n0 + lp * EI;
    TI x[EI];
    if (VEC && k < K && n + EI <= N) {
      const uint4 u = *reinterpret_cast<const uint4*>(Bi + k * ldb + n);
      __builtin_memcpy(x, &u, 16);
    } else {
#pragma unroll
      for (int e = 0; e < EI; ++e) x[e] = (k < K && n + e < N) ? Bi[k * ldb + n + e] : (TI)0;
    }
#pragma unroll
    for (int e = 0; e < EI; ++e) tile[kl][lp * EI + e] = widen(x[e]);
  }
  __syncthreads();
  // stores: kTrT / EO pieces per Bt row, 256 / (kTrT / EO) rows per pass
  constexpr int PW = kTrT / EO, WP = 256 / PW;
  const int wr = threadIdx.x / PW, wp = threadIdx.x % PW;
#pragma unroll
  for (int i = 0; i < kTrT / WP; ++i) {
    const int nl = wr + i * WP;
    T y[EO];
#pragma unroll
    for (int e = 0; e < EO; ++e) {
      const float x = tile[wp * EO + e][nl];
      if constexpr (BF) y[e] = (uint16_t)(__float_as_uint(x) >> 16);   // exact: B is BF16
      else y[e] = x;
    }
    uint4 u;
    __builtin_memcpy(&u, y, 16);
    *reinterpret_cast<uint4*>(Bt + (n0 + nl) * Kp + k0 + wp * EO) = u;
  }
}

// One K step of a wavefront's 2 x 2 blocks of 32 x 32 from the LDS tiles.
template <bool BF>
__device__ __forceinline__ void mfma_step(const typename Op<BF>::T* As,
                                          const typename Op<BF>::T* Bs, int lane, int wm,
                                          int wn, f32x16 (&acc)[2][2]) {
  constexpr int BK = Op<BF>::BK, LDK = Op<BF>::LDK;
  if constexpr (BF) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int kof = kk + 8 * (lane >> 5);
      bf16x8 av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        av[i] = *reinterpret_cast<const bf16x8*>(&As[(wm * 64 + i * 32 + (lane & 31)) * LDK + kof]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bv[j] = *reinterpret_cast<const bf16x8*>(&Bs[(wn * 64 + j * 32 + (lane & 31)) * LDK + kof]);
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
      for (int i = 0; i < 2; ++i) av[i] = As[(wm * 64 + i * 32 + (lane & 31)) * LDK + kof];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Bs[(wn * 64 + j * 32 + (lane & 31)) * LDK + kof];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }
}

// C[m][n] = s_m * sum_k Ad[m][k] Bt[n][k] (+ C[m][n] when beta), m < M, n < N.
// Workgroup tile 128 x 128; wavefront w owns rows 64*(w>>1).., columns
// 64*(w&1).. as 2 x 2 blocks of 32 x 32.  A K step moves 128 x BK of each
// operand global -> registers (16 bytes per thread, 4 per operand) one step
// ahead, then registers -> LDS between two barriers.  MFMA 32 x 32 layouts:
// the A operand of lane l is row l%32 at k offset EPC*(l/32) (8 BF16 or 1
// FP32), the B operand the same for a column, and accumulator r of lane l is
// (row 8*(r/4) + 4*(l/32) + r%4, column l%32).
template <bool BF>
__global__ void __launch_bounds__(256, 2)
k_dense_gemm(const typename Op<BF>::T* __restrict__ Ad, const typename Op<BF>::T* __restrict__ Bt,
             int64_t Kp, int64_t M, int64_t N, int64_t tiles_n, float* __restrict__ C,
             int64_t ldc, const float* __restrict__ row_scale,
             const int32_t* __restrict__ row_perm, int32_t beta) {
  using T = typename Op<BF>::T;
  constexpr int BK = Op<BF>::BK, LDK = Op<BF>::LDK, EPC = Op<BF>::EPC;
  __shared__ __align__(16) T As[kTile * LDK];
  __shared__ __align__(16) T Bs[kTile * LDK];

  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t bm = tile / tiles_n, bn = tile % tiles_n;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const T* Ag = Ad + bm * kTile * Kp;
  const T* Bg = Bt + bn * kTile * Kp;

  // chunk c of a thread: id = t + 256 c, row id / CPR, 16-byte piece id % CPR
  constexpr int CPR = BK / EPC, NCH = kTile * CPR / 256;
  static_assert(NCH == 4, "both operand types move 4 chunks per thread per K step");
  // chunk offsets of this thread (global and LDS), constant over the K steps
  const int r0c = t / CPR, chc = t % CPR, rstep = 256 / CPR;
  const int64_t g0 = r0c * Kp + chc * EPC, gs = rstep * Kp;
  const int s0 = r0c * LDK + chc * EPC, ss = rstep * LDK;
  uint4 xa0, xa1, xa2, xa3, xb0, xb1, xb2, xb3;
#define RK_GLOAD(S, K0)                                                            \
  {                                                                                \
    const T* pa = Ag + g0 + (K0);                                                  \
    const T* pb = Bg + g0 + (K0);                                                  \
    S##a0 = *reinterpret_cast<const uint4*>(pa);                                   \
    S##a1 = *reinterpret_cast<const uint4*>(pa + gs);                              \
    S##a2 = *reinterpret_cast<const uint4*>(pa + 2 * gs);                          \
    S##a3 = *reinterpret_cast<const uint4*>(pa + 3 * gs);                          \
    S##b0 = *reinterpret_cast<const uint4*>(pb);                                   \
    S##b1 = *reinterpret_cast<const uint4*>(pb + gs);                              \
    S##b2 = *reinterpret_cast<const uint4*>(pb + 2 * gs);                          \
    S##b3 = *reinterpret_cast<const uint4*>(pb + 3 * gs);                          \
  }
#define RK_SSTORE(S)                                                               \
  {                                                                                \
    *reinterpret_cast<uint4*>(&As[s0]) = S##a0;                                    \
    *reinterpret_cast<uint4*>(&As[s0 + ss]) = S##a1;                               \
    *reinterpret_cast<uint4*>(&As[s0 + 2 * ss]) = S##a2;                           \
    *reinterpret_cast<uint4*>(&As[s0 + 3 * ss]) = S##a3;                           \
    *reinterpret_cast<uint4*>(&Bs[s0]) = S##b0;                                    \
    *reinterpret_cast<uint4*>(&Bs[s0 + ss]) = S##b1;                               \
    *reinterpret_cast<uint4*>(&Bs[s0 + 2 * ss]) = S##b2;                           \
    *reinterpret_cast<uint4*>(&Bs[s0 + 3 * ss]) = S##b3;                           \
  }

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f32x16)(0.0f);

  // the next step's global loads are in flight while this one is computed;
  // two barriers per step (reads done; next step stored).  (A second register
  // set for two steps in flight measured no faster: 88 against 84 us on the
  // 4096 x 4096 x 2048 BF16 product.)
  const int64_t nk = Kp / BK;
  RK_GLOAD(x, 0)
  RK_SSTORE(x)
  __syncthreads();
  for (int64_t ks = 0; ks < nk; ++ks) {
    if (ks + 1 < nk) RK_GLOAD(x, (ks + 1) * BK)
    mfma_step<BF>(As, Bs, lane, wm, wn, acc);
    __syncthreads();
    if (ks + 1 < nk) {
      RK_SSTORE(x)
      __syncthreads();
    }
  }
#undef RK_GLOAD
#undef RK_SSTORE

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = bm * kTile + wm * 64 + i * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r & 3);
        const int64_t col = bn * kTile + wn * 64 + j * 32 + (lane & 31);
        if (row < M && col < N) {
          float v = acc[i][j][r];
          if (row_scale) v *= row_scale[row];
          float* c = C + perm_row(row_perm, row, M) * ldc + col;
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
  L.Mp = round_up(std::max<int64_t>(1, A->M), kTile);
  L.Kp = round_up(std::max<int64_t>(1, A->K), kKAlign);
  L.Np = round_up(std::max<int64_t>(1, N), kTile);
  L.ad = 0;
  L.bt = (size_t)round_up((int64_t)(es * L.Mp * L.Kp), 256);
  L.bytes = L.bt + (size_t)round_up((int64_t)(es * L.Np * L.Kp), 256);
  return L;
}

template <bool BF>
int32_t run_dense(const rosko_packed* A, const void* B, int32_t b_dtype, int64_t N, int64_t ldb,
                  float* C, int64_t ldc, int32_t beta, void* ws, const DenseWs& L,
                  hipStream_t s) {
  using T = typename Op<BF>::T;
  T* Ad = reinterpret_cast<T*>(static_cast<char*>(ws) + L.ad);
  T* Bt = reinterpret_cast<T*>(static_cast<char*>(ws) + L.bt);
  const int64_t nkb = (A->K + ROSKO_KSTEP - 1) / ROSKO_KSTEP;
  const int64_t rec_bound = A->nrec >= 0 ? std::min(A->nrec, A->nrec_cap) : A->nrec_cap;
  if (A->mr <= kDenseLdsRows) {
    const dim3 dg((unsigned)A->n_panels, (unsigned)ceil_div(L.Kp, kDenseLdsK));
    hipLaunchKernelGGL(k_densify_lds<BF>, dg, dim3(256), 0, s, A->rec, A->kblk_ptr, nkb,
                       rec_bound, A->mr, A->n_panels, A->M, A->K, L.Mp, L.Kp, Ad);
  } else {
    const dim3 dg((unsigned)A->n_panels, (unsigned)ceil_div(L.Kp, kDensifyK));
    hipLaunchKernelGGL(k_densify<BF>, dg, dim3(256), 0, s, A->rec, A->kblk_ptr, nkb, rec_bound,
                       A->mr, A->n_panels, A->M, A->K, L.Mp, L.Kp, Ad);
  }
  ROSKO_LAUNCH_CHECK("k_densify");
  const dim3 tg((unsigned)(L.Np / kTrT), (unsigned)(L.Kp / kTrT));
  const int64_t bes = b_dtype == ROSKO_F32 ? 4 : 2;
  const bool vec = (reinterpret_cast<uintptr_t>(B) % 16 == 0) && ((ldb * bes) % 16 == 0);
#define RK_TR(TB_, V_)                                                                         \
  hipLaunchKernelGGL((k_transpose_b<TB_, BF, V_>), tg, dim3(256), 0, s, B, A->K, N, ldb, Bt, L.Kp)
  if (b_dtype == ROSKO_F32) {
    if (vec) RK_TR(ROSKO_F32, true);
    else RK_TR(ROSKO_F32, false);
  } else {
    if (vec) RK_TR(ROSKO_BF16, true);
    else RK_TR(ROSKO_BF16, false);
  }
#undef RK_TR
  ROSKO_LAUNCH_CHECK("k_transpose_b");
  const int64_t tm = L.Mp / kTile, tn = L.Np / kTile;
  const float* rs = A->val_dtype == ROSKO_FP8_E4M3 ? A->row_scale : nullptr;
  hipLaunchKernelGGL(k_dense_gemm<BF>, dim3((unsigned)(tm * tn)), dim3(256), 0, s, Ad, Bt, L.Kp,
                     A->M, N, tn, C, ldc, rs, A->row_perm, beta);
  ROSKO_LAUNCH_CHECK("k_dense_gemm");
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
  if (L.Mp / kTile * (L.Np / kTile) > INT32_MAX || L.Np / 32 > 65535 || L.Kp / 32 > 65535 ||
      A->n_panels > INT32_MAX) {
    set_error("dense path grid too large");
    return ROSKO_EUNSUPPORTED;
  }
  if (A->n_panels == 0) return launch_fill_zero(C, beta ? 0 : A->M, N, ldc, s);
  return bf ? run_dense<true>(A, B, b_dtype, N, ldb, C, ldc, beta, ws, L, s)
            : run_dense<false>(A, B, b_dtype, N, ldb, C, ldc, beta, ws, L, s);
}

}  // namespace rosko
