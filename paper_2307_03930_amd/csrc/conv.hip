// Sparse direct convolution: a 3x3 convolution (stride 1, zero padding 1) of
// a channels-first input X (C_in x H x W) with a pruned weight, computed as
// the row-skipping product of the packed weight matrix A (C_out x 9 C_in,
// column k = c*9 + ky*3 + kx, the im2col order) and the input itself, without
// forming the im2col matrix (the outer-product method applied to direct
// convolution, Sec. 1).
//
// The output is computed on a padded-pitch grid: output (y, x) is column
// n = y*Wq + x, Wq >= W + 2.  Row k of the im2col matrix at column n is then
// element off(k) + n of the zero-padded input laid out flat (C_in planes of
// (H+2) x Wq, the image at rows 1..H and columns 1..W), off(k) = c*(H+2)*Wq +
// ky*Wq + kx: every row of the implicit B is a contiguous run of the flat
// input, shifted by its tap.  So the SpMM runs unchanged on a "B" whose row
// k starts at element off(k) of a flat array, one element between rows.  To
// keep its 4-wide vector loads aligned, the flat input is stored four times,
// copy r shifted left by r elements, and a column's record names the start
// r*T + off(k) - r in copy r = off(k) mod 4 (a multiple of 4).  Columns
// x >= W of the grid read across the row end and hold values of no meaning.
#include <algorithm>

#include "internal.h"

namespace rosko {

ConvGeom conv_geometry(int64_t C_in, int64_t H, int64_t W) {
  ConvGeom g{};
  g.Wq = W + 2;
  while ((H * g.Wq) % 4 != 0) ++g.Wq;      // N' = H * Wq a multiple of 4
  g.plane = (H + 2) * g.Wq;
  // a row start plus N' elements never passes C_in * plane + 2; slack of 8
  g.T = round_up(C_in * g.plane + 8, 4);
  g.N = H * g.Wq;
  return g;
}

namespace {

constexpr int kT = 256;

// Bc[r*T + e] = flat padded input at e + r (zero past its end), r = 0..3.
// A workgroup takes kConvRows consecutive padded rows (c, yy) of the flat
// input, its lanes over their kConvRows * Wq elements in order: element j
// goes to e = j - r of every copy r (e >= 0); workgroup 0 also zeroes each
// copy's tail past the flat input.  All offsets stay below 2^24 (the host
// checks 4T < 2^24), so 32-bit arithmetic is exact.
constexpr int kConvRows = 4;

__global__ void __launch_bounds__(kT)
k_conv_input(const float* __restrict__ X, int32_t C_in, int32_t H, int32_t W, int32_t Wq,
             int32_t T, float* __restrict__ Bc) {
  const int32_t rows = C_in * (H + 2);
  const int32_t row0 = blockIdx.x * kConvRows;
  const int32_t n = min(kConvRows, rows - row0) * Wq;
  for (int32_t li = threadIdx.x; li < n; li += kT) {
    const int32_t dr = li / Wq, xx = li - dr * Wq;
    const int32_t row = row0 + dr;                    // c * (H + 2) + yy
    const int32_t c = row / (H + 2), yy = row - c * (H + 2);
    const float v = (yy >= 1 && yy <= H && xx >= 1 && xx <= W)
                        ? X[((int64_t)c * H + (yy - 1)) * W + (xx - 1)] : 0.0f;
    const int32_t j = row0 * Wq + li;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (j >= r) Bc[r * T + j - r] = v;
  }
  if (blockIdx.x == 0) {
    const int32_t flat = rows * Wq;
    for (int32_t t = threadIdx.x; t < 4 * 16; t += kT) {
      const int32_t r = t / 16, e = flat - r + (t % 16);     // past the copied part
      if (e >= 0 && e < T) Bc[r * T + e] = 0.0f;
    }
  }
}

// The column records with each column index k replaced by its tap's start in
// the four shifted copies; everything else copied.
__global__ void __launch_bounds__(kT)
k_conv_records(const uint4* __restrict__ rec, int64_t nrec, int64_t K, int64_t Wq,
               int64_t plane, int64_t T, uint4* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (q >= nrec) return;
  uint4 h = rec[q * 4];
  const int64_t k = std::min<int64_t>(h.x >> 8, K - 1);
  const int64_t c = k / 9, t = k - c * 9, ky = t / 3, kx = t - ky * 3;
  const int64_t off = c * plane + ky * Wq + kx;
  const int64_t r = off & 3;
  h.x = (uint32_t)((r * T + off - r) << 8) | (h.x & 0xFFu);
  out[q * 4] = h;
  out[q * 4 + 1] = rec[q * 4 + 1];
  out[q * 4 + 2] = rec[q * 4 + 2];
  out[q * 4 + 3] = rec[q * 4 + 3];
}

// Y[o][y][x] = Yq[o][y*Wq + x], x < W.
__global__ void __launch_bounds__(kT)
k_conv_unpad(const float* __restrict__ Yq, int64_t ldy, int64_t C_out, int64_t H, int64_t W,
             int64_t Wq, float* __restrict__ Y) {
  const int64_t total = C_out * H * W;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kT) {
    const int64_t o = i / (H * W), rem = i - o * H * W, y = rem / W, x = rem - y * W;
    Y[i] = Yq[o * ldy + y * Wq + x];
  }
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kT), 65536));
}

}  // namespace

int32_t launch_conv_input(const float* X, int64_t C_in, int64_t H, int64_t W, float* Bc,
                          hipStream_t s) {
  const ConvGeom g = conv_geometry(C_in, H, W);
  hipLaunchKernelGGL(k_conv_input, dim3((unsigned)ceil_div(C_in * (H + 2), kConvRows)),
                     dim3(kT), 0, s, X, (int32_t)C_in, (int32_t)H, (int32_t)W, (int32_t)g.Wq,
                     (int32_t)g.T, Bc);
  ROSKO_LAUNCH_CHECK("k_conv_input");
  return ROSKO_OK;
}

int32_t launch_conv_records(const rosko_packed* A, int64_t nrec, int64_t C_in, int64_t H,
                            int64_t W, uint32_t* rec_out, hipStream_t s) {
  if (nrec == 0) return ROSKO_OK;
  const ConvGeom g = conv_geometry(C_in, H, W);
  hipLaunchKernelGGL(k_conv_records, dim3((unsigned)ceil_div(nrec, kT)), dim3(kT), 0, s,
                     reinterpret_cast<const uint4*>(A->rec), nrec, A->K, g.Wq, g.plane, g.T,
                     reinterpret_cast<uint4*>(rec_out));
  ROSKO_LAUNCH_CHECK("k_conv_records");
  return ROSKO_OK;
}

int32_t launch_conv_unpad(const float* Yq, int64_t ldy, int64_t C_out, int64_t H, int64_t W,
                          int64_t Wq, float* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_conv_unpad, dim3(grid_for(C_out * H * W)), dim3(kT), 0, s, Yq, ldy,
                     C_out, H, W, Wq, Y);
  ROSKO_LAUNCH_CHECK("k_conv_unpad");
  return ROSKO_OK;
}

}  // namespace rosko
