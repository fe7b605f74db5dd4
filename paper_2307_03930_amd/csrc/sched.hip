// Learned plan selection: packing statistics and a small MLP.
//
// The method tunes its tiling from an analytic model of the machine
// (Sec. 4.2) and exposes the tiling parameters for auto-tuning (Sec. 6).  Here the
// choice (panel height mr, register tile, sparse or dense-MFMA path) is made
// by a 3-layer MLP on 16 statistics of A that the packing count pass can
// see, trained on measured runtimes.  Everything the network does runs in
// these kernels: statistics, input normalisation, forward, the MSE gradient,
// backward, Adam and the arg-min; all reductions run in a fixed order, so
// results are reproducible.
//
// Statistics (rosko_features): one pass over A with the kept-value test of
// Alg. 1 counts kept values per row, per column and per 32-row panel, and
// the kept panel columns at 32 and 8 rows (integer atomics, exact); a
// single-workgroup pass turns them into the features with exact int64 sums
// (a coefficient of variation is sqrt(n*sum x^2 - (sum x)^2) / sum x).
#include <algorithm>

#include "internal.h"

namespace rosko {
namespace {

struct FeatWs {
  size_t rows, cols, panels, counters, bytes;
};
FeatWs feat_ws_layout(int64_t M, int64_t K) {
  FeatWs L{};
  const int64_t P = (M + 31) / 32;
  L.rows = 0;
  L.cols = L.rows + (size_t)round_up(4 * std::max<int64_t>(M, 1), 256);
  L.panels = L.cols + (size_t)round_up(4 * std::max<int64_t>(K, 1), 256);
  L.counters = L.panels + (size_t)round_up(4 * std::max<int64_t>(P, 1), 256);
  L.bytes = L.counters + 256;
  return L;
}

__global__ void __launch_bounds__(256) k_feat_zero(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0u;
}

// counters: [0] kept values, [1] kept panel columns (32 rows), [2] (8 rows)
__global__ void __launch_bounds__(256)
k_feat_count(const float* __restrict__ A, int64_t M, int64_t K, int64_t lda,
             uint32_t* __restrict__ rows, uint32_t* __restrict__ cols,
             uint32_t* __restrict__ panels, unsigned long long* __restrict__ counters) {
  __shared__ uint32_t srow[32];
  __shared__ uint32_t sc[3];
  const int t = threadIdx.x;
  const int64_t k = (int64_t)blockIdx.x * 256 + t;
  const int64_t r0 = (int64_t)blockIdx.y * 32;
  const int nrows = (int)std::min<int64_t>(32, M - r0);
  if (t < 32) srow[t] = 0;
  if (t < 3) sc[t] = 0;
  __syncthreads();
  if (k < K) {
    uint32_t g[4] = {0, 0, 0, 0};
    for (int i = 0; i < nrows; ++i) {
      const uint32_t bits = __float_as_uint(A[(r0 + i) * lda + k]);
      if (bits & 0x7FFFFFFFu) {
        ++g[i >> 3];
        atomicAdd(&srow[i], 1u);
      }
    }
    const uint32_t tot = g[0] + g[1] + g[2] + g[3];
    if (tot) {
      atomicAdd(&cols[k], tot);
      atomicAdd(&sc[0], tot);
      atomicAdd(&sc[1], 1u);
      atomicAdd(&sc[2], (uint32_t)(g[0] > 0) + (g[1] > 0) + (g[2] > 0) + (g[3] > 0));
    }
  }
  __syncthreads();
  if (t < nrows && srow[t]) atomicAdd(&rows[r0 + t], srow[t]);
  if (t == 0 && sc[0]) {
    atomicAdd(&panels[blockIdx.y], sc[0]);
    atomicAdd(&counters[0], (unsigned long long)sc[0]);
    atomicAdd(&counters[1], (unsigned long long)sc[1]);
    atomicAdd(&counters[2], (unsigned long long)sc[2]);
  }
}

// Block-wide sums of (x, x^2, [x == 0], max x) over an array of counts.
struct Moments {
  long long s, s2, zeros, mx;
};
__device__ Moments block_moments(const uint32_t* __restrict__ x, int64_t n, long long* red) {
  long long s = 0, s2 = 0, z = 0, mx = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const long long v = x[i];
    s += v;
    s2 += v * v;
    z += (v == 0);
    mx = v > mx ? v : mx;
  }
  const int t = threadIdx.x;
  red[t] = s; red[256 + t] = s2; red[512 + t] = z; red[768 + t] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      red[t] += red[t + w];
      red[256 + t] += red[256 + t + w];
      red[512 + t] += red[512 + t + w];
      red[768 + t] = red[768 + t] > red[768 + t + w] ? red[768 + t] : red[768 + t + w];
    }
    __syncthreads();
  }
  Moments m{red[0], red[256], red[512], red[768]};
  __syncthreads();
  return m;
}

__device__ float cv_of(const Moments& m, int64_t n) {
  if (m.s == 0 || n == 0) return 0.0f;
  const long long num = (long long)n * m.s2 - m.s * m.s;   // n^2 * variance, exact
  return sqrtf((float)num) / (float)m.s;
}

__global__ void __launch_bounds__(256)
k_feat_final(const uint32_t* __restrict__ rows, const uint32_t* __restrict__ cols,
             const uint32_t* __restrict__ panels, const unsigned long long* __restrict__ counters,
             int64_t M, int64_t K, int64_t N, float* __restrict__ f) {
  __shared__ long long red[1024];
  const int64_t P = (M + 31) / 32;
  const Moments mr = block_moments(rows, M, red);
  const Moments mc = block_moments(cols, K, red);
  const Moments mp = block_moments(panels, P, red);
  if (threadIdx.x != 0) return;
  const double nnz = (double)counters[0];
  const double c32 = (double)counters[1], c8 = (double)counters[2];
  const float d = (M * K) ? (float)(nnz / ((double)M * (double)K)) : 0.0f;
  f[0] = log2f((float)M);
  f[1] = log2f((float)K);
  f[2] = log2f((float)N);
  f[3] = d;
  f[4] = log10f(d + 1e-6f);
  f[5] = cv_of(mr, M);
  f[6] = M ? (float)mr.zeros / (float)M : 0.0f;
  f[7] = cv_of(mc, K);
  f[8] = K ? (float)mc.zeros / (float)K : 0.0f;
  f[9] = c32 > 0 ? (float)(nnz / c32) : 0.0f;
  f[10] = (P * K) ? (float)(c32 / ((double)P * (double)K)) : 0.0f;
  f[11] = c8 > 0 ? (float)(nnz / c8) : 0.0f;
  f[12] = cv_of(mp, P);
  f[13] = mp.s ? (float)((double)mp.mx * (double)P / (double)mp.s) : 0.0f;
  f[14] = log2f(1.0f + (float)(nnz * (double)N));
  f[15] = log2f((float)M * (float)N);
}

// ------------------------------------------------------------------ MLP
// Xn[b][i] = (X[b][i] - mu[i]) / sigma[i]
__global__ void __launch_bounds__(256)
k_normalize(const float* __restrict__ X, int64_t Bn, int32_t F, const float* __restrict__ mu,
            const float* __restrict__ sigma, float* __restrict__ Xn) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= Bn * F) return;
  const int i = (int)(id % F);
  Xn[id] = (X[id] - mu[i]) / sigma[i];
}

// Y[b][o] = sum_i X[b][i] W[i][o] + bias[o], ReLU when relu; one thread per
// output, i ascending.
__global__ void __launch_bounds__(256)
k_linear_fwd(const float* __restrict__ X, const float* __restrict__ W,
             const float* __restrict__ bias, int64_t Bn, int32_t I, int32_t O, int32_t relu,
             float* __restrict__ Y) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= Bn * O) return;
  const int64_t b = id / O;
  const int o = (int)(id % O);
  float acc = bias[o];
  for (int i = 0; i < I; ++i) acc = fmaf(X[b * I + i], W[(int64_t)i * O + o], acc);
  Y[id] = relu ? fmaxf(acc, 0.0f) : acc;
}

// dY = 2 (Y - T) mask / max(1, sum mask); loss = sum(mask (Y - T)^2) / max(1, sum mask).
// One workgroup; fixed-order reduction.
__global__ void __launch_bounds__(256)
k_mse(const float* __restrict__ Y, const float* __restrict__ T, const float* __restrict__ mask,
      int64_t n, float* __restrict__ dY, float* __restrict__ loss) {
  __shared__ float red[2][256];
  float s = 0.0f, c = 0.0f;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const float d = (Y[i] - T[i]) * mask[i];
    s = fmaf(d, d, s);
    c += mask[i];
  }
  red[0][threadIdx.x] = s;
  red[1][threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  const float cnt = fmaxf(1.0f, red[1][0]);
  for (int64_t i = threadIdx.x; i < n; i += 256) dY[i] = 2.0f * (Y[i] - T[i]) * mask[i] / cnt;
  if (threadIdx.x == 0) loss[0] = red[0][0] / cnt;
}

// dX[b][i] = (sum_o dY[b][o] W[i][o]) * [H[b][i] > 0]   (H = the ReLU output
// that fed the layer; its sign equals that of the pre-activation)
__global__ void __launch_bounds__(256)
k_linear_bwd_dx(const float* __restrict__ dY, const float* __restrict__ W,
                const float* __restrict__ H, int64_t Bn, int32_t I, int32_t O,
                float* __restrict__ dX) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= Bn * I) return;
  const int64_t b = id / I;
  const int i = (int)(id % I);
  float acc = 0.0f;
  for (int o = 0; o < O; ++o) acc = fmaf(dY[b * O + o], W[(int64_t)i * O + o], acc);
  dX[id] = H[id] > 0.0f ? acc : 0.0f;
}

// dW[i][o] = sum_b X[b][i] dY[b][o], db[o] = sum_b dY[b][o]; b ascending.
__global__ void __launch_bounds__(256)
k_linear_bwd_dw(const float* __restrict__ X, const float* __restrict__ dY, int64_t Bn, int32_t I,
                int32_t O, float* __restrict__ dW, float* __restrict__ db) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id < (int64_t)I * O) {
    const int i = (int)(id / O), o = (int)(id % O);
    float acc = 0.0f;
    for (int64_t b = 0; b < Bn; ++b) acc = fmaf(X[b * I + i], dY[b * O + o], acc);
    dW[id] = acc;
  } else if (id < (int64_t)I * O + O) {
    const int o = (int)(id - (int64_t)I * O);
    float acc = 0.0f;
    for (int64_t b = 0; b < Bn; ++b) acc += dY[b * O + o];
    db[o] = acc;
  }
}

// Adam with bias correction, step t >= 1.
__global__ void __launch_bounds__(256)
k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
       float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// out[b] = the first o with the smallest Y[b][o]
__global__ void __launch_bounds__(256)
k_argmin(const float* __restrict__ Y, int64_t Bn, int32_t C, int32_t* __restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= Bn) return;
  int best = 0;
  float bv = Y[b * C];
  for (int o = 1; o < C; ++o) {
    const float y = Y[b * C + o];
    if (y < bv) { bv = y; best = o; }
  }
  out[b] = best;
}

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, 256)); }

}  // namespace

size_t features_ws_bytes(int64_t M, int64_t K) { return feat_ws_layout(M, K).bytes; }

int32_t launch_features(const float* A, int64_t M, int64_t K, int64_t lda, int64_t N, void* ws,
                        float* f, hipStream_t s) {
  const FeatWs L = feat_ws_layout(M, K);
  char* w = static_cast<char*>(ws);
  uint32_t* rows = reinterpret_cast<uint32_t*>(w + L.rows);
  uint32_t* cols = reinterpret_cast<uint32_t*>(w + L.cols);
  uint32_t* panels = reinterpret_cast<uint32_t*>(w + L.panels);
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(w + L.counters);
  const int64_t words = (int64_t)(L.bytes / 4);
  hipLaunchKernelGGL(k_feat_zero, dim3((unsigned)std::min<int64_t>(grid_for(words), 4096)),
                     dim3(256), 0, s, reinterpret_cast<uint32_t*>(w), words);
  ROSKO_LAUNCH_CHECK("k_feat_zero");
  const int64_t P = (M + 31) / 32;
  if (M > 0 && K > 0) {
    if (P > 65535) {
      set_error("features: M = %lld too large", (long long)M);
      return ROSKO_EUNSUPPORTED;
    }
    hipLaunchKernelGGL(k_feat_count, dim3((unsigned)ceil_div(K, 256), (unsigned)P), dim3(256), 0,
                       s, A, M, K, lda, rows, cols, panels, cnt);
    ROSKO_LAUNCH_CHECK("k_feat_count");
  }
  hipLaunchKernelGGL(k_feat_final, dim3(1), dim3(256), 0, s, rows, cols, panels, cnt, M, K, N, f);
  ROSKO_LAUNCH_CHECK("k_feat_final");
  return ROSKO_OK;
}

int32_t launch_normalize(const float* X, int64_t Bn, int32_t F, const float* mu,
                         const float* sigma, float* Xn, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize, dim3(grid_for(Bn * F)), dim3(256), 0, s, X, Bn, F, mu, sigma, Xn);
  ROSKO_LAUNCH_CHECK("k_normalize");
  return ROSKO_OK;
}

// params: W1 [F,H], b1 [H], W2 [H,H], b2 [H], W3 [H,C], b3 [C]
int32_t launch_mlp_forward(const float* prm, int32_t F, int32_t H, int32_t C, const float* X,
                           int64_t Bn, float* H1, float* H2, float* Y, hipStream_t s) {
  const float* W1 = prm;
  const float* b1 = W1 + (int64_t)F * H;
  const float* W2 = b1 + H;
  const float* b2 = W2 + (int64_t)H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + (int64_t)H * C;
  hipLaunchKernelGGL(k_linear_fwd, dim3(grid_for(Bn * H)), dim3(256), 0, s, X, W1, b1, Bn, F, H, 1, H1);
  hipLaunchKernelGGL(k_linear_fwd, dim3(grid_for(Bn * H)), dim3(256), 0, s, H1, W2, b2, Bn, H, H, 1, H2);
  hipLaunchKernelGGL(k_linear_fwd, dim3(grid_for(Bn * C)), dim3(256), 0, s, H2, W3, b3, Bn, H, C, 0, Y);
  ROSKO_LAUNCH_CHECK("k_linear_fwd");
  return ROSKO_OK;
}

// ws: dY [Bn,C], dH2 [Bn,H], dH1 [Bn,H]
int32_t launch_mlp_backward(const float* prm, int32_t F, int32_t H, int32_t C, const float* X,
                            const float* H1, const float* H2, const float* Y, const float* T,
                            const float* mask, int64_t Bn, float* grads, float* ws, float* loss,
                            hipStream_t s) {
  const float* W2 = prm + (int64_t)F * H + H;
  const float* W3 = W2 + (int64_t)H * H + H;
  float* gW1 = grads;
  float* gb1 = gW1 + (int64_t)F * H;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (int64_t)H * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + (int64_t)H * C;
  float* dY = ws;
  float* dH2 = dY + Bn * C;
  float* dH1 = dH2 + Bn * H;
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, s, Y, T, mask, Bn * C, dY, loss);
  hipLaunchKernelGGL(k_linear_bwd_dw, dim3(grid_for((int64_t)H * C + C)), dim3(256), 0, s, H2, dY,
                     Bn, H, C, gW3, gb3);
  hipLaunchKernelGGL(k_linear_bwd_dx, dim3(grid_for(Bn * H)), dim3(256), 0, s, dY, W3, H2, Bn, H,
                     C, dH2);
  hipLaunchKernelGGL(k_linear_bwd_dw, dim3(grid_for((int64_t)H * H + H)), dim3(256), 0, s, H1, dH2,
                     Bn, H, H, gW2, gb2);
  hipLaunchKernelGGL(k_linear_bwd_dx, dim3(grid_for(Bn * H)), dim3(256), 0, s, dH2, W2, H1, Bn, H,
                     H, dH1);
  hipLaunchKernelGGL(k_linear_bwd_dw, dim3(grid_for((int64_t)F * H + H)), dim3(256), 0, s, X, dH1,
                     Bn, F, H, gW1, gb1);
  ROSKO_LAUNCH_CHECK("mlp backward");
  return ROSKO_OK;
}

int32_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                    float b2, float eps, int32_t t, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                     c1, c2);
  ROSKO_LAUNCH_CHECK("k_adam");
  return ROSKO_OK;
}

int32_t launch_argmin(const float* Y, int64_t Bn, int32_t C, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_argmin, dim3(grid_for(Bn)), dim3(256), 0, s, Y, Bn, C, out);
  ROSKO_LAUNCH_CHECK("k_argmin");
  return ROSKO_OK;
}

}  // namespace rosko
