/*
 * rosko_oracle.c -- plain, slow CPU oracle for Rosko packing and SpMM.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP implementation; both sides only read
 * the same seeded inputs.
 *
 * Floating point is FP64 except where the method fixes FP32 (the FP8 row
 * scale and the value divided by it are FP32 quantities, computed here with
 * ordinary IEEE FP32 division, which C on x86-64 rounds correctly).
 *
 * What each routine follows:
 *   ro_pack*          Alg. 1 (Rosko packing), applied to every mr-row panel of
 *                     A with the panel's k range equal to all of K (Sec. 4.1).
 *   ro_spmm_csr       the plain definition of C = A*B restricted to the
 *                     nonzeros of A; row skipping (Sec. 3, Fig. 4) drops only
 *                     terms whose A factor is exactly zero, so this is the
 *                     exact result the packed outer products (Alg. 2) reach.
 *   ro_dense_mm       a second, dense route: all K terms, same k order.
 *   ro_spmm_packed    Alg. 2 executed literally on the oracle's own packed
 *                     arrays (the register tile is an FP64 array), with the
 *                     stored values decoded (FP32, BF16 or FP8 x row scale).
 *   ro_grad_dB        dB = A^T dC (the activation-gradient product of the
 *                     training decomposition, Sec. 5.4), over A's nonzeros.
 *   ro_grad_dA_packed dA = (dC B^T) restricted to A's nonzeros, emitted in
 *                     packed order (an SDDMM on A's mask).
 *   ro_conv3x3        direct 3x3 convolution (stride 1, zero padding 1) with
 *                     the weight matrix A (C_out x C_in*9, column c*9+ky*3+kx),
 *                     by its definition over A's nonzeros: the product the
 *                     method computes without forming im2col (Sec. 1).
 *
 * Readings of the paper taken here:
 *   - "A[k + mK] != 0" is tested on the bits: (bits & 0x7fffffff) != 0, so
 *     -0.0 counts as zero and NaN, Inf and subnormals are kept.
 *   - Order of the packed arrays: panels ascending, then k ascending, then m
 *     ascending within a column; empty columns are dropped.
 *   - loc is the row within the panel (0 .. rows_p-1), one byte.
 *   - The inner loop of Alg. 2 runs exactly nnz[k] times (exclusive bound).
 *   - M not a multiple of mr: the last panel simply has fewer rows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RO_F32 0
#define RO_BF16 1
#define RO_FP8 2

static uint32_t bits_of(float x) { uint32_t u; memcpy(&u, &x, 4); return u; }
static float float_of(uint32_t u) { float x; memcpy(&x, &u, 4); return x; }

/* A value is "nonzero" when any bit other than the sign is set. */
int ro_is_nonzero(float x) { return (bits_of(x) & 0x7fffffffu) != 0u; }

/* ---------------------------------------------------------------- BF16 --- */
/* Round an FP32 value to BF16, nearest with ties to even.  NaN becomes the
 * canonical quiet NaN 0x7FC0.  Computed by comparing the two candidate BF16
 * neighbours (truncation and truncation + 1 ulp) against the exact value in
 * FP64, which represents every FP32 and BF16 value exactly. */
uint16_t ro_bf16_encode(float x) {
  if (isnan(x)) return 0x7FC0u;
  uint32_t u = bits_of(x);
  uint32_t lo = u & 0xFFFF0000u;            /* toward zero */
  if (lo == u) return (uint16_t)(u >> 16);  /* already a BF16 value */
  uint32_t hi = lo + 0x00010000u;           /* away from zero (may be Inf) */
  double ax = fabs((double)x);
  double alo = fabs((double)float_of(lo));
  double ahi;
  if (((hi >> 23) & 0xFFu) == 0xFFu) {
    /* away-from-zero neighbour is Inf: treat it as 2^128 for rounding */
    ahi = ldexp(1.0, 128);
  } else {
    ahi = fabs((double)float_of(hi));
  }
  double dlo = ax - alo, dhi = ahi - ax;
  uint32_t pick;
  if (dlo < dhi) pick = lo;
  else if (dhi < dlo) pick = hi;
  else pick = (((lo >> 16) & 1u) == 0u) ? lo : hi;   /* tie: even mantissa */
  return (uint16_t)(pick >> 16);
}

float ro_bf16_decode(uint16_t h) { return float_of(((uint32_t)h) << 16); }

/* --------------------------------------------------------- FP8 E4M3FN --- */
/* OCP E4M3FN: 1 sign, 4 exponent (bias 7), 3 mantissa bits; no Inf; the
 * only NaN codes are S.1111.111; largest finite 448; subnormals m * 2^-9. */
double ro_fp8_decode_d(uint8_t c) {
  int s = (c >> 7) & 1, e = (c >> 3) & 15, m = c & 7;
  double v;
  if (e == 15 && m == 7) return NAN;
  if (e == 0) v = ldexp((double)m, -9);
  else v = ldexp(1.0 + m / 8.0, e - 7);
  return s ? -v : v;
}
float ro_fp8_decode(uint8_t c) { return (float)ro_fp8_decode_d(c); }

/* Encode y to E4M3FN: nearest representable value, ties to the even code,
 * magnitudes at or above 448 (and Inf) saturate to +-448, NaN -> 0x7F.
 * Done by brute force over the 127 non-negative finite codes: the code
 * table is monotone in the code, so the nearest code, and on a tie the one
 * with a zero last mantissa bit, is the rounding result by definition. */
uint8_t ro_fp8_encode(float y) {
  if (isnan(y)) return 0x7Fu;
  uint8_t sign = signbit(y) ? 0x80u : 0x00u;
  double a = fabs((double)y);
  if (a >= 448.0) return (uint8_t)(sign | 0x7Eu);
  int best = 0;
  double bestd = INFINITY;
  for (int c = 0; c <= 0x7E; ++c) {
    double d = fabs(ro_fp8_decode_d((uint8_t)c) - a);
    if (d < bestd) { bestd = d; best = c; }
    else if (d == bestd && (c & 1) == 0) { best = c; }
  }
  return (uint8_t)(sign | (uint8_t)best);
}

/* Per-row scale for FP8 storage: s_m = absmax_k |A[m][k]| / 448 in FP32,
 * 1.0 for a row with no nonzero magnitude.  NaN entries are ignored by the
 * max; an Inf entry gives an Inf scale. */
void ro_row_scale(const float *A, int64_t M, int64_t K, int64_t lda, float *scale) {
  for (int64_t m = 0; m < M; ++m) {
    float amax = 0.0f;
    for (int64_t k = 0; k < K; ++k) {
      float v = fabsf(A[m * lda + k]);
      if (v > amax) amax = v;              /* false for NaN */
    }
    volatile float num = amax, den = 448.0f; /* keep it an FP32 division */
    scale[m] = (amax == 0.0f) ? 1.0f : num / den;
  }
}

/* ------------------------------------------------------------- packing --- */
/* Counts only: total stored nonzeros and nonempty panel columns. */
int64_t ro_pack_count(const float *A, int64_t M, int64_t K, int64_t lda, int32_t mr,
                      int64_t *ncols_out) {
  int64_t nnz = 0, ncols = 0;
  int64_t P = (M + mr - 1) / mr;
  for (int64_t p = 0; p < P; ++p) {
    int64_t r0 = p * mr, rows = (M - r0 < mr) ? (M - r0) : mr;
    for (int64_t k = 0; k < K; ++k) {
      int64_t cols = 0;
      for (int64_t m = 0; m < rows; ++m)
        if (ro_is_nonzero(A[(r0 + m) * lda + k])) ++cols;
      nnz += cols;
      if (cols != 0) ++ncols;
    }
  }
  *ncols_out = ncols;
  return nnz;
}

/* Alg. 1 on each mr-row panel.  Arrays are caller-allocated:
 *   panel_nz_ptr[P+1], panel_col_ptr[P+1]  (int64 running offsets)
 *   col_ind[ncols], col_nnz[ncols]          (int32)
 *   col_ptr[ncols+1]                        (int64 offset of each column's
 *                                            first value; col_ptr[ncols]=nnz)
 *   loc[nnz] (uint8), val[nnz] (4, 2 or 1 bytes per value by dtype)
 *   row_scale[M] (FP8 only; may be NULL otherwise)
 * The structure (which entries are stored) always comes from the FP32 bits;
 * the value encoding only changes what is written to val. */
void ro_pack(const float *A, int64_t M, int64_t K, int64_t lda, int32_t mr, int32_t dtype,
             int64_t *panel_nz_ptr, int64_t *panel_col_ptr, int32_t *col_ind, int32_t *col_nnz,
             int64_t *col_ptr, uint8_t *loc, void *val, float *row_scale) {
  int64_t P = (M + mr - 1) / mr;
  if (dtype == RO_FP8) ro_row_scale(A, M, K, lda, row_scale);
  int64_t i1 = 0, i2 = 0;                 /* running value / column slots */
  for (int64_t p = 0; p < P; ++p) {
    int64_t r0 = p * mr, rows = (M - r0 < mr) ? (M - r0) : mr;
    panel_nz_ptr[p] = i1;
    panel_col_ptr[p] = i2;
    for (int64_t k = 0; k < K; ++k) {     /* outer loop of Alg. 1: columns */
      int64_t cols = 0;
      int64_t first = i1;
      for (int64_t m = 0; m < rows; ++m) {  /* inner loop: rows, ascending */
        float x = A[(r0 + m) * lda + k];
        if (ro_is_nonzero(x)) {
          if (dtype == RO_F32) {
            ((float *)val)[i1] = x;
          } else if (dtype == RO_BF16) {
            ((uint16_t *)val)[i1] = ro_bf16_encode(x);
          } else {
            volatile float num = x, den = row_scale[r0 + m];
            ((uint8_t *)val)[i1] = ro_fp8_encode(num / den);
          }
          loc[i1] = (uint8_t)m;
          ++i1;
          ++cols;
        }
      }
      if (cols != 0) {                    /* keep only nonempty columns */
        col_ind[i2] = (int32_t)k;
        col_nnz[i2] = (int32_t)cols;
        col_ptr[i2] = first;
        ++i2;
      }
    }
  }
  panel_nz_ptr[P] = i1;
  panel_col_ptr[P] = i2;
  col_ptr[i2] = i1;
}

/* Decoded value of packed entry z as FP32 bits (FP8: the code's value,
 * without the row scale). */
static uint32_t decoded_bits(int32_t dtype, const void *val, int64_t z) {
  float f;
  if (dtype == RO_F32) f = ((const float *)val)[z];
  else if (dtype == RO_BF16) f = ro_bf16_decode(((const uint16_t *)val)[z]);
  else {
    uint8_t c = ((const uint8_t *)val)[z];
    if (((c >> 3) & 15) == 15 && (c & 7) == 7) return 0x7FC00000u;
    f = (float)ro_fp8_decode_d(c);
  }
  return bits_of(f);
}

/* Column records: the GPU execution copy of the packed panels.  Every kept
 * column becomes ceil(nnz/12) records of 16 dwords, in packed order:
 *   dword 0      (k << 8) | count (count 1..12 values in this record)
 *   dwords 1..3  the in-panel rows of the record's values, one byte each,
 *                value t in byte t%4 of dword 1 + t/4 (unused bytes 0)
 *   dwords 4..15 the values as FP32 bits (decoded; unused slots 0)
 * rec_kblk[p*(nkb+1) + j] is the first record of panel p whose column has
 * k >= j*kstep (the panel's end if none), for j = 0..nkb, nkb = ceil(K/kstep).
 * Returns the number of records. */
int64_t ro_records(int64_t M, int64_t K, int32_t mr, int32_t dtype, int32_t kstep,
                   const int64_t *panel_col_ptr, const int32_t *col_ind, const int32_t *col_nnz,
                   const int64_t *col_ptr, const uint8_t *loc, const void *val,
                   uint32_t *rec, int64_t *rec_kblk) {
  int64_t P = (M + mr - 1) / mr;
  int64_t nkb = (K + kstep - 1) / kstep;
  int64_t r = 0;
  for (int64_t p = 0; p < P; ++p) {
    int64_t j = 0;
    for (int64_t c = panel_col_ptr[p]; c < panel_col_ptr[p + 1]; ++c) {
      while (j <= nkb && j * kstep <= col_ind[c]) {
        if (rec_kblk) rec_kblk[p * (nkb + 1) + j] = r;
        ++j;
      }
      for (int64_t first = 0; first < col_nnz[c]; first += 12) {
        int64_t cnt = col_nnz[c] - first < 12 ? col_nnz[c] - first : 12;
        if (rec) {
          uint32_t *d = rec + r * 16;
          for (int q = 0; q < 16; ++q) d[q] = 0u;
          d[0] = ((uint32_t)col_ind[c] << 8) | (uint32_t)cnt;
          for (int64_t t = 0; t < cnt; ++t) {
            int64_t z = col_ptr[c] + first + t;
            d[1 + t / 4] |= (uint32_t)loc[z] << (8 * (t % 4));
            d[4 + t] = decoded_bits(dtype, val, z);
          }
        }
        ++r;
      }
    }
    while (j <= nkb) {
      if (rec_kblk) rec_kblk[p * (nkb + 1) + j] = r;
      ++j;
    }
  }
  return r;
}

/* Decoded value of packed entry z as a double. */
static double packed_value(int32_t dtype, const void *val, const float *row_scale,
                           int64_t row, int64_t z) {
  if (dtype == RO_F32) return (double)((const float *)val)[z];
  if (dtype == RO_BF16) return (double)ro_bf16_decode(((const uint16_t *)val)[z]);
  return ro_fp8_decode_d(((const uint8_t *)val)[z]) * (double)row_scale[row];
}

/* Dense M x K array rebuilt from the packed arrays (decoded values, FP64). */
void ro_unpack(int64_t M, int64_t K, int32_t mr, int32_t dtype,
               const int64_t *panel_col_ptr, const int32_t *col_ind, const int32_t *col_nnz,
               const int64_t *col_ptr, const uint8_t *loc, const void *val,
               const float *row_scale, double *Aout) {
  int64_t P = (M + mr - 1) / mr;
  for (int64_t i = 0; i < M * K; ++i) Aout[i] = 0.0;
  for (int64_t p = 0; p < P; ++p) {
    for (int64_t c = panel_col_ptr[p]; c < panel_col_ptr[p + 1]; ++c) {
      for (int64_t j = 0; j < col_nnz[c]; ++j) {
        int64_t z = col_ptr[c] + j;
        int64_t row = p * mr + loc[z];
        Aout[row * K + col_ind[c]] = packed_value(dtype, val, row_scale, row, z);
      }
    }
  }
}

/* ---------------------------------------------------------------- SpMM --- */
/* C[m][n] = sum over k with A[m][k] nonzero, ascending k, of A[m][k]*B[k][n],
 * accumulated in FP64 from 0.  B is FP32 (ldb), C is FP64 M x N dense. */
void ro_spmm_csr(const float *A, int64_t M, int64_t K, int64_t lda,
                 const float *B, int64_t N, int64_t ldb, double *C) {
  int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)(K > 0 ? K : 1));
  for (int64_t m = 0; m < M; ++m) {
    /* the CSR row of m: column indices of its nonzeros, ascending */
    int64_t cnt = 0;
    for (int64_t k = 0; k < K; ++k)
      if (ro_is_nonzero(A[m * lda + k])) cols[cnt++] = k;
    double *crow = C + m * N;
    for (int64_t n = 0; n < N; ++n) crow[n] = 0.0;
    for (int64_t j = 0; j < cnt; ++j) {
      double a = (double)A[m * lda + cols[j]];
      const float *brow = B + cols[j] * ldb;
      for (int64_t n = 0; n < N; ++n) crow[n] += a * (double)brow[n];
    }
  }
  free(cols);
}

/* Same product with every one of the K terms included (zeros too). */
void ro_dense_mm(const float *A, int64_t M, int64_t K, int64_t lda,
                 const float *B, int64_t N, int64_t ldb, double *C) {
  for (int64_t m = 0; m < M; ++m) {
    for (int64_t n = 0; n < N; ++n) {
      double acc = 0.0;
      for (int64_t k = 0; k < K; ++k) acc += (double)A[m * lda + k] * (double)B[k * ldb + n];
      C[m * N + n] = acc;
    }
  }
}

/* Sum over A's nonzeros of |A[m][k]|*|B[k][n]|: the scale of the
 * componentwise rounding-error bound, used as the error denominator. */
void ro_abs_product(const float *A, int64_t M, int64_t K, int64_t lda,
                    const float *B, int64_t N, int64_t ldb, double *C) {
  for (int64_t m = 0; m < M; ++m) {
    double *crow = C + m * N;
    for (int64_t n = 0; n < N; ++n) crow[n] = 0.0;
    for (int64_t k = 0; k < K; ++k) {
      float x = A[m * lda + k];
      if (!ro_is_nonzero(x)) continue;
      double a = fabs((double)x);
      const float *brow = B + k * ldb;
      for (int64_t n = 0; n < N; ++n) crow[n] += a * fabs((double)brow[n]);
    }
  }
}

/* Alg. 2 run literally over every panel of the oracle's packed arrays: load
 * the panel's C rows (here: zeros, or the given C_in when beta is 1), then
 * for each nonempty column load B[col_ind] and, for each of its nnz values,
 * multiply-accumulate into row loc of the panel tile; finally store. */
void ro_spmm_packed(int64_t M, int64_t K, int32_t mr, int32_t dtype,
                    const int64_t *panel_col_ptr, const int32_t *col_ind, const int32_t *col_nnz,
                    const int64_t *col_ptr, const uint8_t *loc, const void *val,
                    const float *row_scale, const float *B, int64_t N, int64_t ldb,
                    const double *C_in, int beta, double *C) {
  (void)K;
  int64_t P = (M + mr - 1) / mr;
  double *tile = (double *)malloc(sizeof(double) * (size_t)mr * (size_t)(N > 0 ? N : 1));
  for (int64_t p = 0; p < P; ++p) {
    int64_t r0 = p * mr, rows = (M - r0 < mr) ? (M - r0) : mr;
    for (int64_t m = 0; m < rows; ++m)
      for (int64_t n = 0; n < N; ++n)
        tile[m * N + n] = beta ? C_in[(r0 + m) * N + n] : 0.0;
    for (int64_t c = panel_col_ptr[p]; c < panel_col_ptr[p + 1]; ++c) {
      const float *b = B + (int64_t)col_ind[c] * ldb;
      int64_t z = col_ptr[c];
      for (int64_t j = 0; j < col_nnz[c]; ++j, ++z) {
        double a = packed_value(dtype, val, row_scale, r0 + loc[z], z);
        double *crow = tile + (int64_t)loc[z] * N;
        for (int64_t n = 0; n < N; ++n) crow[n] += a * (double)b[n];
      }
    }
    for (int64_t m = 0; m < rows; ++m)
      for (int64_t n = 0; n < N; ++n) C[(r0 + m) * N + n] = tile[m * N + n];
  }
  free(tile);
}

/* ------------------------------------------------------------ backward --- */
/* dB[k][n] = sum over m with A[m][k] nonzero, ascending m, of A[m][k]*dC[m][n]. */
void ro_grad_dB(const float *A, int64_t M, int64_t K, int64_t lda,
                const float *dC, int64_t N, int64_t lddc, double *dB) {
  for (int64_t k = 0; k < K; ++k) {
    double *row = dB + k * N;
    for (int64_t n = 0; n < N; ++n) row[n] = 0.0;
    for (int64_t m = 0; m < M; ++m) {
      float x = A[m * lda + k];
      if (!ro_is_nonzero(x)) continue;
      double a = (double)x;
      const float *g = dC + m * lddc;
      for (int64_t n = 0; n < N; ++n) row[n] += a * (double)g[n];
    }
  }
}

/* dA at every stored entry, in packed order: for entry (m, k),
 * sum over n ascending of dC[m][n]*B[k][n]. */
void ro_grad_dA_packed(int64_t M, int32_t mr, const int64_t *panel_col_ptr,
                       const int32_t *col_ind, const int32_t *col_nnz, const int64_t *col_ptr,
                       const uint8_t *loc, const float *dC, int64_t lddc,
                       const float *B, int64_t ldb, int64_t N, double *dA) {
  int64_t P = (M + mr - 1) / mr;
  for (int64_t p = 0; p < P; ++p) {
    for (int64_t c = panel_col_ptr[p]; c < panel_col_ptr[p + 1]; ++c) {
      const float *b = B + (int64_t)col_ind[c] * ldb;
      for (int64_t j = 0; j < col_nnz[c]; ++j) {
        int64_t z = col_ptr[c] + j;
        const float *g = dC + (p * mr + loc[z]) * lddc;
        double acc = 0.0;
        for (int64_t n = 0; n < N; ++n) acc += (double)g[n] * (double)b[n];
        dA[z] = acc;
      }
    }
  }
}

/* Row-parallel variant of ro_spmm_csr used only to time the oracle on
 * several host cores; each row is computed exactly as above. */
#ifdef _OPENMP
#include <omp.h>
#endif
void ro_spmm_csr_par(const float *A, int64_t M, int64_t K, int64_t lda,
                     const float *B, int64_t N, int64_t ldb, double *C, int32_t threads) {
#ifdef _OPENMP
  #pragma omp parallel for num_threads(threads) schedule(dynamic, 4)
#endif
  for (int64_t m = 0; m < M; ++m)
    ro_spmm_csr(A + m * lda, 1, K, lda, B, N, ldb, C + m * N);
  (void)threads;
}

/* Row-parallel variant of ro_abs_product (same per-row arithmetic). */
void ro_abs_product_par(const float *A, int64_t M, int64_t K, int64_t lda,
                        const float *B, int64_t N, int64_t ldb, double *C, int32_t threads) {
#ifdef _OPENMP
  #pragma omp parallel for num_threads(threads) schedule(dynamic, 4)
#endif
  for (int64_t m = 0; m < M; ++m)
    ro_abs_product(A + m * lda, 1, K, lda, B, N, ldb, C + m * N);
  (void)threads;
}

/* Parallel variant of ro_grad_dB: each thread owns whole rows k of dB, each
 * computed exactly as in ro_grad_dB (ascending m). */
void ro_grad_dB_par(const float *A, int64_t M, int64_t K, int64_t lda,
                    const float *dC, int64_t N, int64_t lddc, double *dB, int32_t threads) {
#ifdef _OPENMP
  #pragma omp parallel for num_threads(threads) schedule(dynamic, 16)
#endif
  for (int64_t k = 0; k < K; ++k) {
    double *row = dB + k * N;
    for (int64_t n = 0; n < N; ++n) row[n] = 0.0;
    for (int64_t m = 0; m < M; ++m) {
      float x = A[m * lda + k];
      if (!ro_is_nonzero(x)) continue;
      double a = (double)x;
      const float *g = dC + m * lddc;
      for (int64_t n = 0; n < N; ++n) row[n] += a * (double)g[n];
    }
  }
  (void)threads;
}

/* Panel-parallel variant of ro_grad_dA_packed (same per-entry sums). */
void ro_grad_dA_packed_par(int64_t M, int32_t mr, const int64_t *panel_col_ptr,
                           const int32_t *col_ind, const int32_t *col_nnz, const int64_t *col_ptr,
                           const uint8_t *loc, const float *dC, int64_t lddc,
                           const float *B, int64_t ldb, int64_t N, double *dA, int32_t threads) {
  int64_t P = (M + mr - 1) / mr;
#ifdef _OPENMP
  #pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
#endif
  for (int64_t p = 0; p < P; ++p) {
    for (int64_t c = panel_col_ptr[p]; c < panel_col_ptr[p + 1]; ++c) {
      const float *b = B + (int64_t)col_ind[c] * ldb;
      for (int64_t j = 0; j < col_nnz[c]; ++j) {
        int64_t z = col_ptr[c] + j;
        const float *g = dC + (p * mr + loc[z]) * lddc;
        double acc = 0.0;
        for (int64_t n = 0; n < N; ++n) acc += (double)g[n] * (double)b[n];
        dA[z] = acc;
      }
    }
  }
  (void)threads;
}

/* out[o][y][x] = sum over kept A[o][c*9 + ky*3 + kx] of that weight times
 * X[c][y+ky-1][x+kx-1] (zero outside the C_in x H x W input); with
 * absolute != 0 the same sum of |weight| * |input| (the error scale).  FP64,
 * weights in ascending column order; rows o split over the threads. */
void ro_conv3x3(const float *A, int64_t C_out, int64_t C_in, int64_t H, int64_t W,
                const float *X, double *out, int32_t absolute, int32_t threads) {
  const int64_t K = C_in * 9;
#ifdef _OPENMP
  #pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
#endif
  for (int64_t o = 0; o < C_out; ++o) {
    double *y_o = out + o * H * W;
    for (int64_t i = 0; i < H * W; ++i) y_o[i] = 0.0;
    for (int64_t k = 0; k < K; ++k) {
      float wv = A[o * K + k];
      if (!ro_is_nonzero(wv)) continue;
      double w = absolute ? fabs((double)wv) : (double)wv;
      int64_t c = k / 9, ky = (k % 9) / 3, kx = k % 3;
      const float *xc = X + c * H * W;
      for (int64_t y = 0; y < H; ++y) {
        int64_t yy = y + ky - 1;
        if (yy < 0 || yy >= H) continue;
        for (int64_t x = 0; x < W; ++x) {
          int64_t xx = x + kx - 1;
          if (xx < 0 || xx >= W) continue;
          double v = (double)xc[yy * W + xx];
          y_o[y * W + x] += w * (absolute ? fabs(v) : v);
        }
      }
    }
  }
  (void)threads;
}

int32_t ro_max_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}
