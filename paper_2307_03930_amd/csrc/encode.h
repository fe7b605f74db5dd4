// Value encodings of the packed form (the kept-entry test, BF16 and OCP
// FP8 E4M3 encoders, and the FP32 value of a stored code), shared by the
// dense and the CSR packers so both write the same bits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rosko {
namespace {

// Kept-entry test on the FP32 bits: every bit except the sign.
__device__ __forceinline__ int kept(float x) {
  return (__float_as_uint(x) & 0x7fffffffu) != 0u;
}

// BF16 round-to-nearest-even by integer carry; NaN -> 0x7FC0.
__device__ __forceinline__ uint16_t enc_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7FC0u;
  uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

// OCP E4M3FN, nearest-even, saturating at 448, NaN -> 0x7F.  Normal range
// rounds the FP32 mantissa to 3 bits with a carry into the exponent;
// magnitudes below 2^-6 are scaled by 2^9 (exact) and rounded to an integer
// number of subnormal steps with rintf (nearest-even).
__device__ __forceinline__ uint8_t enc_fp8(float y) {
  uint32_t u = __float_as_uint(y);
  uint32_t sign = (u >> 24) & 0x80u;
  uint32_t a = u & 0x7fffffffu;
  if (a > 0x7f800000u) return (uint8_t)0x7Fu;
  if (a >= 0x43E00000u) return (uint8_t)(sign | 0x7Eu);        // >= 448
  if (a >= 0x3C800000u) {                                       // >= 2^-6
    uint32_t e = (a >> 23) - 127u + 7u;                         // 1..8+7
    uint32_t m = (a >> 20) & 7u;
    uint32_t rest = a & 0xFFFFFu;
    uint32_t code = (e << 3) | m;
    if (rest > 0x80000u || (rest == 0x80000u && (m & 1u))) code += 1u;
    return (uint8_t)(sign | code);
  }
  float q = __uint_as_float(a) * 512.0f;                        // units of 2^-9
  uint32_t code = (uint32_t)rintf(q);                           // 0..8
  return (uint8_t)(sign | code);
}

// FP32 value of a packed value (FP8: the code's value, unscaled), as bits.
__device__ __forceinline__ uint32_t dec_bf16(uint16_t h) { return (uint32_t)h << 16; }
__device__ __forceinline__ uint32_t dec_fp8(uint8_t c) {
  const uint32_t e = (c >> 3) & 15u, m = c & 7u, s = (uint32_t)(c & 0x80u) << 24;
  if (e == 15 && m == 7) return 0x7FC00000u;
  if (e == 0) return s | __float_as_uint((float)m * 0.001953125f);     // m * 2^-9
  return s | ((e + 120u) << 23) | (m << 20);                            // (1+m/8) 2^(e-7)
}

}  // namespace
}  // namespace rosko
