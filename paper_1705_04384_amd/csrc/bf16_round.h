// Rounding to BF16, to nearest with ties to even, from FP32 and (in one rounding) from
// FP64, for the reduced-precision preconditioner passes and the factor copies.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace fdg {

// BF16 bits of an FP32 value; infinities and NaNs keep their class.
__host__ __device__ inline uint16_t bf16_bits_rne(uint32_t u) {
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// FP32 bits of an FP64 value rounded to odd: the value truncated toward zero, with the
// last bit set when anything was cut off.  FP32 keeps 16 significand bits more than BF16,
// so rounding this to nearest BF16 gives the nearest BF16 of the FP64 value itself
// (rounding to odd first makes the double rounding innocuous), where going through the
// nearest FP32 would not when that lands on a BF16 tie.
__host__ __device__ inline uint32_t fp32_bits_round_to_odd(double x) {
  const float f = (float)x;  // nearest
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  const double back = (double)f;
  if (back != x) {                          // inexact (NaN stays NaN)
    if (std::fabs(back) > std::fabs(x)) u -= 1u;  // it went away from zero: one step back
    u |= 1u;
  }
  return u;
}

__host__ __device__ inline uint16_t bf16_bits_from_f64(double x) { return bf16_bits_rne(fp32_bits_round_to_odd(x)); }

__host__ __device__ inline uint16_t bf16_bits_from_f32(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  return bf16_bits_rne(u);
}

__device__ inline __bf16 bf16_from_bits(uint16_t h) {
  __bf16 r;
  __builtin_memcpy(&r, &h, 2);
  return r;
}
// A mode-product input rounded to BF16 once, from its stored precision.  On the device the
// last step is the conversion instruction (gfx950 converts FP32 to BF16 rounding to
// nearest even, which is bf16_bits_rne); an FP64 input goes through the round-to-odd FP32
// value first, as above.
#ifdef FDG_BF16_SOFT_RNE
__device__ inline __bf16 to_bf16_once(float f) { return bf16_from_bits(bf16_bits_from_f32(f)); }
__device__ inline __bf16 to_bf16_once(double x) { return bf16_from_bits(bf16_bits_from_f64(x)); }
#else
__device__ inline __bf16 to_bf16_once(float f) { return (__bf16)f; }
__device__ inline __bf16 to_bf16_once(double x) {
  const uint32_t u = fp32_bits_round_to_odd(x);
  float f;
  __builtin_memcpy(&f, &u, 4);
  return (__bf16)f;
}
#endif
// An input already stored in BF16 (an intermediate rounded by the pass that wrote it).
__device__ inline __bf16 to_bf16_once(__bf16 h) { return h; }

}  // namespace fdg
