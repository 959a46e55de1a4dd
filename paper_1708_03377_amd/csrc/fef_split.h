// Two-term operand splitting shared by the split-precision packers.
#pragma once

#include "fef_device.h"

namespace fef {

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline double bf16_to_double(uint16_t h) {
  return (double)__uint_as_float(((uint32_t)h) << 16);
}
__device__ inline uint16_t f16_rne(float f) {
  _Float16 h = (_Float16)f;
  return __builtin_bit_cast(uint16_t, h);
}
__device__ inline double f16_to_double(uint16_t h) {
  return (double)__builtin_bit_cast(_Float16, h);
}

template <bool kFp16>
__device__ inline void split2(double x, uint16_t& hi, uint16_t& lo) {
  if (kFp16) {
    hi = f16_rne((float)x);
    lo = f16_rne((float)(x - f16_to_double(hi)));
  } else {
    hi = bf16_rne((float)x);
    lo = bf16_rne((float)(x - bf16_to_double(hi)));
  }
}

// Power-of-two scale placing the largest magnitude m in [2^13, 2^14), so the
// FP16 lo parts of all but the smallest values stay normal.
__device__ inline double split_scale(double m) {
  if (!(m > 0.0)) return 1.0;
  int ex;
  frexp(m, &ex);
  return ldexp(1.0, 14 - ex);
}

}  // namespace fef
