// Multi-term operand splitting shared by the split-precision packers.
#pragma once

#include "fef_internal.h"
#include "fef_device.h"

namespace fef {

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline uint16_t f16_rne(float f) {
  _Float16 h = (_Float16)f;
  return __builtin_bit_cast(uint16_t, h);
}

// x = hi + lo with hi = rn(x) and lo = rn(x - hi) in the 16-bit format.
// FP16: formed in FP32 (hi + lo carries 22 significant bits, fewer than
// FP32's 24, and xf - hi is exact in FP32 since hi is the 16-bit rounding of
// xf), one FP64 -> FP32 conversion per value.  Measured on the water box this
// lowers the bias of the representation error and the FP16x2 total error
// (7.1e-7 -> 6.6e-7 Eh).  BF16: the residual x - hi is taken in FP64 before
// its rounding; the FP32 form raised the bias of BF16's 16-bit split.
template <bool kFp16>
__device__ inline void split2(double x, uint16_t& hi, uint16_t& lo) {
  if (kFp16) {
    const float xf = (float)x;
    const _Float16 h = (_Float16)xf;
    hi = __builtin_bit_cast(uint16_t, h);
    lo = f16_rne(xf - (float)h);
  } else {
    hi = bf16_rne((float)x);
    lo = bf16_rne((float)(x - (double)__uint_as_float(((uint32_t)hi) << 16)));
  }
}

// x = t0 + t1 + ... in the 16-bit format of mode PREC: FP16X2 and BF16X2 as
// split2, BF16X3 as three BF16 terms t_k = rn(x - t_0 - ... - t_{k-1}) with
// the residuals taken in FP64.
template <int PREC, int NTERM>
__device__ inline void split_terms(double x, uint16_t (&t)[NTERM]) {
  if constexpr (NTERM == 2) {
    split2<PREC == FEF_FP16X2>(x, t[0], t[1]);
  } else {
    double r = x;
#pragma unroll
    for (int k = 0; k < NTERM; ++k) {
      t[k] = bf16_rne((float)r);
      r -= (double)__uint_as_float(((uint32_t)t[k]) << 16);
    }
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
