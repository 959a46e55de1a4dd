// Epilogue shared by the pair kernels: orbital-energy denominators and the
// weighted squared sum of MFMA accumulator tiles.
#pragma once

#include "fef_internal.h"
#include "fef_device.h"

namespace fef {

// Weighted squared sums of MFMA accumulator tiles.  gx / gy point at the
// gap vectors Delta_ia = eps_i - eps_a of the tile's first row / column
// (fragment gap pools are padded with -1 where the operands are zero, so
// padded elements add 0).  Lane layout of a 16x16 MFMA result: column =
// lane % 16 and, for accumulator element r = 0..3,
//   row = 4 * (lane / 16) + r   (FP32 / BF16 / FP16 MFMA)
//   row = lane / 16 + 4 * r     (FP64 MFMA, kRowsInterleaved).

// FP64 weights and sums.
template <bool kRowsInterleaved, int TI, int TJ, typename AccT>
__device__ inline double weighted_tiles(const AccT (&acc)[TI][TJ], const double* gx,
                                        const double* gy, int lane, double scale) {
  const int li = lane & 15, lk = lane >> 4;
  double dx[TI][4], dy[TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) dx[i][r] = gx[16 * i + (kRowsInterleaved ? lk + 4 * r : 4 * lk + r)];
#pragma unroll
  for (int j = 0; j < TJ; ++j) dy[j] = gy[16 * j + li];
  double sum = 0.0;
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = (double)acc[i][j][r] * scale;
        sum += v * v / (dx[i][r] + dy[j]);
      }
  return sum;
}

// Split-precision epilogue.  The four elements r = 0..3 that a lane holds
// of one 16x16 tile share a column, and their weighted squares are summed as
// one fraction over the product of the four FP32 denominators:
//     sum_r v_r^2 / d_r = N / P,   P = (d0 d1)(d2 d3),
//     N = d2 d3 (v0^2 d1 + v1^2 d0) + d0 d1 (v2^2 d3 + v3^2 d2),
// so a tile costs one hardware reciprocal instead of four.  The quotient
// q = N r is corrected once, q + r (N - P q) (error about half an ulp,
// symmetric); the TI x TJ tile quotients of a call (terms of one sign) are
// summed in FP32 and the call's sum is returned for FP64 accumulation.  Magnitudes stay
// inside FP32: the FP16 operand scales bound |v| by 2^28 K, and |d| is an
// orbital-energy gap.  The column gaps gy may be stored in FP32 or FP64
// (converted on load).
template <int TI, int TJ>
__device__ inline double weighted_tiles_f32_regs(const f4 (&acc)[TI][TJ], const float (&dx)[TI][4],
                                                 const float (&dy)[TJ]) {
  float sum = 0.0f;
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const float d0 = dx[i][0] + dy[j], d1 = dx[i][1] + dy[j];
      const float d2 = dx[i][2] + dy[j], d3 = dx[i][3] + dy[j];
      const float v0 = acc[i][j][0], v1 = acc[i][j][1];
      const float v2 = acc[i][j][2], v3 = acc[i][j][3];
      const float n01 = fmaf(v0 * v0, d1, (v1 * v1) * d0);
      const float n23 = fmaf(v2 * v2, d3, (v3 * v3) * d2);
      const float a = d0 * d1, b = d2 * d3;
      const float num = fmaf(b, n01, a * n23);
      const float den = a * b;
      const float r = __builtin_amdgcn_rcpf(den);
      const float q = num * r;
      sum += fmaf(r, fmaf(-den, q, num), q);
    }
  return (double)sum;
}

// One tile of weighted_tiles_f32_regs: the same operations on one tile, its
// FP32 quotient returned (summing these in the order (i, j) from 0 gives
// the FP32 sum weighted_tiles_f32_regs forms).
__device__ inline float weighted_tile_f32(const f4& acc, const float (&dx)[4], float dy) {
  const float d0 = dx[0] + dy, d1 = dx[1] + dy;
  const float d2 = dx[2] + dy, d3 = dx[3] + dy;
  const float v0 = acc[0], v1 = acc[1];
  const float v2 = acc[2], v3 = acc[3];
  const float n01 = fmaf(v0 * v0, d1, (v1 * v1) * d0);
  const float n23 = fmaf(v2 * v2, d3, (v3 * v3) * d2);
  const float a = d0 * d1, b = d2 * d3;
  const float num = fmaf(b, n01, a * n23);
  const float den = a * b;
  const float r = __builtin_amdgcn_rcpf(den);
  const float q = num * r;
  return fmaf(r, fmaf(-den, q, num), q);
}

// The same with the row gaps gx and column gaps gy read from memory (gy in
// FP32 or FP64, converted on load).
template <int TI, int TJ, typename GyT>
__device__ inline double weighted_tiles_f32(const f4 (&acc)[TI][TJ], const float* gx,
                                            const GyT* gy, int lane) {
  const int li = lane & 15, lk = lane >> 4;
  float dx[TI][4], dy[TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) dx[i][r] = gx[16 * i + 4 * lk + r];
#pragma unroll
  for (int j = 0; j < TJ; ++j) dy[j] = (float)gy[16 * j + li];
  return weighted_tiles_f32_regs<TI, TJ>(acc, dx, dy);
}

}  // namespace fef
