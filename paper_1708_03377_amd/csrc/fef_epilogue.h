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

// Split-precision epilogue: FP32 weights 1/(Delta_x + Delta_y) from the
// hardware reciprocal refined by one Newton step, r <- r (2 - d r) (error
// about half an ulp, symmetric), FP32 squares summed over the 4 elements of
// a tile, tile sums accumulated in FP64.  The column gaps gy may be stored in
// FP32 or FP64 (converted on load).
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
  double sum = 0.0;
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      float t = 0.0f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float d = dx[i][r] + dy[j];
        float w = __builtin_amdgcn_rcpf(d);
        w = fmaf(w, fmaf(-d, w, 1.0f), w);
        const float v = acc[i][j][r];
        t = fmaf(v * v, w, t);
      }
      sum += (double)t;
    }
  return sum;
}

}  // namespace fef
