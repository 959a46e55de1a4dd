// Epilogue shared by the pair kernels: orbital-energy denominators and the
// weighted squared sum of MFMA accumulator tiles.
#pragma once

#include "fef_internal.h"
#include "fef_device.h"

namespace fef {

// Delta_ia for a row/column index of a fragment's ov range.
__device__ inline double gap_of(const double* e, int nocc, int nvir, int idx) {
  const int i = idx / nvir;
  const int a = idx - i * nvir;
  return e[i] - e[nocc + a];
}

// Weighted sum of one lane's accumulator tiles.  Lane layout of a 16x16 MFMA
// result: column = lane % 16 and, for accumulator element r = 0..3,
//   row = 4 * (lane / 16) + r   (FP32 / BF16 / FP16 MFMA)
//   row = lane / 16 + 4 * r     (FP64 MFMA, kRowsInterleaved).
template <bool kRowsInterleaved, typename AccT>
__device__ inline double weighted_tiles(const AccT (&acc)[3][3], int r0, int c0, int lane,
                                        const FragInfo& fx, const FragInfo& fy,
                                        const double* ex, const double* ey, int32_t* flags,
                                        double scale) {
  const int li = lane & 15, lk = lane >> 4;
  double gx[3][4];
  bool vx[3][4];
  bool bad = false;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = r0 + 16 * i + (kRowsInterleaved ? lk + 4 * r : 4 * lk + r);
      vx[i][r] = row < fx.ov;
      gx[i][r] = vx[i][r] ? gap_of(ex, fx.nocc, fx.nvir, row) : -1.0;
      bad |= vx[i][r] && !(gx[i][r] < 0.0);
    }
  double gy[3];
  bool vy[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int col = c0 + 16 * j + li;
    vy[j] = col < fy.ov;
    gy[j] = vy[j] ? gap_of(ey, fy.nocc, fy.nvir, col) : -1.0;
    bad |= vy[j] && !(gy[j] < 0.0);
  }
  if (bad) atomicOr(flags, FEF_FLAG_GAP);
  double sum = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = (double)acc[i][j][r] * scale;
        const double t = (vx[i][r] && vy[j]) ? v * v / (gx[i][r] + gy[j]) : 0.0;
        sum += t;
      }
  return sum;
}

}  // namespace fef
