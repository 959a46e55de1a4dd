// Two-term split-precision pair contraction (BF16 or FP16 operands, FP32
// MFMA accumulation, FP64 weighting and sums).
//
// Each operand value x is split as x = hi + lo with hi = rn(x), lo = rn(x - hi)
// (rn = round to nearest even in the 16-bit format).  The product keeps the
// three leading terms
//     x y ~ hi_x hi_y + hi_x lo_y + lo_x hi_y
// and drops lo_x lo_y.  The three products are laid out as ONE contraction
// over a concatenated K axis of length 3 P0 (padded to a multiple of 32):
//     left  row ia: [ hi(W^x) | hi(W^x) | lo(W^x) ]
//     right row jb: [ hi(B^y) | lo(B^y) | hi(B^y) ]
// so a single 16x16x32 MFMA chain computes all three.  FP16 operands carry a
// per-fragment power-of-two scale that places each operand's largest value
// in [2^13, 2^14), keeping lo parts out of the subnormal range; the scales
// are undone exactly in FP64.
#include "fef_internal.h"
#include "fef_device.h"
#include "fef_epilogue.h"

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

// Per-fragment scales: hdr[2 f] = 1 / scale_left, hdr[2 f + 1] = 1 / scale_right.
template <bool kFp16>
__global__ __launch_bounds__(256) void split_scale_kernel(const FragInfo* __restrict__ frag,
                                                          int P0, const double* __restrict__ bov,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ hdr) {
  __shared__ double red[4];
  const FragInfo fi = frag[blockIdx.x];
  double mL = 0.0, mR = 0.0;
  const int64_t nL = (int64_t)P0 * fi.ov;
  for (int64_t e = threadIdx.x; e < nL; e += blockDim.x) {
    mL = fmax(mL, fabs(w[fi.off_w + e]));
    if (fi.cls == 0) mR = fmax(mR, fabs(bov[fi.off_bov + e]));
  }
  mL = block_max(mL, red);
  mR = block_max(mR, red);
  if (threadIdx.x == 0) {
    double sL = 1.0, sR = 1.0;
    if (kFp16) {
      int ex;
      if (mL > 0.0) { frexp(mL, &ex); sL = ldexp(1.0, 14 - ex); }
      if (mR > 0.0) { frexp(mR, &ex); sR = ldexp(1.0, 14 - ex); }
    }
    hdr[2 * blockIdx.x] = 1.0 / sL;
    hdr[2 * blockIdx.x + 1] = 1.0 / sR;
  }
}

// Writes the concatenated hi/lo operands, layout [ld][kc] (k contiguous).
template <bool kFp16>
__global__ __launch_bounds__(256) void split_pack_kernel(const FragInfo* __restrict__ frag,
                                                         int P0, int kc, int prec,
                                                         const double* __restrict__ bov,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ hdr,
                                                         char* __restrict__ ops) {
  const FragInfo fi = frag[blockIdx.x];
  const int tile = blockIdx.y;
  if (tile >= fi.ntile) return;
  const double sL = 1.0 / hdr[2 * blockIdx.x];
  const double sR = 1.0 / hdr[2 * blockIdx.x + 1];
  uint16_t* L = reinterpret_cast<uint16_t*>(ops + fi.off_L[prec]);
  uint16_t* R = fi.off_R[prec] >= 0 ? reinterpret_cast<uint16_t*>(ops + fi.off_R[prec]) : nullptr;
  const int nchunk = kc / 8;
  for (int e = threadIdx.x; e < kTile * nchunk; e += blockDim.x) {
    const int m = tile * kTile + e / nchunk;
    const int k0 = (e % nchunk) * 8;
    u16x8 vl, vr;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int kk = k0 + u;
      const int seg = kk / P0;
      const int k = kk - seg * P0;
      uint16_t l = 0, r = 0;
      if (m < fi.ov && seg < 3) {
        uint16_t hi, lo;
        split2<kFp16>(w[fi.off_w + (int64_t)k * fi.ov + m] * sL, hi, lo);
        l = (seg == 2) ? lo : hi;
        if (R) {
          split2<kFp16>(bov[fi.off_bov + (int64_t)k * fi.ov + m] * sR, hi, lo);
          r = (seg == 1) ? lo : hi;
        }
      }
      vl[u] = l;
      vr[u] = r;
    }
    *reinterpret_cast<u16x8*>(L + (int64_t)m * kc + k0) = vl;
    if (R) *reinterpret_cast<u16x8*>(R + (int64_t)m * kc + k0) = vr;
  }
}

hipError_t launch_pack_split(const fef_plan_s& p, const double* bov, const double* w, void* ops,
                             fef_prec prec, hipStream_t st) {
  char* o = static_cast<char*>(ops);
  double* hdr = reinterpret_cast<double*>(o);
  const int kc = p.geom[prec].kpad;
  int maxtile = 0;
  for (const auto& f : p.frag) maxtile = f.ntile > maxtile ? f.ntile : maxtile;
  if (maxtile == 0) return hipSuccess;
  if (prec == FEF_FP16X2) {
    hipLaunchKernelGGL(split_scale_kernel<true>, dim3(p.nfrag), dim3(256), 0, st, p.d_frag, p.P0,
                       bov, w, hdr);
    hipLaunchKernelGGL(split_pack_kernel<true>, dim3(p.nfrag, maxtile), dim3(256), 0, st,
                       p.d_frag, p.P0, kc, (int)prec, bov, w, hdr, o);
  } else if (prec == FEF_BF16X2) {
    hipLaunchKernelGGL(split_scale_kernel<false>, dim3(p.nfrag), dim3(256), 0, st, p.d_frag,
                       p.P0, bov, w, hdr);
    hipLaunchKernelGGL(split_pack_kernel<false>, dim3(p.nfrag, maxtile), dim3(256), 0, st,
                       p.d_frag, p.P0, kc, (int)prec, bov, w, hdr, o);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool kFp16>
__device__ inline f4 mma16(u16x8 a, u16x8 b, f4 c) {
  if (kFp16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Same decomposition as the plain kernel: 4 waves x (3x3) 16x16 tiles of V.
// A-operand lane layout of the 16x16x32 MFMA: row = lane % 16, k = 8 (lane /
// 16) .. +7; the B operand mirrors it with column = lane % 16.
template <bool kFp16>
__global__ __launch_bounds__(256) void pair_split_kernel(
    const FragInfo* __restrict__ frag, const PairInfo* __restrict__ pairs,
    const Item* __restrict__ items, const char* __restrict__ ops, int prec, int kc,
    const double* __restrict__ eps, double* __restrict__ partial, int32_t* __restrict__ flags) {
  __shared__ double red[4];
  const Item it = items[blockIdx.x];
  const PairInfo pr = pairs[it.pair];
  const FragInfo fx = frag[pr.x];
  const FragInfo fy = frag[pr.y];
  const double* hdr = reinterpret_cast<const double*>(ops);
  const double scale = hdr[2 * pr.x] * hdr[2 * pr.y + 1];
  const uint16_t* L = reinterpret_cast<const uint16_t*>(ops + fx.off_L[prec]);
  const uint16_t* R = reinterpret_cast<const uint16_t*>(ops + fy.off_R[prec]);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = it.mt * kTile + (wave >> 1) * 48;
  const int c0 = it.nt * kTile + (wave & 1) * 48;
  f4 acc[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[i][j] = f4{0, 0, 0, 0};
  for (int k = 0; k < kc; k += 32) {
    u16x8 a[3], b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
      a[i] = *reinterpret_cast<const u16x8*>(L + (int64_t)(r0 + 16 * i + li) * kc + k + 8 * lk);
#pragma unroll
    for (int j = 0; j < 3; ++j)
      b[j] = *reinterpret_cast<const u16x8*>(R + (int64_t)(c0 + 16 * j + li) * kc + k + 8 * lk);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) acc[i][j] = mma16<kFp16>(a[i], b[j], acc[i][j]);
  }
  const double sum = weighted_tiles<false>(acc, r0, c0, lane, fx, fy, eps + fx.off_eps,
                                       eps + fy.off_eps, flags, scale);
  const double total = block_sum(sum, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = 4.0 * pr.s * pr.s * total;
}

hipError_t launch_split_pairs(const fef_plan_s& p, const void* ops, const double* eps,
                              fef_prec prec, double* partial, int32_t* flags, hipStream_t st) {
  const char* o = static_cast<const char*>(ops);
  const int kc = p.geom[prec].kpad;
  if (prec == FEF_FP16X2)
    hipLaunchKernelGGL(pair_split_kernel<true>, dim3((unsigned)p.nitems), dim3(256), 0, st,
                       p.d_frag, p.d_pair, p.d_item, o, (int)prec, kc, eps, partial, flags);
  else if (prec == FEF_BF16X2)
    hipLaunchKernelGGL(pair_split_kernel<false>, dim3((unsigned)p.nitems), dim3(256), 0, st,
                       p.d_frag, p.d_pair, p.d_item, o, (int)prec, kc, eps, partial, flags);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace fef
