// Pair contraction on MFMA and the denominator-weighted squared sum.
//
// For a pair (x, y) (y in class 0):
//   V[ia][jb] = s_xy sum_Q W^x[Q][ia] B_ov^y[Q][jb]        ( = (ia|jb) )
//   E2_xy     = 4 sum_{ia,jb} V^2 / (Delta^x_ia + Delta^y_jb),
//   Delta_ia  = eps_i - eps_a
// (dimer second-order energy with first-order dimer doubles, canonical
// orbitals).  V is produced tile by tile in MFMA accumulators and reduced in
// registers; it is never written to memory.
#include "fef_internal.h"
#include "fef_device.h"
#include "fef_epilogue.h"

namespace fef {

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4 acc_t;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef f4 acc_t;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// One work item = one 96x96 tile of V.  Four waves, each a 48x48 quadrant
// (3x3 MFMA tiles).  Operands are read straight from the operand pool.
template <typename T>
__global__ __launch_bounds__(256) void pair_plain_kernel(
    const FragInfo* __restrict__ frag, const PairInfo* __restrict__ pairs,
    const Item* __restrict__ items, const char* __restrict__ ops, int prec, int kpad,
    const double* __restrict__ eps, double* __restrict__ partial, int32_t* __restrict__ flags) {
  __shared__ double red[4];
  typedef typename Mfma<T>::acc_t acc_t;
  const Item it = items[blockIdx.x];
  const PairInfo pr = pairs[it.pair];
  const FragInfo fx = frag[pr.x];
  const FragInfo fy = frag[pr.y];
  const T* L = reinterpret_cast<const T*>(ops + fx.off_L[prec]);
  const T* R = reinterpret_cast<const T*>(ops + fy.off_R[prec]);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = it.mt * kTile + (wave >> 1) * 48;
  const int c0 = it.nt * kTile + (wave & 1) * 48;
  acc_t acc[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  for (int k = 0; k < kpad; k += 4) {
    const T* Lk = L + (int64_t)(k + lk) * fx.ld + r0 + li;
    const T* Rk = R + (int64_t)(k + lk) * fy.ld + c0 + li;
    T a[3], b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) a[i] = Lk[16 * i];
#pragma unroll
    for (int j = 0; j < 3; ++j) b[j] = Rk[16 * j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) acc[i][j] = Mfma<T>::mma(a[i], b[j], acc[i][j]);
  }
  const double sum = weighted_tiles<sizeof(T) == 8>(acc, r0, c0, lane, fx, fy, eps + fx.off_eps,
                                    eps + fy.off_eps, flags, 1.0);
  const double total = block_sum(sum, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = 4.0 * pr.s * pr.s * total;
}

// E2_pair[p] = sum of the pair's item partials, in item order.
__global__ void pair_reduce_kernel(const PairInfo* __restrict__ pairs, int64_t npair,
                                   const double* __restrict__ partial,
                                   double* __restrict__ E2_pair, int32_t* __restrict__ flags) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npair) return;
  const PairInfo pr = pairs[p];
  double s = 0.0;
  for (int k = 0; k < pr.item_count; ++k) s += partial[pr.item_first + k];
  E2_pair[p] = s;
  if (!isfinite(s)) atomicOr(flags, FEF_FLAG_NONFINITE);
}

// E2_total = sum over pairs: 1024 contiguous chunks summed in order, then a
// fixed-order block reduction.
__global__ __launch_bounds__(1024) void total_kernel(const double* __restrict__ E2_pair,
                                                     int64_t npair, double* __restrict__ out) {
  __shared__ double red[16];
  const int64_t chunk = (npair + blockDim.x - 1) / blockDim.x;
  const int64_t lo = threadIdx.x * chunk;
  const int64_t hi = lo + chunk < npair ? lo + chunk : npair;
  double s = 0.0;
  for (int64_t k = lo; k < hi; ++k) s += E2_pair[k];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) *out = t;
}

hipError_t launch_split_pairs(const fef_plan_s& p, const void* ops, const double* eps,
                              fef_prec prec, double* partial, int32_t* flags, hipStream_t st);

hipError_t launch_pair_energies(const fef_plan_s& p, const void* ops, const double* eps,
                                fef_prec prec, double* E2_pair, double* E2_total,
                                int32_t* flags, void* ws, hipStream_t st) {
  double* partial = static_cast<double*>(ws);
  const char* o = static_cast<const char*>(ops);
  if (p.nitems > 0) {
    const int kpad = p.geom[prec].kpad;
    switch (prec) {
      case FEF_F64:
        hipLaunchKernelGGL(pair_plain_kernel<double>, dim3((unsigned)p.nitems), dim3(256), 0, st,
                           p.d_frag, p.d_pair, p.d_item, o, (int)prec, kpad, eps, partial, flags);
        break;
      case FEF_F32:
        hipLaunchKernelGGL(pair_plain_kernel<float>, dim3((unsigned)p.nitems), dim3(256), 0, st,
                           p.d_frag, p.d_pair, p.d_item, o, (int)prec, kpad, eps, partial, flags);
        break;
      default: {
        hipError_t e = launch_split_pairs(p, ops, eps, prec, partial, flags, st);
        if (e != hipSuccess) return e;
      }
    }
  }
  if (p.npair > 0)
    hipLaunchKernelGGL(pair_reduce_kernel, dim3((unsigned)((p.npair + 255) / 256)), dim3(256), 0,
                       st, p.d_pair, p.npair, partial, E2_pair, flags);
  hipLaunchKernelGGL(total_kernel, dim3(1), dim3(1024), 0, st, E2_pair, p.npair, E2_total);
  return hipGetLastError();
}

}  // namespace fef
