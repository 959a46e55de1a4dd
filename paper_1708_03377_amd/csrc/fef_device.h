// Device-side helpers for the gfx950 kernels (64-wide wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cstdint>

namespace fef {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

// LDS (address space 3) destination of global_load_lds copies
typedef __attribute__((address_space(3))) void lds_void_t;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// DPP move of a double within rows of 16 lanes (both halves moved with the
// same control); every lane has a source for the controls used here.
template <int kCtrl>
__device__ inline double dpp_row_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double readlane_f64(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave sum without LDS traffic: DPP butterflies inside each row of 16 lanes
// (quad swaps, then rotations by 4 and 8), then the four row sums read as
// scalars and added in a fixed order.  The result is uniform across the wave.
__device__ inline double wave_sum_dpp(double v) {
  v += dpp_row_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_row_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_row_f64<0x124>(v);  // row_ror 4
  v += dpp_row_f64<0x128>(v);  // row_ror 8
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Block-wide sum with a fixed reduction order (lane order inside each wave,
// then wave order).  `red` must hold blockDim.x / 64 doubles.  Result valid in
// every thread.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < nw; ++k) t += red[k];
  __syncthreads();
  return t;
}

__device__ inline double block_max(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  double t = red[0];
  for (int k = 1; k < nw; ++k) t = fmax(t, red[k]);
  __syncthreads();
  return t;
}

// Max of non-negative doubles through their bit patterns (monotone for
// values >= 0), so the result does not depend on the order of arrival.
__device__ inline void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            (unsigned long long)__double_as_longlong(v));
}


// Next work item of the grouped persistent queue (8 counters at head):
// the caller's home group first, then the others in turn; -1 when all are
// exhausted.  Called by one thread of the workgroup.
__device__ inline int32_t pull_item(int32_t* head, const int32_t* grp_off, int home) {
  for (int k = 0; k < 8; ++k) {
    const int g = (home + k) & (8 - 1);
    const int32_t cnt = grp_off[g + 1] - grp_off[g];
    if (cnt <= 0 || __atomic_load_n(&head[g], __ATOMIC_RELAXED) >= cnt) continue;
    const int32_t i = atomicAdd(&head[g], 1);
    if (i < cnt) return grp_off[g] + i;
  }
  return -1;
}

}  // namespace fef
