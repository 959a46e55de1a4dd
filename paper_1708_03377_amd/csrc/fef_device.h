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

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
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
