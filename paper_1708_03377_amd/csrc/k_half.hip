// Half transform of the factored integrals (x-side half of the AO -> MO
// transform) and packing of the pair-kernel operands.
//
//   B_ov^x[P][ia] = sum_{mu nu} C^x_{mu i} B^x[P][mu][nu] C^x_{nu a}
//   W^x[Q][ia]    = sum_P G_{c(x),0}[P][Q] B_ov^x[P][ia]
//
// The contraction is done occupied side first (X = C_occ^T B_P, then
// X C_vir), the cheaper order for nocc < nvir.  Both steps read every element
// of B once; the kernel is bound by HBM bandwidth.
#include "fef_internal.h"
#include "fef_device.h"

namespace fef {

// One task = one fragment and up to 8 consecutive factor indices P.
__global__ __launch_bounds__(256) void ht_bov_kernel(const FragInfo* __restrict__ frag,
                                                     const HtTask* __restrict__ tasks,
                                                     const double* __restrict__ B,
                                                     const double* __restrict__ C,
                                                     double* __restrict__ bov) {
  extern __shared__ double smem[];
  const HtTask t = tasks[blockIdx.x];
  const FragInfo fi = frag[t.f];
  const int n = fi.nbf, o = fi.nocc, v = fi.nvir;
  const double* Cf = C + fi.off_C;
  double* X = smem;  // [o][n]
  for (int P = t.p0; P < t.p0 + t.np; ++P) {
    const double* Bp = B + fi.off_B + (int64_t)P * n * n;
    for (int e = threadIdx.x; e < o * n; e += blockDim.x) {
      const int i = e / n, nu = e - (e / n) * n;
      double acc = 0.0;
      for (int mu = 0; mu < n; ++mu) acc = fma(Cf[mu * n + i], Bp[mu * n + nu], acc);
      X[e] = acc;
    }
    __syncthreads();
    double* out = bov + fi.off_bov + (int64_t)P * fi.ov;
    for (int e = threadIdx.x; e < o * v; e += blockDim.x) {
      const int i = e / v, a = e - (e / v) * v;
      double acc = 0.0;
      for (int nu = 0; nu < n; ++nu) acc = fma(X[i * n + nu], Cf[nu * n + o + a], acc);
      out[e] = acc;
    }
    __syncthreads();
  }
}

// W^x[Q][ia] for Q in [8*blockIdx.y, +8).
__global__ __launch_bounds__(256) void ht_w_kernel(const FragInfo* __restrict__ frag,
                                                   const double* __restrict__ G,
                                                   const int64_t* __restrict__ off_G, int P0,
                                                   const double* __restrict__ bov,
                                                   double* __restrict__ w) {
  const FragInfo fi = frag[blockIdx.x];
  if (fi.ov == 0) return;
  const double* g = G + off_G[fi.cls];  // [P_c][P0]
  const double* b = bov + fi.off_bov;   // [P_c][ov]
  const int q0 = blockIdx.y * 8;
  const int nq = min(8, P0 - q0);
  for (int e = threadIdx.x; e < nq * fi.ov; e += blockDim.x) {
    const int q = q0 + e / fi.ov, ia = e - (e / fi.ov) * fi.ov;
    double acc = 0.0;
    for (int P = 0; P < fi.naux; ++P) acc = fma(g[(int64_t)P * P0 + q], b[(int64_t)P * fi.ov + ia], acc);
    w[fi.off_w + (int64_t)q * fi.ov + ia] = acc;
  }
}

// Operand pool, FP64 / FP32 modes: L^x = W^x and R^y = B_ov^y stored
// [kpad][ld] (row k, column ia), zero padded in both directions.
template <typename T>
__global__ __launch_bounds__(256) void pack_plain_kernel(const FragInfo* __restrict__ frag,
                                                         int P0, int kpad, int prec,
                                                         const double* __restrict__ bov,
                                                         const double* __restrict__ w,
                                                         char* __restrict__ ops) {
  const FragInfo fi = frag[blockIdx.x];
  const int k = blockIdx.y;
  if (fi.ld == 0) return;
  T* L = reinterpret_cast<T*>(ops + fi.off_L[prec]) + (int64_t)k * fi.ld;
  T* R = fi.off_R[prec] >= 0 ? reinterpret_cast<T*>(ops + fi.off_R[prec]) + (int64_t)k * fi.ld
                             : nullptr;
  for (int m = threadIdx.x; m < fi.ld; m += blockDim.x) {
    const bool in = (k < P0) && (m < fi.ov);
    L[m] = in ? (T)w[fi.off_w + (int64_t)k * fi.ov + m] : (T)0;
    if (R) R[m] = in ? (T)bov[fi.off_bov + (int64_t)k * fi.ov + m] : (T)0;
  }
}

hipError_t launch_half_transform(const fef_plan_s& p, const double* B, const double* C,
                                 const double* G, double* bov, double* w, void* ops,
                                 fef_prec prec, hipStream_t st) {
  if (p.ht_ntasks > 0) {
    const size_t lds = (size_t)std::max<int64_t>(p.max_on, 1) * sizeof(double);
    hipLaunchKernelGGL(ht_bov_kernel, dim3((unsigned)p.ht_ntasks), dim3(256), lds, st,
                       p.d_frag, p.d_ht, B, C, bov);
    hipLaunchKernelGGL(ht_w_kernel, dim3(p.nfrag, (p.P0 + 7) / 8), dim3(256), 0, st, p.d_frag,
                       G, p.d_off_G, p.P0, bov, w);
  }
  const int kpad = p.geom[prec].kpad;
  char* o = static_cast<char*>(ops);
  switch (prec) {
    case FEF_F64:
      hipLaunchKernelGGL(pack_plain_kernel<double>, dim3(p.nfrag, kpad), dim3(256), 0, st,
                         p.d_frag, p.P0, kpad, (int)prec, bov, w, o);
      break;
    case FEF_F32:
      hipLaunchKernelGGL(pack_plain_kernel<float>, dim3(p.nfrag, kpad), dim3(256), 0, st,
                         p.d_frag, p.P0, kpad, (int)prec, bov, w, o);
      break;
    default:
      return launch_pack_split(p, bov, w, ops, prec, st);
  }
  return hipGetLastError();
}

}  // namespace fef
