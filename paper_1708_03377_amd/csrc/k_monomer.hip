// Monomer part of the second-order energy (Sec. II.B, Eq. EFEF2): for every
// fragment x the contraction of its two-body de-excitation operator with its
// first-order doubles (Eq. EM2), the doubles solving the fragment equation
// of Eq. monDoubles with the two-body part of H0 dropped (as for the pair
// energies), in closed-shell spatial orbitals:
//   E_M2^x = sum_{ijab} (ia|jb) [2 (ia|jb) - (ib|ja)] / (eps_i + eps_j - eps_a - eps_b).
//
// Integrals inside a fragment: the factored tensor with the solvent class's
// own coupling block at unit scale,
//   (ia|jb)^{xx} = sum_PQ B^x_ov[P][ia] G_{0,0}[P][Q] B^x_ov[Q][jb]
//                = sum_Q W^x[Q][ia] B^x_ov[Q][jb],   W^x = G_{0,0}^T B^x_ov,
// so the half transform's dense FP64 outputs B_ov and W give the whole
// ov x ov block V = W^T B_ov in one GEMM over P_0.  Only class 0 has such a
// block.
//
// One workgroup per fragment: the waves form V on FP64 MFMA (16 x 16 output
// tiles, one row strip per wave, the strip's W operand loaded once for all
// column tiles) into LDS, then every thread takes fixed (a, b) and runs over
// the occupied pairs (i, j), reading (ia|jb) and its exchange partner
// (ib|ja) from LDS.  The LDS row stride is odd, so the exchange reads of
// consecutive b (a stride of one row) fall in different banks.
#include <algorithm>
#include <cmath>

#include "fef_internal.h"
#include "fef_device.h"

namespace fef {

namespace {

constexpr int kMonoThreads = 512;
constexpr int kMonoWaves = kMonoThreads / kWave;
// row strips of 16 (one per wave): ov <= 128
constexpr int kMonoMaxOv = 16 * kMonoWaves;

typedef double d4v __attribute__((ext_vector_type(4)));

__host__ __device__ inline int mono_ld(int ov) { return ov | 1; }

__global__ __launch_bounds__(kMonoThreads) void monomer_energy_kernel(
    const FragInfo* __restrict__ frag, const double* __restrict__ bov,
    const double* __restrict__ w, const double* __restrict__ eps, double* __restrict__ E_M2,
    int32_t* __restrict__ flags) {
  extern __shared__ double V[];  // [ov][ld], then eps of the fragment [nbf]
  __shared__ double red[kMonoWaves];
  const FragInfo fi = frag[blockIdx.x];
  const int o = fi.nocc, v = fi.nvir, ov = fi.ov, P = fi.naux, ld = mono_ld(ov);
  double* es = V + (int64_t)ov * ld;
  for (int k = threadIdx.x; k < fi.nbf; k += kMonoThreads) es[k] = eps[fi.off_eps + k];

  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int li = lane & 15, lk = lane >> 4;
  const int nt = (ov + 15) >> 4;
  if (wave < nt) {
    const double* Wf = w + fi.off_w;
    const double* Bf = bov + fi.off_bov;
    const int m = wave * 16 + li;
    const int mc = min(m, ov - 1);
    d4v acc[kMonoWaves];
#pragma unroll
    for (int t = 0; t < kMonoWaves; ++t) acc[t] = d4v{0.0, 0.0, 0.0, 0.0};
    // A[m][k] = W[k][m], B[k][n] = B_ov[k][n]; rows past P and columns past
    // ov read a valid element and contribute zero.  Two k steps in flight:
    // the loads of the next step are issued before the products of this one.
    auto load = [&](int k0, double& a, double (&b)[kMonoWaves]) __attribute__((always_inline)) {
      const int k = k0 + lk;
      const bool kin = k < P;
      const int64_t kr = (int64_t)(kin ? k : P - 1) * ov;
      a = (kin && m < ov) ? Wf[kr + mc] : 0.0;
#pragma unroll
      for (int t = 0; t < kMonoWaves; ++t) {
        const int n = t * 16 + li;
        b[t] = (t < nt && kin && n < ov) ? Bf[kr + min(n, ov - 1)] : 0.0;
      }
    };
    auto mult = [&](double a, const double (&b)[kMonoWaves]) __attribute__((always_inline)) {
#pragma unroll
      for (int t = 0; t < kMonoWaves; ++t)
        if (t < nt) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[t], acc[t], 0, 0, 0);
    };
    double a0 = 0.0, a1 = 0.0, b0[kMonoWaves] = {}, b1[kMonoWaves] = {};
    if (P > 0) load(0, a0, b0);
    for (int k0 = 0; k0 < P; k0 += 8) {
      load(k0 + 4, a1, b1);
      mult(a0, b0);
      if (k0 + 8 < P) load(k0 + 8, a0, b0);
      if (k0 + 4 < P) mult(a1, b1);
    }
    // FP64 MFMA result: row lk + 4 r, column li of each 16 x 16 tile
#pragma unroll
    for (int t = 0; t < kMonoWaves; ++t) {
      if (t >= nt) continue;
      const int n = t * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wave * 16 + lk + 4 * r;
        if (row < ov && n < ov) V[(int64_t)row * ld + n] = acc[t][r];
      }
    }
  }
  __syncthreads();

  double sum = 0.0;
  for (int ab = threadIdx.x; ab < v * v; ab += kMonoThreads) {
    const int a = ab / v, b = ab - (ab / v) * v;
    const double eab = es[o + a] + es[o + b];
    for (int i = 0; i < o; ++i) {
      const double* Vi_a = V + (int64_t)(i * v + a) * ld;
      const double* Vi_b = V + (int64_t)(i * v + b) * ld;
      const double ei = es[i];
      for (int j = 0; j < o; ++j) {
        const double x = Vi_a[j * v + b];   // (ia|jb)
        const double xe = Vi_b[j * v + a];  // (ib|ja)
        sum += x * (2.0 * x - xe) / (ei + es[j] - eab);
      }
    }
  }
  const double tot = block_sum(sum, red);
  if (threadIdx.x == 0) {
    E_M2[blockIdx.x] = tot;
    if (!std::isfinite(tot)) atomicOr(flags, 2);
  }
}

// Sum of the fragment energies in a fixed order (strided per thread, then
// the block-wide sum).
__global__ __launch_bounds__(256) void monomer_total_kernel(const double* __restrict__ E_M2,
                                                            int64_t nfrag,
                                                            double* __restrict__ out) {
  __shared__ double red[256 / kWave];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < nfrag; k += 256) s += E_M2[k];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) *out = t;
}

size_t monomer_lds_bytes(const fef_plan_s& p) {
  int64_t mx = 0;
  for (const FragInfo& fi : p.frag)
    mx = std::max<int64_t>(mx, (int64_t)fi.ov * mono_ld(fi.ov) + fi.nbf);
  return (size_t)(8 * mx);
}

}  // namespace

}  // namespace fef

using namespace fef;

extern "C" {

fef_status fef_monomer_energies(fef_plan p, const double* Bov, const double* W,
                                const double* eps, double* E_M2, double* E_M2_total,
                                int32_t* flags, void* stream) {
  if (!p) return FEF_E_ARG;
  if (!E_M2_total || !flags) return FEF_E_ARG;
  if (p->nfrag > 0 && (!Bov || !W || !eps || !E_M2)) return FEF_E_ARG;
  for (const FragInfo& fi : p->frag) {
    if (fi.cls != 0) return FEF_E_SHAPE;
    if (fi.ov > kMonoMaxOv) return FEF_E_UNSUPPORTED;
  }
  const size_t lds = monomer_lds_bytes(*p);
  static bool configured = false;
  if (!configured) {
    // lifts the dynamic-LDS limit once per process; a refusal is left to
    // the launch to report
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&monomer_energy_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
    (void)hipGetLastError();
    configured = true;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->nfrag > 0)
    hipLaunchKernelGGL(monomer_energy_kernel, dim3(p->nfrag), dim3(kMonoThreads), lds, st,
                       p->d_frag, Bov, W, eps, E_M2, flags);
  hipLaunchKernelGGL(monomer_total_kernel, dim3(1), dim3(256), 0, st, E_M2, (int64_t)p->nfrag,
                     E_M2_total);
  return hipGetLastError() == hipSuccess ? FEF_OK : FEF_E_HIP;
}

}  // extern "C"
