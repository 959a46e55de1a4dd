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
// One workgroup per fragment.  Each wave loads its row strip of W (16 ia
// rows, every k step) into registers while the workgroup stages B_ov in LDS,
// all of those loads in flight together; the waves then form V on FP64 MFMA
// (16 x 16 output tiles, one row strip per wave, its W registers reused for
// every column tile; V = B_ov^T G_{0,0} B_ov is symmetric, so only the tiles
// on and above the diagonal are formed and the others mirrored) and write it
// over the staged B_ov.  Every thread then
// takes fixed (a, b) and runs over the occupied pairs (i, j), reading (ia|jb)
// and its exchange partner (ib|ja) from LDS.  The LDS row stride of V is
// odd, so the exchange reads of consecutive b (a stride of one row) fall in
// different banks.
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
// k steps of 4 held in registers: P_0 <= 80
constexpr int kMonoKSteps = 20;
constexpr int kMonoMaxP = 4 * kMonoKSteps;

typedef double d4v __attribute__((ext_vector_type(4)));

__host__ __device__ inline int mono_ld(int ov) { return ov | 1; }

// Row strip of each wave.  Strip s forms NT - s tiles (those on and right of
// the diagonal); the waves of a workgroup sit on the four SIMDs in turn
// (wave w on SIMD w % 4), so the strips are dealt longest first to the
// SIMD with the least work so far (-1: no strip).
template <int NT>
struct StripMap {
  int strip[kMonoWaves];
  constexpr StripMap() : strip() {
    int load[4] = {0, 0, 0, 0};
    for (int w = 0; w < kMonoWaves; ++w) strip[w] = -1;
    for (int s = 0; s < NT; ++s) {
      int best = -1;
      for (int w = 0; w < kMonoWaves; ++w)
        if (strip[w] < 0 && (best < 0 || load[w % 4] < load[best % 4])) best = w;
      strip[best] = s;
      load[best % 4] += NT - s;
    }
  }
};

// NT: column tiles of the launch (ceil(max ov / 16)); a fragment with fewer
// reads zeros for the rest, so the product loops have no branches
template <int NT>
__global__ __launch_bounds__(kMonoThreads) void monomer_energy_kernel(
    const FragInfo* __restrict__ frag, const double* __restrict__ bov,
    const double* __restrict__ w, const double* __restrict__ eps, double* __restrict__ E_M2,
    int32_t* __restrict__ flags) {
  // LDS: B_ov staged as [P][ov], then V [ov][ld] written over it once every
  // wave has finished reading it; the fragment's orbital energies after the
  // larger of the two
  extern __shared__ double lds[];
  __shared__ double red[kMonoWaves];
  const FragInfo fi = frag[blockIdx.x];
  const int o = fi.nocc, v = fi.nvir, ov = fi.ov, P = fi.naux, ld = mono_ld(ov);
  const int nB = P * ov;
  double* V = lds;
  double* es = lds + max(nB, ov * ld);

  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int li = lane & 15, lk = lane >> 4;
  const int nt = (ov + 15) >> 4;
  constexpr StripMap<NT> kMap;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int sp = kMap.strip[wv];  // this wave's row strip
  const bool has_strip = sp >= 0 && sp < nt;
  const bool gemm = has_strip && P > 0;
  const int m = sp * 16 + li;
  const int mc = min(m, ov - 1);
  // this wave's W strip, A[m][k] = W[k][m], every k step loaded at once:
  // rows past P read row P - 1 and columns past ov column ov - 1, and are
  // multiplied by zero (a select would let the compiler turn each load into
  // a branch of its own that waits for it)
  double areg[kMonoKSteps];
  if (gemm) {
    const double* Wf = w + fi.off_w;
#pragma unroll
    for (int s2 = 0; s2 < kMonoKSteps; ++s2)
      areg[s2] = Wf[(int64_t)min(4 * s2 + lk, P - 1) * ov + mc];
  }
  // B_ov into LDS, sixteen loads per thread in flight.  The first chunk
  // (all of B_ov up to 8192 elements) is straight-line code: at the head of
  // a loop the compiler waits for every load in flight, the W loads too.
  {
    const double* Bf = bov + fi.off_bov;
    auto stage = [&](int e0) __attribute__((always_inline)) {
      double tmp[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = e0 + u * kMonoThreads + threadIdx.x;
        tmp[u] = Bf[min(e, nB - 1)];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = e0 + u * kMonoThreads + threadIdx.x;
        if (e < nB) V[e] = tmp[u];
      }
    };
    if (nB > 0) stage(0);
    for (int e0 = 16 * kMonoThreads; e0 < nB; e0 += 16 * kMonoThreads) stage(e0);
  }
  for (int k = threadIdx.x; k < fi.nbf; k += kMonoThreads) es[k] = eps[fi.off_eps + k];
  if (gemm) {
    // zeroed only now, so that the B_ov loads above are issued before the
    // W loads are waited for
#pragma unroll
    for (int s2 = 0; s2 < kMonoKSteps; ++s2)
      areg[s2] *= (4 * s2 + lk < P && m < ov) ? 1.0 : 0.0;
  }
  __syncthreads();

  // V is symmetric (G_{0,0} is), so each wave forms only the tiles of its
  // row strip on and right of the diagonal and mirrors them
  d4v acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = d4v{0.0, 0.0, 0.0, 0.0};
  if (gemm) {
    // the k steps up to P, the NT reads of a step issued together.  B is
    // not masked: its rows past P meet zeros of the strip, and its columns
    // past ov only reach output columns that are not kept.
#pragma unroll
    for (int s2 = 0; s2 < kMonoKSteps; ++s2) {
      if (4 * s2 >= P) break;
      const int kr = min(4 * s2 + lk, P - 1) * ov;
      double b[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) b[t] = V[kr + min(t * 16 + li, ov - 1)];
#pragma unroll
      for (int t = 0; t < NT; ++t)
        if (t >= sp) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(areg[s2], b[t], acc[t], 0, 0, 0);
    }
  }
  __syncthreads();  // every wave is done with the staged B_ov
  if (has_strip) {
    // FP64 MFMA result: row lk + 4 r, column li of each 16 x 16 tile
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (t < sp) continue;
      const int n = t * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = sp * 16 + lk + 4 * r;
        if (row < ov && n < ov) {
          V[row * ld + n] = acc[t][r];
          if (t > sp) V[n * ld + row] = acc[t][r];
        }
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
    mx = std::max<int64_t>(mx, std::max<int64_t>((int64_t)fi.naux * fi.ov,
                                                 (int64_t)fi.ov * mono_ld(fi.ov)) + fi.nbf);
  return (size_t)(8 * mx);
}

// Lifts the dynamic-LDS limit of each instantiation once per process (a
// refusal is left to the launch to report).
template <int NT>
void launch_monomer(const fef_plan_s& p, size_t lds, hipStream_t st, const double* Bov,
                    const double* W, const double* eps, double* E_M2, int32_t* flags) {
  static bool configured = false;
  if (!configured) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&monomer_energy_kernel<NT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
    (void)hipGetLastError();
    configured = true;
  }
  hipLaunchKernelGGL(monomer_energy_kernel<NT>, dim3(p.nfrag), dim3(kMonoThreads), lds, st,
                     p.d_frag, Bov, W, eps, E_M2, flags);
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
    if (fi.ov > kMonoMaxOv || fi.naux > kMonoMaxP) return FEF_E_UNSUPPORTED;
  }
  const size_t lds = monomer_lds_bytes(*p);
  int max_ov = 0;
  for (const FragInfo& fi : p->frag) max_ov = std::max(max_ov, fi.ov);
  const int nt = std::max(1, (max_ov + 15) / 16);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->nfrag > 0) {
    switch (nt) {
      case 1: launch_monomer<1>(*p, lds, st, Bov, W, eps, E_M2, flags); break;
      case 2: launch_monomer<2>(*p, lds, st, Bov, W, eps, E_M2, flags); break;
      case 3: launch_monomer<3>(*p, lds, st, Bov, W, eps, E_M2, flags); break;
      case 4: launch_monomer<4>(*p, lds, st, Bov, W, eps, E_M2, flags); break;
      case 5: launch_monomer<5>(*p, lds, st, Bov, W, eps, E_M2, flags); break;
      case 6: launch_monomer<6>(*p, lds, st, Bov, W, eps, E_M2, flags); break;
      case 7: launch_monomer<7>(*p, lds, st, Bov, W, eps, E_M2, flags); break;
      default: launch_monomer<8>(*p, lds, st, Bov, W, eps, E_M2, flags); break;
    }
  }
  hipLaunchKernelGGL(monomer_total_kernel, dim3(1), dim3(256), 0, st, E_M2, (int64_t)p->nfrag,
                     E_M2_total);
  return hipGetLastError() == hipSuccess ? FEF_OK : FEF_E_HIP;
}

}  // extern "C"
