// Batched FP64 symmetric eigensolver for the fragment Fock matrices
// (polarisation-screened SCF update: canonical orbitals of F~, ascending,
// Aufbau occupation), the new density and its change.
//
// Method: cyclic two-sided Jacobi with the round-robin (circle) parallel
// ordering -- in each of the m-1 rounds of a sweep, m/2 disjoint rotations
// (m = n rounded up to even) are applied at once: rows first (A <- J^T A),
// then columns (A <- A J, V <- V J).  Rotation angles follow the classical
// symmetric Schur decomposition of the 2x2 block:
//   tau = (a_qq - a_pp) / (2 a_pq),  t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1 / sqrt(1 + t^2),  s = t c.
// Sweeps stop when ||offdiag(A)||_F <= 1e-14 ||diag(A)||_2 (at most 40).
// One workgroup per matrix; the matrix and eigenvectors live in LDS for
// n <= 48 and in a global workspace slot otherwise.
#include "fef_internal.h"
#include "fef_device.h"

namespace fef {

__device__ inline void round_robin_pair(int r, int k, int m, int& p, int& q) {
  if (k == 0) {
    p = r;
    q = m - 1;
  } else {
    p = (r + k) % (m - 1);
    q = (r - k + m - 1) % (m - 1);
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

template <int NT, bool kLds>
__global__ __launch_bounds__(NT) void eigh_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ list,
    const double* __restrict__ F, const double* __restrict__ Dold, double* __restrict__ C,
    double* __restrict__ eps, double* __restrict__ Dnew, double* __restrict__ dD_max,
    int32_t* __restrict__ flags, double* __restrict__ ws_eig, int max_n) {
  extern __shared__ double sm[];
  __shared__ double red[NT / 64];
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  const int n = fi.nbf;
  const int m = n + (n & 1);
  const int half = m / 2;
  const int lda = kLds ? n + 1 : n;  // odd stride in LDS spreads the banks
  double *A, *V, *cs;
  if (kLds) {
    A = sm;
    V = sm + (size_t)max_n * (max_n + 1);
    cs = V + (size_t)max_n * (max_n + 1);
  } else {
    A = ws_eig + (size_t)blockIdx.x * 2 * max_n * max_n;
    V = A + (size_t)max_n * max_n;
    cs = sm;
  }
  double* cc = cs;
  double* ss = cs + half;
  int* rank = reinterpret_cast<int*>(ss + half);
  double* lam = reinterpret_cast<double*>(rank + ((n + 1) & ~1));

  const double* Fx = F + fi.off_C;
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int i = e / n, j = e - (e / n) * n;
    A[i * lda + j] = 0.5 * (Fx[i * n + j] + Fx[j * n + i]);
    V[i * lda + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();

  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = threadIdx.x; e < n * n; e += NT) {
      const int i = e / n, j = e - (e / n) * n;
      const double a = A[i * lda + j];
      if (i == j) dia += a * a; else off += a * a;
    }
    off = block_sum(off, red);
    dia = block_sum(dia, red);
    if (off <= 1e-28 * dia || !(off == off)) break;
    for (int r = 0; r < m - 1; ++r) {
      for (int k = threadIdx.x; k < half; k += NT) {
        int p, q;
        round_robin_pair(r, k, m, p, q);
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * lda + q];
          if (apq != 0.0) {
            const double tau = (A[q * lda + q] - A[p * lda + p]) / (2.0 * apq);
            double t;
            if (fabs(tau) > 1e150) t = 0.5 / tau;
            else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        cc[k] = c;
        ss[k] = s;
      }
      __syncthreads();
      for (int e = threadIdx.x; e < half * n; e += NT) {  // rows p, q of A
        const int k = e / n, j = e - (e / n) * n;
        int p, q;
        round_robin_pair(r, k, m, p, q);
        if (q >= n) continue;
        const double c = cc[k], s = ss[k];
        const double ap = A[p * lda + j], aq = A[q * lda + j];
        A[p * lda + j] = c * ap - s * aq;
        A[q * lda + j] = s * ap + c * aq;
      }
      __syncthreads();
      for (int e = threadIdx.x; e < half * n; e += NT) {  // columns p, q of A and V
        const int k = e / n, i = e - (e / n) * n;
        int p, q;
        round_robin_pair(r, k, m, p, q);
        if (q >= n) continue;
        const double c = cc[k], s = ss[k];
        const double ap = A[i * lda + p], aq = A[i * lda + q];
        A[i * lda + p] = c * ap - s * aq;
        A[i * lda + q] = s * ap + c * aq;
        const double vp = V[i * lda + p], vq = V[i * lda + q];
        V[i * lda + p] = c * vp - s * vq;
        V[i * lda + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }

  // ascending order, ties broken by index
  for (int i = threadIdx.x; i < n; i += NT) {
    const double li = A[i * lda + i];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[j * lda + j];
      rk += (lj < li) || (lj == li && j < i);
    }
    rank[i] = rk;
    lam[rk] = li;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) eps[fi.off_eps + rank[i]] = A[i * lda + i];
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int row = e / n, i = e - (e / n) * n;
    C[fi.off_C + (size_t)row * n + rank[i]] = V[row * lda + i];
  }
  // new density from the eigenvectors whose rank is below nocc
  double dmax = 0.0;
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int l = e / n, s = e - (e / n) * n;
    double acc = 0.0;
    for (int i = 0; i < n; ++i)
      if (rank[i] < fi.nocc) acc = fma(V[l * lda + i], V[s * lda + i], acc);
    Dnew[fi.off_C + e] = acc;
    dmax = fmax(dmax, fabs(acc - Dold[fi.off_C + e]));
  }
  dmax = block_max(dmax, red);
  if (threadIdx.x == 0) {
    atomic_max_nonneg(dD_max, dmax);
    if (fi.nocc > 0 && fi.nocc < n && !(lam[fi.nocc] > lam[fi.nocc - 1]))
      atomicOr(flags, FEF_FLAG_GAP);
  }
}

static size_t eig_scratch_bytes(int n) {
  const int half = (n + 1) / 2 + 1;
  return (size_t)2 * half * sizeof(double) + (size_t)((n + 2) & ~1) * sizeof(int) +
         (size_t)(n + 1) * sizeof(double);
}

hipError_t launch_eigh(const fef_plan_s& p, const double* F, const double* Dold, double* C,
                       double* eps, double* Dnew, double* dD_max, int32_t* flags,
                       double* ws_eig, hipStream_t st) {
  if (!p.eig_small.empty()) {
    const int nmax = 32;
    const size_t lds = 2 * (size_t)nmax * (nmax + 1) * sizeof(double) + eig_scratch_bytes(nmax);
    hipLaunchKernelGGL((eigh_kernel<64, true>), dim3((unsigned)p.eig_small.size()), dim3(64), lds,
                       st, p.d_frag, p.d_eig_small, F, Dold, C, eps, Dnew, dD_max, flags, ws_eig,
                       nmax);
  }
  if (!p.eig_mid.empty()) {
    const int nmax = 48;
    const size_t lds = 2 * (size_t)nmax * (nmax + 1) * sizeof(double) + eig_scratch_bytes(nmax);
    hipLaunchKernelGGL((eigh_kernel<256, true>), dim3((unsigned)p.eig_mid.size()), dim3(256), lds,
                       st, p.d_frag, p.d_eig_mid, F, Dold, C, eps, Dnew, dD_max, flags, ws_eig,
                       nmax);
  }
  if (!p.eig_large.empty()) {
    const int nmax = p.eig_large_max_nbf;
    hipLaunchKernelGGL((eigh_kernel<1024, false>), dim3((unsigned)p.eig_large.size()), dim3(1024),
                       eig_scratch_bytes(nmax), st, p.d_frag, p.d_eig_large, F, Dold, C, eps,
                       Dnew, dD_max, flags, ws_eig, nmax);
  }
  return hipGetLastError();
}

}  // namespace fef
