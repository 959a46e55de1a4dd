// FP64 eigensolver for the large fragment Fock matrices (48 < n <= 152,
// the nucleobase-like solute): canonical orbitals of F~ ascending, Aufbau
// occupation, the new density and its change, as the Jacobi solvers.
//
// Three kernels, one 512-thread workgroup per matrix each, so that every
// stage has the whole register file to itself:
//   1. eigh_tri_reduce: Householder tridiagonalisation Q^T A Q = T
//      (A = (F + F^T) / 2).  For k = 0 .. n-3 the reflector
//      H_k = I - tau_k v_k v_k^T maps the part of row k right of the
//      diagonal onto its first entry; the trailing block takes the
//      symmetric rank-2 update A <- A - v w^T - w v^T with p = tau A v,
//      w = p - (tau / 2)(p . v) v.  A lives in registers, one row per two
//      lanes (a segment of SEG columns each).
//   2. eigh_tri_values: the eigenvalues of T by multisection on the Sturm
//      count (the number of negative pivots of the LDL^T factorisation of
//      T - x I): four lanes per eigenvalue count at four interior points,
//      shrinking the bracket five-fold per round until it is a few ulps of
//      the eigenvalue (or of ||T|| near zero) wide.  Eigenvalue j is the
//      (j+1)-th smallest, so the order is ascending with ties in index
//      order.  Then the eigenvectors of T by inverse iteration: Gaussian
//      elimination with partial pivoting of T - lambda I, three solves
//      from a fixed pseudo-random start; eigenvalues closer than
//      1e-3 ||T|| form a cluster that one thread handles in order, each
//      vector orthogonalised against the cluster's earlier ones after every
//      solve (modified Gram-Schmidt), a repeated eigenvalue nudged by a few
//      ulps first.
//   3. eigh_tri_back: back-transformation C = H_0 H_1 ... H_{n-3} Z, one
//      eigenvector per two lanes, then C, the density and its change.
// Eigenvalues are accurate to a few ulps of ||T||; eigenvector residuals
// and orthogonality are at rounding level times ||T|| / gap.
#include <algorithm>
#include <cfloat>

#include "fef_internal.h"
#include "fef_device.h"

namespace fef {

namespace {

constexpr int kTriThreads = 512;
constexpr int kTriLanes = 2;  // lanes per row / eigenvector
constexpr int kTriRowsPerWave = 64 / kTriLanes;
constexpr int kTriHelper = kTriThreads / 64 - 1;  // the last wave holds no row

// sum over the two lanes of a row
__device__ inline double pair_sum(double v) {
  return v + dpp_row_f64<0xB1>(v);  // quad_perm [1, 0, 3, 2]
}

// packed offset of reflector k's entries k+1 .. n-1
__host__ __device__ inline int refl_off(int k, int n) { return k * (n - 1) - k * (k - 1) / 2; }

// A copy of x the compiler cannot see through: index tests against it in
// one place are not merged with the same tests elsewhere, so their
// per-element masks do not stay live (and spill) across the kernel.
__device__ inline int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Sturm count: the number of eigenvalues of T below x (negative pivots of
// T - x I = L D L^T), tiny pivots replaced by -pivmin.
__device__ inline int sturm_count(const double* d, const double* e2, int n, double x,
                                  double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// Fixed pseudo-random start vector entry in [-1, 1) (a counter hash).
__device__ inline double start_entry(int j, int i) {
  uint32_t h = (uint32_t)j * 2654435761u + (uint32_t)i * 40503u + 12345u;
  h ^= h >> 16;
  h *= 0x45D9F3Bu;
  h ^= h >> 16;
  return (double)h * (1.0 / 2147483648.0) - 1.0;
}

// Per-matrix workspace (doubles, a slot of eig_large_slot(max_n)):
//   T: d [n], e [n], tau [n]; the reflectors, packed [refl_off(n - 2, n)];
//   Z [n][n + 64] (row j = eigenvector j of T, zero past n); per eigenvalue
//   six vectors of elimination factors [n][6 n].
struct TriWs {
  double *d, *e, *tau, *refl, *Z, *fac;
};
__device__ inline TriWs tri_ws(double* ws_eig, int max_n, int n) {
  TriWs w;
  w.d = ws_eig + (size_t)blockIdx.x * eig_large_slot(max_n);
  w.e = w.d + n;
  w.tau = w.e + n;
  w.refl = w.tau + n;
  w.Z = w.refl + (n > 2 ? refl_off(n - 2, n) : 0);
  w.fac = w.Z + (size_t)n * (n + 64);
  return w;
}

}  // namespace

// ---------------------------------------------------------------------------
// 1. tridiagonalisation
template <int SEG>
__global__ __launch_bounds__(kTriThreads) void eigh_tri_reduce_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ list,
    const double* __restrict__ F, double* __restrict__ ws_eig, int max_n) {
  constexpr int NC = kTriLanes * SEG;  // padded column count
  __shared__ double pb[NC];            // p (zero on rows <= k and past n)
  __shared__ double vbuf[2][NC];       // reflector k over every column
  __shared__ double xbuf[NC];          // the row being reduced
  __shared__ double wpart[kTriThreads / 64];
  __shared__ double s_tau;
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  const int n = fi.nbf;
  const TriWs W = tri_ws(ws_eig, max_n, n);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = kTriRowsPerWave * wave + lane / kTriLanes, seg = lane % kTriLanes;
  const int c0 = SEG * seg;
  const bool has_row = row < n;
  const double* Fx = F + fi.off_C;
  double a[SEG];
#pragma unroll
  for (int c = 0; c < SEG; ++c) a[c] = 0.0;
  if (has_row) {
#pragma unroll
    for (int c = 0; c < SEG; ++c) {
      const int j = opaque(c0) + c;
      const int jc = j < n ? j : n - 1;  // every load in bounds, no branch
      const double v = 0.5 * (Fx[(size_t)row * n + jc] + Fx[(size_t)jc * n + row]);
      a[c] = j < n ? v : 0.0;
    }
  }
  for (int i = threadIdx.x; i < NC; i += kTriThreads) pb[i] = 0.0;
  if (row == 0) {
#pragma unroll
    for (int c = 0; c < SEG; ++c) xbuf[c0 + c] = a[c];
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    double* vc = vbuf[k & 1];
    if (wave == kTriHelper) {
      // x = A[k][k+1 ..]; sigma = |x|^2 - x0^2; lane l takes columns l, l + 64, ...
      double sig = 0.0;
      for (int j = lane; j < NC; j += 64) {
        const double xj = xbuf[j];
        if (j > k + 1) sig = fma(xj, xj, sig);
      }
      sig = wave_sum_dpp(sig);
      const double x0 = xbuf[k + 1];
      double t = 0.0, alpha = x0;
      if (sig != 0.0) {
        alpha = -copysign(sqrt(x0 * x0 + sig), x0);
        t = 2.0 / ((x0 - alpha) * (x0 - alpha) + sig);
      }
      double* vk = W.refl + refl_off(k, n) - (k + 1);  // packed, entries k+1 .. n-1
      for (int j = lane; j < NC; j += 64) {
        const double vj = (t == 0.0 || j <= k) ? 0.0 : (j == k + 1 ? x0 - alpha : xbuf[j]);
        vc[j] = vj;
        if (j > k && j < n) vk[j] = vj;
      }
      if (lane == 0) {
        s_tau = t;
        W.tau[k] = t;
        W.d[k] = xbuf[k];
        W.e[k] = alpha;
      }
    }
    __syncthreads();
    const double t = s_tau;
    if (t != 0.0) {
      // p = tau A v over the trailing block (zero on rows <= k), p . v by waves
      double pr = 0.0;
#pragma unroll
      for (int c = 0; c < SEG; ++c) pr = fma(a[c], vc[c0 + c], pr);
      pr = row > k ? t * pair_sum(pr) : 0.0;
      const double vr = has_row ? vc[row] : 0.0;
      if (has_row && seg == 0) pb[row] = pr;
      const double pv = wave_sum_dpp(seg == 0 ? pr * vr : 0.0);
      if (lane == 0) wpart[wave] = pv;
      __syncthreads();
      double s = 0.0;
      for (int w = 0; w < kTriThreads / 64; ++w) s += wpart[w];
      const double K = 0.5 * t * s;
      // A <- A - v w^T - w v^T with w = p - K v; rows and columns outside the
      // trailing block have v = p = 0 and keep their values.  Two rounded
      // products and their sum (no contraction): entry (j, r) gets the same
      // two products, so A stays exactly symmetric.
      const double wr = pr - K * vr;
      {
#pragma clang fp contract(off)
#pragma unroll
        for (int c = 0; c < SEG; ++c) {
          const double vj = vc[c0 + c];
          const double wj = pb[c0 + c] - K * vj;
          a[c] -= vr * wj + wr * vj;
        }
      }
    }
    // the next row to reduce
    if (row == k + 1) {
#pragma unroll
      for (int c = 0; c < SEG; ++c) xbuf[c0 + c] = a[c];
    }
    __syncthreads();
  }
  // the last 2 x 2 block
  if (n >= 2 && (row == n - 2 || row == n - 1)) {
    double dd = 0.0, off = 0.0;
#pragma unroll
    for (int c = 0; c < SEG; ++c) {
      const int j = opaque(c0) + c;
      if (j == row) dd = a[c];
      if (row == n - 1 && j == n - 2) off = a[c];
    }
    dd = pair_sum(dd);
    off = pair_sum(off);
    if (seg == 0) {
      W.d[row] = dd;
      if (row == n - 1) {
        W.e[n - 2] = off;
        W.e[n - 1] = 0.0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 2. eigenvalues (written to eps) and eigenvectors of T
__global__ __launch_bounds__(kTriThreads) void eigh_tri_values_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ list,
    double* __restrict__ eps, double* __restrict__ ws_eig, int max_n) {
  extern __shared__ double sm[];  // d, e, e^2, lambda [n] each
  __shared__ double sc[4];
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  const int n = fi.nbf;
  const TriWs W = tri_ws(ws_eig, max_n, n);
  double* dg = sm;
  double* ee = dg + n;
  double* e2 = ee + n;
  double* lam = e2 + n;
  for (int i = threadIdx.x; i < n; i += kTriThreads) {
    dg[i] = W.d[i];
    ee[i] = i + 1 < n ? W.e[i] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tn = 0.0, lo = 0.0, hi = 0.0, e2max = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
      tn = fmax(tn, fabs(dg[i]) + r);
      lo = i == 0 ? dg[i] - r : fmin(lo, dg[i] - r);
      hi = i == 0 ? dg[i] + r : fmax(hi, dg[i] + r);
      e2[i] = ee[i] * ee[i];
      e2max = fmax(e2max, e2[i]);
    }
    const double pivmin = 1e-290 * fmax(1.0, e2max);
    const double pad = 2.0 * DBL_EPSILON * tn + 2.0 * pivmin;
    sc[0] = lo - pad;
    sc[1] = hi + pad;
    sc[2] = tn;
    sc[3] = pivmin;
  }
  __syncthreads();
  {
    const double pivmin = sc[3];
    const int m = threadIdx.x & 3;
    for (int j = threadIdx.x >> 2; j < n; j += kTriThreads / 4) {
      double lo = sc[0], hi = sc[1];
      for (int it = 0; it < 80; ++it) {
        // a bracket of a few ulps of the eigenvalue, or of ||T|| near zero
        if (!(hi - lo > 2.0 * DBL_EPSILON * (fmax(fabs(lo), fabs(hi)) + sc[2]) + 2.0 * pivmin))
          break;
        const double x = lo + (double)(m + 1) * ((hi - lo) * 0.2);
        const int cnt = sturm_count(dg, e2, n, x, pivmin);
        // the quad's four points: the new bracket is [last point below the
        // (j+1)-th eigenvalue, first point at or above it]
        const int above = cnt >= j + 1;
        const int m0 = __builtin_amdgcn_mov_dpp(above, 0x00, 0xF, 0xF, false);  // quad lane 0
        const int m1 = __builtin_amdgcn_mov_dpp(above, 0x55, 0xF, 0xF, false);  // quad lane 1
        const int m2 = __builtin_amdgcn_mov_dpp(above, 0xAA, 0xF, 0xF, false);  // quad lane 2
        const int m3 = __builtin_amdgcn_mov_dpp(above, 0xFF, 0xF, 0xF, false);  // quad lane 3
        const int first = m0 ? 0 : m1 ? 1 : m2 ? 2 : m3 ? 3 : 4;
        const double w = (hi - lo) * 0.2;
        const double nlo = first == 0 ? lo : lo + (double)first * w;
        const double nhi = first == 4 ? hi : lo + (double)(first + 1) * w;
        lo = nlo;
        hi = nhi;
      }
      if (m == 0) {
        lam[j] = 0.5 * (lo + hi);
        eps[fi.off_eps + j] = lam[j];
      }
    }
  }
  __syncthreads();
  // inverse iteration, one thread per cluster of close eigenvalues
  if ((int)threadIdx.x < n) {
    const int j = threadIdx.x;
    const int ld = n + 64;
    const double tn = sc[2];
    const double ortol = 1e-3 * tn, tiny = DBL_EPSILON * fmax(tn, 1e-300);
    if (j == 0 || lam[j] - lam[j - 1] > ortol) {
      int j1 = j;
      while (j1 + 1 < n && lam[j1 + 1] - lam[j1] <= ortol) ++j1;
      // this thread's six work vectors, interleaved with the other threads'
      // (entry i of vector v at (v n + i) n + j), so that threads stepping
      // through their recurrences together touch neighbouring addresses
      double* base = W.fac + j;
      const size_t sv = (size_t)n * n;
      auto A_ = [&](int i) -> double& { return base[(size_t)i * n]; };           // diagonal of U
      auto B_ = [&](int i) -> double& { return base[sv + (size_t)i * n]; };      // first superdiagonal
      auto D_ = [&](int i) -> double& { return base[2 * sv + (size_t)i * n]; };  // second superdiagonal
      auto L_ = [&](int i) -> double& { return base[3 * sv + (size_t)i * n]; };  // multipliers
      auto P_ = [&](int i) -> double& { return base[4 * sv + (size_t)i * n]; };  // 1: rows i, i+1 swapped
      auto x = [&](int i) -> double& { return base[5 * sv + (size_t)i * n]; };   // iterate
      double prev = 0.0;
      for (int jj = j; jj <= j1; ++jj) {
        double lm = lam[jj];
        if (jj > j && lm - prev < 10.0 * DBL_EPSILON * fabs(lm))
          lm = prev + 10.0 * DBL_EPSILON * fabs(lm);
        prev = lm;
        // T - lm I = P L U with row interchanges between neighbours; the
        // current row's diagonal and superdiagonal ride in registers
        double ak = dg[0] - lm, bk = n > 1 ? ee[0] : 0.0;
        for (int k = 0; k + 1 < n; ++k) {
          const double ck = ee[k];
          double ak1 = dg[k + 1] - lm, bk1 = k + 2 < n ? ee[k + 1] : 0.0;
          if (fabs(ak) >= fabs(ck)) {
            if (ak == 0.0) ak = tiny;
            const double l = ck / ak;
            L_(k) = l;
            P_(k) = 0.0;
            D_(k) = 0.0;
            A_(k) = ak;
            B_(k) = bk;
            ak1 -= l * bk;
          } else {
            const double l = ak / ck;
            L_(k) = l;
            P_(k) = 1.0;
            A_(k) = ck;
            B_(k) = ak1;
            D_(k) = bk1;
            const double na = bk - l * ak1;
            bk1 = -l * bk1;
            ak1 = na;
          }
          ak = ak1;
          bk = bk1;
        }
        A_(n - 1) = ak;
        B_(n - 1) = 0.0;
        for (int i = 0; i < n; ++i)
          if (fabs(A_(i)) < tiny) A_(i) = A_(i) < 0.0 ? -tiny : tiny;
        for (int i = 0; i < n; ++i) x(i) = start_entry(jj, i);
        for (int itn = 0; itn < 3; ++itn) {
          double mx = 0.0;
          for (int i = 0; i < n; ++i) mx = fmax(mx, fabs(x(i)));
          const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
          for (int i = 0; i < n; ++i) x(i) *= inv;
          // forward: the row interchanges and multipliers; backward: U
          double xk = x(0);
          for (int k = 0; k + 1 < n; ++k) {
            double x1 = x(k + 1);
            if (P_(k) != 0.0) {
              const double t = xk;
              xk = x1;
              x1 = t;
            }
            x1 -= L_(k) * xk;
            x(k) = xk;
            xk = x1;
          }
          x(n - 1) = xk;
          double x1 = 0.0, x2 = 0.0;  // x(k + 1), x(k + 2)
          for (int k = n - 1; k >= 0; --k) {
            const double xv = (x(k) - B_(k) * x1 - D_(k) * x2) / A_(k);
            x(k) = xv;
            x2 = x1;
            x1 = xv;
          }
          for (int q = j; q < jj; ++q) {
            const double* zq = W.Z + (size_t)q * ld;
            double dot = 0.0;
            for (int i = 0; i < n; ++i) dot = fma(zq[i], x(i), dot);
            for (int i = 0; i < n; ++i) x(i) -= dot * zq[i];
          }
          double nrm = 0.0;
          for (int i = 0; i < n; ++i) nrm = fma(x(i), x(i), nrm);
          const double r = 1.0 / sqrt(nrm);
          for (int i = 0; i < n; ++i) x(i) *= r;
        }
        double* zj = W.Z + (size_t)jj * ld;
        for (int i = 0; i < n; ++i) zj[i] = x(i);
        for (int i = n; i < ld; ++i) zj[i] = 0.0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 3. back-transformation and outputs
template <int SEG>
__global__ __launch_bounds__(kTriThreads) void eigh_tri_back_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ list,
    const double* __restrict__ Dold, double* __restrict__ C, const double* __restrict__ eps,
    double* __restrict__ Dnew, double* __restrict__ dD_max, int32_t* __restrict__ flags,
    double* __restrict__ ws_eig, int max_n) {
  constexpr int NC = kTriLanes * SEG;
  extern __shared__ double sm[];  // the packed reflectors, later the occupied block
  __shared__ double vbuf[2][NC];
  __shared__ double red[kTriThreads / 64];
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  const int n = fi.nbf;
  const TriWs W = tri_ws(ws_eig, max_n, n);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = kTriRowsPerWave * wave + lane / kTriLanes, seg = lane % kTriLanes;
  const int c0 = SEG * seg;
  const bool has_row = row < n;
  const int nrefl = n > 2 ? refl_off(n - 2, n) : 0;
  for (int i = threadIdx.x; i < nrefl; i += kTriThreads) sm[i] = W.refl[i];
  // z[c]: component c0 + c of eigenvector `row` of T
  double z[SEG];
#pragma unroll
  for (int c = 0; c < SEG; ++c) z[c] = 0.0;
  if (has_row) {
    const double* zr = W.Z + (size_t)row * (n + 64) + c0;
#pragma unroll
    for (int c = 0; c < SEG; ++c) z[c] = zr[c];
  }
  __syncthreads();
  // reflector k expanded over every column (zeros outside k+1 .. n-1) by
  // the helper wave into the buffer of its parity, one step ahead
  auto expand = [&](int k) {
    const double* vk = sm + refl_off(k, n) - (k + 1);
    double* dst = vbuf[k & 1];
    for (int j = lane; j < NC; j += 64) dst[j] = (j > k && j < n) ? vk[j] : 0.0;
  };
  if (wave == kTriHelper && n >= 3) expand(n - 3);
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    if (wave == kTriHelper && k >= 1) expand(k - 1);
    const double t = W.tau[k];
    const double* v = vbuf[k & 1];
    double dot = 0.0;
#pragma unroll
    for (int c = 0; c < SEG; ++c) dot = fma(v[c0 + c], z[c], dot);
    dot = t * pair_sum(dot);
    // read v again rather than keep SEG values of it live next to z
    asm volatile("" ::: "memory");
#pragma unroll
    for (int c = 0; c < SEG; ++c) z[c] -= dot * v[c0 + c];
    __syncthreads();
  }
  // C column `row` (ascending eigenvalue order)
  if (has_row) {
#pragma unroll
    for (int c = 0; c < SEG; ++c) {
      const int i = opaque(c0) + c;
      if (i < n) C[fi.off_C + (size_t)i * n + row] = z[c];
    }
  }
  // occupied columns into LDS (the reflectors are no longer needed), then
  // D = C_occ C_occ^T and max |D - D_old|
  const int nocc = fi.nocc;
  double* Co = sm;  // [nocc][n]
  if (has_row && row < nocc) {
#pragma unroll
    for (int c = 0; c < SEG; ++c) {
      const int i = opaque(c0) + c;
      if (i < n) Co[row * n + i] = z[c];
    }
  }
  __syncthreads();
  double dmax = 0.0;
  for (int e = threadIdx.x; e < n * n; e += kTriThreads) {
    const int l = e / n, s = e - (e / n) * n;
    double acc = 0.0;
    for (int k = 0; k < nocc; ++k) acc = fma(Co[k * n + l], Co[k * n + s], acc);
    Dnew[fi.off_C + e] = acc;
    dmax = fmax(dmax, fabs(acc - Dold[fi.off_C + e]));
  }
  dmax = block_max(dmax, red);
  if (threadIdx.x == 0) {
    atomic_max_nonneg(dD_max, dmax);
    const double* ev = eps + fi.off_eps;
    if (nocc > 0 && nocc < n && !(ev[nocc] > ev[nocc - 1])) atomicOr(flags, FEF_FLAG_GAP);
  }
}

hipError_t launch_eigh_tri(const fef_plan_s& p, const double* F, const double* Dold, double* C,
                           double* eps, double* Dnew, double* dD_max, int32_t* flags,
                           double* ws_eig, hipStream_t st) {
  const int nmax = p.eig_large_max_nbf;
  if (nmax > kTriMax) return hipErrorInvalidValue;
  int omax = 0;
  for (int32_t f : p.eig_large) omax = std::max(omax, p.frag[f].nocc);
  // back kernel: the packed reflectors, later the occupied block
  const size_t lds_back =
      std::max<size_t>((size_t)refl_off(std::max(nmax - 2, 0), nmax), (size_t)omax * nmax) *
      sizeof(double);
  const size_t lds_val = 4 * (size_t)nmax * sizeof(double);
  if (lds_back > 140 * 1024) return hipErrorInvalidValue;
  const dim3 grid((unsigned)p.eig_large.size());
#define FEF_TRI(S)                                                                             \
  {                                                                                            \
    static bool configured = false;                                                            \
    if (!configured) {                                                                         \
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&eigh_tri_back_kernel<S>),       \
                                hipFuncAttributeMaxDynamicSharedMemorySize, 140 * 1024);       \
      (void)hipGetLastError();                                                                 \
      configured = true;                                                                       \
    }                                                                                          \
    hipLaunchKernelGGL(eigh_tri_reduce_kernel<S>, grid, dim3(kTriThreads), 0, st, p.d_frag,    \
                       p.d_eig_large, F, ws_eig, nmax);                                        \
    hipLaunchKernelGGL(eigh_tri_values_kernel, grid, dim3(kTriThreads), lds_val, st, p.d_frag, \
                       p.d_eig_large, eps, ws_eig, nmax);                                      \
    hipLaunchKernelGGL(eigh_tri_back_kernel<S>, grid, dim3(kTriThreads), lds_back, st,        \
                       p.d_frag, p.d_eig_large, Dold, C, eps, Dnew, dD_max, flags, ws_eig,     \
                       nmax);                                                                  \
  }
  if (nmax <= 96) FEF_TRI(48) else FEF_TRI(76)
#undef FEF_TRI
  return hipGetLastError();
}

}  // namespace fef
