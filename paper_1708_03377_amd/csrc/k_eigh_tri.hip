// FP64 eigensolver for the large fragment Fock matrices (48 < n <= 152,
// the nucleobase-like solute): canonical orbitals of F~ ascending, Aufbau
// occupation, the new density and its change, as the Jacobi solvers.
//
// Four kernels; the reduction and the back-transformation run one
// 512-thread workgroup per matrix, so that they have the whole register
// file to themselves:
//   1. eigh_tri_reduce: Householder tridiagonalisation Q^T A Q = T
//      (A = (F + F^T) / 2).  For k = 0 .. n-3 the reflector
//      H_k = I - tau_k v_k v_k^T maps the part of row k right of the
//      diagonal onto its first entry; the trailing block takes the
//      symmetric rank-2 update A <- A - v w^T - w v^T with p = tau A v,
//      w = p - (tau / 2)(p . v) v.  A lives in registers, one row per two
//      lanes (lane s of a row holds columns 2 c + s, c < SEG), so that the
//      columns the shrinking trailing block leaves behind can be skipped in
//      groups by every lane alike.
//   2. eigh_tri_bisect: the eigenvalues of T by multisection on the Sturm
//      count (the number of negative pivots of the LDL^T factorisation of
//      T - x I): 16 lanes per eigenvalue count at 16 interior points,
//      shrinking the bracket 17-fold per round until it is a few ulps of
//      the eigenvalue (or of ||T|| near zero) wide; 16 eigenvalues per
//      workgroup, as many workgroups as needed.  Eigenvalue j is the
//      (j+1)-th smallest, so the order is ascending with ties in index
//      order.
//      eigh_tri_vectors: the eigenvectors of T by inverse iteration, one
//      thread per eigenvalue: Gaussian elimination with partial pivoting of
//      T - lambda I, three solves from a fixed pseudo-random start;
//      eigenvalues closer than 1e-3 ||T|| form a cluster that one thread
//      handles in order, each vector orthogonalised against the cluster's
//      earlier ones after every solve (modified Gram-Schmidt), a repeated
//      eigenvalue nudged by a few ulps first.
//   3. eigh_tri_back: back-transformation C = H_0 H_1 ... H_{n-3} Z, one
//      eigenvector per two lanes (components interleaved as the columns of
//      the reduction), four reflectors per step: for z <- H_{r_3} H_{r_2}
//      H_{r_1} H_{r_0} z (H_{r_0} first) the coefficients are
//      y_i = tau_i (v_i . z - sum_{j < i} (v_i . v_j) y_j), then
//      z <- z - sum_i y_i v_i; then C, the density and its change.
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
constexpr int kChunk = 4;  // register entries per skipped group (kTriLanes kChunk columns)
constexpr int kBackBlock = 4;  // reflectors applied per step of the back-transformation

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

// Reciprocal: the hardware approximation refined by one Newton step
// (relative error about 1e-16).
__device__ inline double tri_rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// Sturm count: the number of eigenvalues of T below x (negative pivots of
// T - x I = L D L^T), tiny pivots replaced by -pivmin.  Each pivot is
// formed with a few ulps of error, which makes the count exact for a T
// whose off-diagonal squares differ by a few ulps.
__device__ inline int sturm_count(const double* d, const double* e2, int n, double x,
                                  double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e2[i - 1] * tri_rcp(q);
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// Bound ||T|| >= max_i |d_i| + |e_{i-1}| + |e_i| and the Gershgorin interval.
struct TriNorm {
  double tn, lo, hi, e2max;
};
__device__ inline TriNorm tri_norm(const double* dg, const double* ee, int n) {
  TriNorm t{0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
    t.tn = fmax(t.tn, fabs(dg[i]) + r);
    t.lo = i == 0 ? dg[i] - r : fmin(t.lo, dg[i] - r);
    t.hi = i == 0 ? dg[i] + r : fmax(t.hi, dg[i] + r);
    t.e2max = fmax(t.e2max, ee[i] * ee[i]);
  }
  return t;
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
//   Z [n][n + 64] (row j = eigenvector j of T, zero past n); the reflector
//   blocks of the back-transformation expanded, VB [nb][kBackBlock]
//   [kTriVbStride], and their Gram entries GB [nb][16].
struct TriWs {
  double *d, *e, *tau, *refl, *Z, *VB, *GB;
};
__device__ inline int back_blocks(int n) { return n >= 3 ? (n - 2 + kBackBlock - 1) / kBackBlock : 0; }
__device__ inline TriWs tri_ws(double* ws_eig, int max_n, int n) {
  TriWs w;
  w.d = ws_eig + (size_t)blockIdx.x * eig_large_slot(max_n);
  w.e = w.d + n;
  w.tau = w.e + n;
  w.refl = w.tau + n;
  w.Z = w.refl + (n > 2 ? refl_off(n - 2, n) : 0);
  w.VB = w.Z + (size_t)n * (n + 64);
  w.GB = w.VB + (size_t)back_blocks(n) * kBackBlock * kTriVbStride;
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
  static_assert(SEG % kChunk == 0, "whole groups of skipped columns");
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
  const bool has_row = row < n;
  // first row of this wave: a wave whose rows all lie at or above the
  // reduced row k has no work in step k
  const int row0 = kTriRowsPerWave * wave;
  const double* Fx = F + fi.off_C;
  double a[SEG];
#pragma unroll
  for (int c = 0; c < SEG; ++c) a[c] = 0.0;
  if (has_row) {
#pragma unroll
    for (int c = 0; c < SEG; ++c) {
      const int j = opaque(seg) + kTriLanes * c;
      const int jc = j < n ? j : n - 1;  // every load in bounds, no branch
      const double v = 0.5 * (Fx[(size_t)row * n + jc] + Fx[(size_t)jc * n + row]);
      a[c] = j < n ? v : 0.0;
    }
  }
  for (int i = threadIdx.x; i < NC; i += kTriThreads) pb[i] = 0.0;
  if (row == 0) {
#pragma unroll
    for (int c = 0; c < SEG; ++c) xbuf[kTriLanes * c + seg] = a[c];
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
    // v and p vanish on columns <= k: groups of kChunk columns entirely
    // there are skipped (a test uniform over the workgroup)
    const bool live = t != 0.0 && row0 + kTriRowsPerWave - 1 > k && row0 < n;
    if (t != 0.0) {
      // p = tau A v over the trailing block (zero on rows <= k), p . v by waves
      double pr = 0.0, vr = 0.0;
      if (live) {
#pragma unroll
        for (int q = 0; q < SEG / kChunk; ++q)
          if (kTriLanes * kChunk * (q + 1) - 1 > k)
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
              pr = fma(a[kChunk * q + u], vc[kTriLanes * (kChunk * q + u) + seg], pr);
        pr = row > k ? t * pair_sum(pr) : 0.0;
        vr = has_row ? vc[row] : 0.0;
        if (has_row && seg == 0) pb[row] = pr;
      }
      const double pv = live ? wave_sum_dpp(seg == 0 ? pr * vr : 0.0) : 0.0;
      if (lane == 0) wpart[wave] = pv;
      __syncthreads();
      double sp = 0.0;
      for (int w = 0; w < kTriThreads / 64; ++w) sp += wpart[w];
      const double K = 0.5 * t * sp;
      // A <- A - v w^T - w v^T with w = p - K v; rows and columns outside the
      // trailing block have v = p = 0 and keep their values.  Two rounded
      // products and their sum (no contraction): entry (j, r) gets the same
      // two products, so A stays exactly symmetric.
      const double wr = pr - K * vr;
      if (live) {
#pragma clang fp contract(off)
#pragma unroll
        for (int q = 0; q < SEG / kChunk; ++q)
          if (kTriLanes * kChunk * (q + 1) - 1 > k)
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
              const int c = kChunk * q + u, j = kTriLanes * c + seg;
              const double vj = vc[j];
              const double wj = pb[j] - K * vj;
              a[c] -= vr * wj + wr * vj;
            }
      }
    }
    // the next row to reduce
    if (row == k + 1) {
#pragma unroll
      for (int c = 0; c < SEG; ++c) xbuf[kTriLanes * c + seg] = a[c];
    }
    __syncthreads();
  }
  // the last 2 x 2 block
  if (n >= 2 && (row == n - 2 || row == n - 1)) {
    double dd = 0.0, off = 0.0;
#pragma unroll
    for (int c = 0; c < SEG; ++c) {
      const int j = opaque(seg) + kTriLanes * c;
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
// 2a. eigenvalues of T (written to eps), kBisPer per workgroup
constexpr int kBisLanes = 16;  // interior points per eigenvalue and round
constexpr int kBisThreads = 256;
constexpr int kBisPer = kBisThreads / kBisLanes;

__global__ __launch_bounds__(kBisThreads) void eigh_tri_bisect_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ list,
    double* __restrict__ eps, double* __restrict__ ws_eig, int max_n) {
  extern __shared__ double sm[];  // d, e, e^2 [n] each
  __shared__ double sc[4];
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  const int n = fi.nbf;
  const int j0 = blockIdx.y * kBisPer;
  if (j0 >= n) return;  // uniform over the workgroup
  const TriWs W = tri_ws(ws_eig, max_n, n);
  double* dg = sm;
  double* ee = dg + n;
  double* e2 = ee + n;
  for (int i = threadIdx.x; i < n; i += kBisThreads) {
    dg[i] = W.d[i];
    ee[i] = i + 1 < n ? W.e[i] : 0.0;
    e2[i] = ee[i] * ee[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const TriNorm t = tri_norm(dg, ee, n);
    const double pivmin = 1e-290 * fmax(1.0, t.e2max);
    const double pad = 2.0 * DBL_EPSILON * t.tn + 2.0 * pivmin;
    sc[0] = t.lo - pad;
    sc[1] = t.hi + pad;
    sc[2] = t.tn;
    sc[3] = pivmin;
  }
  __syncthreads();
  // eigenvalue j (the (j+1)-th smallest) by a group of kBisLanes lanes: each
  // counts at one of kBisLanes interior points that cut the bracket into
  // kBisLanes + 1 equal parts; the new bracket runs from the last point
  // below the eigenvalue to the first at or above it.  A bracket a few ulps
  // of the eigenvalue (or of ||T|| near zero) wide ends the search.
  const int j = j0 + (int)threadIdx.x / kBisLanes, m = (int)threadIdx.x % kBisLanes;
  const int gsh = (int)(threadIdx.x & 63) & ~(kBisLanes - 1);
  if (j < n) {  // uniform over each group of lanes
    const double pivmin = sc[3], tn = sc[2];
    double lo = sc[0], hi = sc[1];
    for (int it = 0; it < 100; ++it) {
      if (!(hi - lo > 2.0 * DBL_EPSILON * (fmax(fabs(lo), fabs(hi)) + tn) + 2.0 * pivmin)) break;
      const double w = (hi - lo) * (1.0 / (kBisLanes + 1));
      const double x = lo + (double)(m + 1) * w;
      const int cnt = sturm_count(dg, e2, n, x, pivmin);
      const uint64_t ball = __ballot(cnt >= j + 1);
      const uint32_t g = (uint32_t)(ball >> gsh) & ((1u << kBisLanes) - 1);
      const int first = g ? __builtin_ctz(g) : kBisLanes;
      const double nlo = first == 0 ? lo : lo + (double)first * w;
      const double nhi = first == kBisLanes ? hi : lo + (double)(first + 1) * w;
      lo = nlo;
      hi = nhi;
    }
    if (m == 0) eps[fi.off_eps + j] = 0.5 * (lo + hi);
  }
}

// ---------------------------------------------------------------------------
// 2b. eigenvectors of T by inverse iteration, one thread per cluster, its
// work vectors in LDS
constexpr int kVecThreads = 16;
constexpr int kVecBatch = 8;  // recurrence steps whose operands load together

// dynamic LDS bytes: d, e, lambda [n]; five work vectors and the row
// interchange flags [n][kVecThreads], interleaved over the threads
__host__ __device__ inline size_t vec_lds_bytes(int n) {
  return (size_t)(3 * n + 5 * n * kVecThreads) * sizeof(double) + (size_t)n * kVecThreads;
}

__global__ __launch_bounds__(64) void eigh_tri_vectors_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ list,
    const double* __restrict__ eps, double* __restrict__ ws_eig, int max_n) {
  extern __shared__ double sm[];
  __shared__ double s_tn;
  constexpr int T = kVecThreads;
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  const int n = fi.nbf;
  if ((int)blockIdx.y * T >= n) return;  // uniform over the workgroup
  const TriWs W = tri_ws(ws_eig, max_n, n);
  double* dg = sm;
  double* ee = dg + n;
  double* lam = ee + n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    dg[i] = W.d[i];
    ee[i] = i + 1 < n ? W.e[i] : 0.0;
    lam[i] = eps[fi.off_eps + i];
  }
  __syncthreads();
  if (threadIdx.x == 0) s_tn = tri_norm(dg, ee, n).tn;
  __syncthreads();
  const int t = (int)threadIdx.x;
  const int j = (int)blockIdx.y * T + t;
  if (t >= T || j >= n) return;
  const int ld = n + 64;
  const double tn = s_tn;
  const double ortol = 1e-3 * tn, tiny = DBL_EPSILON * fmax(tn, 1e-300);
  // eigenvalues closer than ortol form a cluster; its first index leads it
  if (!(j == 0 || lam[j] - lam[j - 1] > ortol)) return;
  int j1 = j;
  while (j1 + 1 < n && lam[j1 + 1] - lam[j1] <= ortol) ++j1;
  // this thread's work vectors, interleaved with the other threads' (entry
  // i of a vector at i T + t), so that threads stepping through their
  // recurrences together touch neighbouring banks
  const size_t sv = (size_t)n * T;
  double* const ra = lam + n + t;  // 1 / (diagonal of U)
  double* const ub = ra + sv;      // first superdiagonal of U
  double* const ud = ub + sv;      // second superdiagonal of U
  double* const ml = ud + sv;      // multipliers
  double* const xv = ml + sv;      // iterate
  unsigned char* const pv = reinterpret_cast<unsigned char*>(lam + n + 5 * sv) + t;  // 1: rows i, i+1 interchanged
  auto at = [](double* v, int i) -> double& { return v[i * T]; };
  auto swp = [pv](int i) -> unsigned char& { return pv[i * T]; };
  double prev = 0.0;
  for (int jj = j; jj <= j1; ++jj) {
    double lm = lam[jj];
    if (jj > j && lm - prev < 10.0 * DBL_EPSILON * fabs(lm))
      lm = prev + 10.0 * DBL_EPSILON * fabs(lm);
    prev = lm;
    // T - lm I = P L U with row interchanges between neighbours; the
    // current row's diagonal and superdiagonal ride in registers
    {
      double ak = dg[0] - lm, bk = n > 1 ? ee[0] : 0.0;
      for (int k = 0; k + 1 < n; ++k) {
        const double ck = ee[k];
        double ak1 = dg[k + 1] - lm, bk1 = k + 2 < n ? ee[k + 1] : 0.0;
        // pivots below tiny are replaced by +-tiny (as a singular T - lm I
        // would otherwise stop the solve)
        auto guard = [tiny](double v) { return fabs(v) < tiny ? (v < 0.0 ? -tiny : tiny) : v; };
        double piv, b, d, l;
        if (fabs(ak) >= fabs(ck)) {
          piv = guard(ak);
          l = ck * tri_rcp(piv);
          b = bk;
          d = 0.0;
          swp(k) = 0;
          ak1 -= l * bk;
        } else {
          piv = guard(ck);
          l = ak * tri_rcp(ck);
          b = ak1;
          d = bk1;
          swp(k) = 1;
          const double na = bk - l * ak1;
          bk1 = -l * bk1;
          ak1 = na;
        }
        at(ra, k) = tri_rcp(piv);
        at(ub, k) = b;
        at(ud, k) = d;
        at(ml, k) = l;
        ak = ak1;
        bk = bk1;
      }
      at(ra, n - 1) = tri_rcp(fabs(ak) < tiny ? (ak < 0.0 ? -tiny : tiny) : ak);  // last pivot
      at(ub, n - 1) = 0.0;
      at(ud, n - 1) = 0.0;
    }
    for (int i = 0; i < n; ++i) at(xv, i) = start_entry(jj, i);
    for (int itn = 0; itn < 3; ++itn) {
      double mx = 0.0;
#pragma unroll 8
      for (int i = 0; i < n; ++i) mx = fmax(mx, fabs(at(xv, i)));
      const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
      // forward: the row interchanges and multipliers, kVecBatch steps'
      // operands loaded ahead of their serial updates
      double xk = at(xv, 0) * inv;
      for (int k0 = 0; k0 + 1 < n; k0 += kVecBatch) {
        double xl[kVecBatch], ll[kVecBatch];
        bool pl[kVecBatch];
#pragma unroll
        for (int u = 0; u < kVecBatch; ++u) {
          const int k = min(k0 + u, n - 2);
          xl[u] = at(xv, k + 1);
          ll[u] = at(ml, k);
          pl[u] = swp(k) != 0;
        }
#pragma unroll
        for (int u = 0; u < kVecBatch; ++u) {
          const int k = k0 + u;
          if (k + 1 < n) {
            double x1 = xl[u] * inv;
            if (pl[u]) {
              const double t = xk;
              xk = x1;
              x1 = t;
            }
            x1 -= ll[u] * xk;
            at(xv, k) = xk;
            xk = x1;
          }
        }
      }
      at(xv, n - 1) = xk;
      // backward: U x = y
      double x1 = 0.0, x2 = 0.0;  // x(k + 1), x(k + 2)
      for (int k0 = n - 1; k0 >= 0; k0 -= kVecBatch) {
        double yl[kVecBatch], bl[kVecBatch], dl[kVecBatch], rl[kVecBatch];
#pragma unroll
        for (int u = 0; u < kVecBatch; ++u) {
          const int k = max(k0 - u, 0);
          yl[u] = at(xv, k);
          bl[u] = at(ub, k);
          dl[u] = at(ud, k);
          rl[u] = at(ra, k);
        }
#pragma unroll
        for (int u = 0; u < kVecBatch; ++u) {
          const int k = k0 - u;
          if (k >= 0) {
            const double xv_ = (yl[u] - bl[u] * x1 - dl[u] * x2) * rl[u];
            at(xv, k) = xv_;
            x2 = x1;
            x1 = xv_;
          }
        }
      }
      for (int q = j; q < jj; ++q) {
        const double* zq = W.Z + (size_t)q * ld;
        // four partial sums (added in a fixed order) break the chain
        double d4[4] = {0.0, 0.0, 0.0, 0.0};
        int i = 0;
        for (; i + 4 <= n; i += 4)
#pragma unroll
          for (int u = 0; u < 4; ++u) d4[u] = fma(zq[i + u], at(xv, i + u), d4[u]);
        for (; i < n; ++i) d4[0] = fma(zq[i], at(xv, i), d4[0]);
        const double dot = (d4[0] + d4[1]) + (d4[2] + d4[3]);
#pragma unroll 8
        for (int i2 = 0; i2 < n; ++i2) at(xv, i2) -= dot * zq[i2];
      }
      double nrm = 0.0;
#pragma unroll 8
      for (int i = 0; i < n; ++i) nrm = fma(at(xv, i), at(xv, i), nrm);
      const double r = 1.0 / sqrt(nrm);
#pragma unroll 8
      for (int i = 0; i < n; ++i) at(xv, i) *= r;
    }
    double* zj = W.Z + (size_t)jj * ld;
#pragma unroll 8
    for (int i = 0; i < n; ++i) zj[i] = at(xv, i);
    for (int i = n; i < ld; ++i) zj[i] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// 3. back-transformation and outputs
//
// The eigenvectors z of T go back through the reflectors, C = H_0 H_1 ...
// H_{n-3} Z, four reflectors per step.  Block b holds reflectors r_i = k0 -
// i, i < kBackBlock, k0 = n - 3 - kBackBlock b, applied in the order r_0,
// r_1, ... (H_{r_0} first); a reflector index below 0 is a zero vector with
// tau = 0.  With the Gram entries g_ij = v_i . v_j (i > j) and g_ii = tau_i,
// the block maps z to z - sum_i y_i v_i with
//   y_i = tau_i (v_i . z - sum_{j < i} g_ij y_j).
// (a) eigh_tri_expand_kernel: one wave per block writes the expanded
//     vectors (zeros outside r_i + 1 .. n - 1) and the Gram entries;
// (b) eigh_tri_back_kernel: one wave per 32 eigenvectors (two lanes per
//     eigenvector, as in the vector kernel) streams the blocks through LDS
//     (the next block's copy issued before the current one is applied) and
//     writes its columns of C;
// (c) eigh_tri_density_kernel: D = C_occ C_occ^T, max |D - D_old| and the
//     gap flag.
template <int SEG>
__global__ __launch_bounds__(64) void eigh_tri_expand_kernel(const FragInfo* __restrict__ frag,
                                                             const int32_t* __restrict__ list,
                                                             double* __restrict__ ws_eig,
                                                             int max_n) {
  constexpr int NC = kTriLanes * SEG;
  static_assert(NC <= kTriVbStride, "expanded reflector stride");
  const int n = frag[list[blockIdx.x]].nbf;
  const int b = blockIdx.y;
  if (b >= back_blocks(n)) return;
  const TriWs W = tri_ws(ws_eig, max_n, n);
  const int lane = threadIdx.x;
  const int k0 = n - 3 - kBackBlock * b;
  double* dst = W.VB + (size_t)b * kBackBlock * kTriVbStride;
  double* g = W.GB + (size_t)b * 16;
  double vv[kBackBlock][(NC + 63) / 64];
#pragma unroll
  for (int i = 0; i < kBackBlock; ++i) {
    const int k = k0 - i;
    const double* vk = W.refl + (k >= 0 ? refl_off(k, n) - (k + 1) : 0);
#pragma unroll
    for (int u = 0; u < (NC + 63) / 64; ++u) {
      const int j = lane + 64 * u;
      const double x = (k >= 0 && j > k && j < n) ? vk[j] : 0.0;
      vv[i][u] = x;
      if (j < NC) dst[i * kTriVbStride + j] = x;
    }
  }
#pragma unroll
  for (int i = 1; i < kBackBlock; ++i)
#pragma unroll
    for (int jj = 0; jj < i; ++jj) {
      double d = 0.0;
#pragma unroll
      for (int u = 0; u < (NC + 63) / 64; ++u)
        if (lane + 64 * u < NC) d = fma(vv[i][u], vv[jj][u], d);
      d = wave_sum_dpp(d);
      if (lane == 0) g[i * kBackBlock + jj] = d;
    }
  if (lane < kBackBlock) {
    const int k = k0 - lane;
    g[lane * kBackBlock + lane] = k >= 0 ? W.tau[k] : 0.0;
  }
}

template <int SEG>
__global__ __launch_bounds__(64) void eigh_tri_back_kernel(const FragInfo* __restrict__ frag,
                                                           const int32_t* __restrict__ list,
                                                           double* __restrict__ C,
                                                           double* __restrict__ ws_eig,
                                                           int max_n) {
  constexpr int NC = kTriLanes * SEG;
  constexpr int BLK = kBackBlock * kTriVbStride + 16;  // doubles of one staged block
  __shared__ __align__(16) double buf[2][BLK];
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  const int n = fi.nbf;
  const TriWs W = tri_ws(ws_eig, max_n, n);
  const int lane = threadIdx.x;
  const int row = kTriRowsPerWave * blockIdx.y + lane / kTriLanes, seg = lane % kTriLanes;
  if (kTriRowsPerWave * blockIdx.y >= n) return;
  const bool has_row = row < n;
  // z[c]: component 2 c + seg of eigenvector `row` of T
  double z[SEG];
#pragma unroll
  for (int c = 0; c < SEG; ++c) z[c] = 0.0;
  if (has_row) {
    const double* zr = W.Z + (size_t)row * (n + 64) + seg;
#pragma unroll
    for (int c = 0; c < SEG; ++c) z[c] = zr[kTriLanes * c];
  }
  const int nb = back_blocks(n);
  // block b's vectors and Gram entries into buf[b & 1] (whole-wave copies)
  auto stage = [&](int b) __attribute__((always_inline)) {
    const double* v = W.VB + (size_t)b * kBackBlock * kTriVbStride;
    const double* g = W.GB + (size_t)b * 16;
    double* d = buf[b & 1];
    for (int e = lane; e < kBackBlock * kTriVbStride; e += 64) d[e] = v[e];
    if (lane < 16) d[kBackBlock * kTriVbStride + lane] = g[lane];
  };
  if (nb > 0) stage(0);
  __syncthreads();
  for (int b = 0; b < nb; ++b) {
    // the next block's loads are issued first; their LDS writes land after
    // this block's reads (the barrier below)
    double nxt[(kBackBlock * kTriVbStride + 63) / 64];
    double gn = 0.0;
    const bool more = b + 1 < nb;
    if (more) {
      const double* v = W.VB + (size_t)(b + 1) * kBackBlock * kTriVbStride;
#pragma unroll
      for (int u = 0; u < (kBackBlock * kTriVbStride + 63) / 64; ++u) {
        const int e = lane + 64 * u;
        nxt[u] = e < kBackBlock * kTriVbStride ? v[e] : 0.0;
      }
      if (lane < 16) gn = W.GB[(size_t)(b + 1) * 16 + lane];
    }
    const int kmin = n - 3 - kBackBlock * b - (kBackBlock - 1);  // every v_i vanishes on <= kmin
    const double* v = buf[b & 1];
    const double* g = v + kBackBlock * kTriVbStride;
    // w_i = v_i . z; groups of kChunk components entirely at or below kmin
    // are skipped (a test uniform over the wave)
    double w[kBackBlock];
#pragma unroll
    for (int i = 0; i < kBackBlock; ++i) w[i] = 0.0;
#pragma unroll
    for (int q = 0; q < SEG / kChunk; ++q)
      if (kTriLanes * kChunk * (q + 1) - 1 > kmin)
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          const int c = kChunk * q + u, j = kTriLanes * c + seg;
#pragma unroll
          for (int i = 0; i < kBackBlock; ++i) w[i] = fma(v[i * kTriVbStride + j], z[c], w[i]);
        }
    // y_i = tau_i (w_i - sum_{j < i} g_ij y_j): H_{r_0} first, then H_{r_1}, ...
    double y[kBackBlock];
#pragma unroll
    for (int i = 0; i < kBackBlock; ++i) {
      double a = pair_sum(w[i]);
#pragma unroll
      for (int jj = 0; jj < i; ++jj) a -= g[i * kBackBlock + jj] * y[jj];
      y[i] = g[i * kBackBlock + i] * a;
    }
#pragma unroll
    for (int q = 0; q < SEG / kChunk; ++q)
      if (kTriLanes * kChunk * (q + 1) - 1 > kmin)
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          const int c = kChunk * q + u, j = kTriLanes * c + seg;
          double zc = z[c];
#pragma unroll
          for (int i = 0; i < kBackBlock; ++i) zc -= y[i] * v[i * kTriVbStride + j];
          z[c] = zc;
        }
    __syncthreads();
    if (more) {
      double* d = buf[(b + 1) & 1];
#pragma unroll
      for (int u = 0; u < (kBackBlock * kTriVbStride + 63) / 64; ++u) {
        const int e = lane + 64 * u;
        if (e < kBackBlock * kTriVbStride) d[e] = nxt[u];
      }
      if (lane < 16) d[kBackBlock * kTriVbStride + lane] = gn;
    }
    __syncthreads();
  }
  // C column `row` (ascending eigenvalue order)
  if (has_row) {
#pragma unroll
    for (int c = 0; c < SEG; ++c) {
      const int i = opaque(seg) + kTriLanes * c;
      if (i < n) C[fi.off_C + (size_t)i * n + row] = z[c];
    }
  }
}

__global__ __launch_bounds__(256) void eigh_tri_density_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ list,
    const double* __restrict__ Dold, const double* __restrict__ C,
    const double* __restrict__ eps, double* __restrict__ Dnew, double* __restrict__ dD_max,
    int32_t* __restrict__ flags) {
  __shared__ double red[4];
  const FragInfo fi = frag[list[blockIdx.x]];
  const int n = fi.nbf, nocc = fi.nocc;
  const double* Cf = C + fi.off_C;
  double dmax = 0.0;
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e < n * n) {
    const int l = e / n, s = e - (e / n) * n;
    double acc = 0.0;
    for (int k = 0; k < nocc; ++k) acc = fma(Cf[(size_t)l * n + k], Cf[(size_t)s * n + k], acc);
    Dnew[fi.off_C + e] = acc;
    dmax = fabs(acc - Dold[fi.off_C + e]);
  }
  dmax = block_max(dmax, red);
  if (threadIdx.x == 0) {
    atomic_max_nonneg(dD_max, dmax);
    const double* ev = eps + fi.off_eps;
    if (blockIdx.y == 0 && nocc > 0 && nocc < n && !(ev[nocc] > ev[nocc - 1]))
      atomicOr(flags, FEF_FLAG_GAP);
  }
}

hipError_t launch_eigh_tri(const fef_plan_s& p, const double* F, const double* Dold, double* C,
                           double* eps, double* Dnew, double* dD_max, int32_t* flags,
                           double* ws_eig, hipStream_t st) {
  const int nmax = p.eig_large_max_nbf;
  if (nmax > kTriMax) return hipErrorInvalidValue;
  const size_t lds_bis = 3 * (size_t)nmax * sizeof(double);
  const size_t lds_vec = vec_lds_bytes(nmax);
  if (lds_vec > 150 * 1024) return hipErrorInvalidValue;
  {
    static bool configured = false;
    if (!configured) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&eigh_tri_vectors_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
      (void)hipGetLastError();
      configured = true;
    }
  }
  const dim3 grid((unsigned)p.eig_large.size());
  const dim3 grid_bis(grid.x, (unsigned)((nmax + kBisPer - 1) / kBisPer));
  const dim3 grid_vec(grid.x, (unsigned)((nmax + kVecThreads - 1) / kVecThreads));
  const int nbmax = nmax >= 3 ? (nmax - 2 + kBackBlock - 1) / kBackBlock : 0;
  const dim3 grid_exp(grid.x, (unsigned)std::max(nbmax, 1));
  const dim3 grid_back(grid.x, (unsigned)((nmax + kTriRowsPerWave - 1) / kTriRowsPerWave));
  const dim3 grid_den(grid.x, (unsigned)((nmax * nmax + 255) / 256));
#define FEF_TRI(S)                                                                             \
  {                                                                                            \
    hipLaunchKernelGGL(eigh_tri_reduce_kernel<S>, grid, dim3(kTriThreads), 0, st, p.d_frag,    \
                       p.d_eig_large, F, ws_eig, nmax);                                        \
    hipLaunchKernelGGL(eigh_tri_bisect_kernel, grid_bis, dim3(kBisThreads), lds_bis, st,       \
                       p.d_frag, p.d_eig_large, eps, ws_eig, nmax);                            \
    hipLaunchKernelGGL(eigh_tri_vectors_kernel, grid_vec, dim3(64), lds_vec, st, p.d_frag,     \
                       p.d_eig_large, eps, ws_eig, nmax);                                      \
    hipLaunchKernelGGL(eigh_tri_expand_kernel<S>, grid_exp, dim3(64), 0, st, p.d_frag,         \
                       p.d_eig_large, ws_eig, nmax);                                           \
    hipLaunchKernelGGL(eigh_tri_back_kernel<S>, grid_back, dim3(64), 0, st, p.d_frag,          \
                       p.d_eig_large, C, ws_eig, nmax);                                        \
    hipLaunchKernelGGL(eigh_tri_density_kernel, grid_den, dim3(256), 0, st, p.d_frag,          \
                       p.d_eig_large, Dold, C, eps, Dnew, dD_max, flags);                      \
  }
  if (nmax <= 96) FEF_TRI(48) else FEF_TRI(76)
#undef FEF_TRI
  return hipGetLastError();
}

}  // namespace fef
