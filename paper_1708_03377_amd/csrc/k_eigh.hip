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
// Sweeps stop when ||offdiag(A)||_F <= 1e-12 ||diag(A)||_2 (at most 40):
// eigenvalue errors are then second order in that bound, eigenvector
// errors first order, about 1e-12 ||A|| / gap.
// One workgroup per matrix; the matrix and eigenvectors live in LDS for
// n <= 48 and in a global workspace slot otherwise.  Each round makes two
// passes: the rotation table, then every 2x2 block of A (rows of one pair,
// columns of another: A_blk <- R_k^T A_blk R_l) together with V <- V J.
#include "fef_internal.h"
#include "fef_device.h"

namespace fef {

// Rotation (c, s) that zeroes a_pq of the 2x2 block [[a_pp, a_pq], [a_pq, a_qq]]
// (classical symmetric Schur step).  Reciprocal and reciprocal square root
// come from the hardware approximations refined by one Newton step each
// (relative error ~1e-16); the rotation only has to zero a_pq to rounding
// level, while c^2 + s^2 = 1 holds to rounding because s = t c exactly.
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ inline double rsq_nr(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  return r * fma(-0.5 * x * r, r, 1.5);
}
__device__ inline void jacobi_rotation(double app, double aqq, double apq, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (apq == 0.0) return;
  const double tau = (aqq - app) * 0.5 * rcp_nr(apq);
  double t;
  if (fabs(tau) > 1e150) {
    t = 0.5 * rcp_nr(tau);
  } else {
    const double q = 1.0 + tau * tau;
    const double sq = q * rsq_nr(q);  // sqrt(1 + tau^2)
    t = (tau >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(tau) + sq);
  }
  c = rsq_nr(1.0 + t * t);
  s = t * c;
}

// Pair k of round r in the circle ordering of m (even) indices, p < q.
__device__ inline void round_robin_pair(int r, int k, int m, int& p, int& q) {
  const int m1 = m - 1;
  if (k == 0) {
    p = r;
    q = m1;
  } else {
    p = r + k;
    if (p >= m1) p -= m1;
    q = r - k;
    if (q < 0) q += m1;
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// kNmax > 0: matrices up to kNmax, held in LDS with stride kNmax + 1, index
// decode by constant divisors, warm start from the input orbitals.
// kNmax == 0: any size, matrices in a global workspace slot with stride m,
// cold start from the identity.
//
// Warm start: with C the input orbitals (orthonormal columns), the solver
// diagonalises A = C^T F C and accumulates V = C J_1 J_2 ..., so V ends as the
// eigenvectors of F in the AO basis.  Near self-consistency A is nearly
// diagonal and fewer sweeps are needed; the spectrum is the same for any
// orthonormal C.
template <int NT, int kNmax>
__global__ __launch_bounds__(NT) void eigh_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ list,
    const double* __restrict__ F, const double* __restrict__ Dold, double* __restrict__ C,
    double* __restrict__ eps, double* __restrict__ Dnew, double* __restrict__ dD_max,
    int32_t* __restrict__ flags, double* __restrict__ ws_eig, int max_n) {
  constexpr bool kLds = kNmax > 0;
  constexpr int kH = kNmax / 2;
  constexpr int kNB = kLds ? (kH * kH + NT - 1) / NT : 1;       // blocks per thread
  constexpr int kNV = kLds ? (kNmax * kH + NT - 1) / NT : 1;    // V pairs per thread
  extern __shared__ double sm[];
  __shared__ double red[NT / 64];
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  const int n = fi.nbf;
  const int m = n + (n & 1);  // an odd n gets a dummy index n (zero row/column)
  const int half = m / 2;
  const int lda = kLds ? kNmax + 1 : m;
  double *A, *V, *cs;
  if (kLds) {
    A = sm;
    V = sm + kNmax * (kNmax + 1);
    cs = V + kNmax * (kNmax + 1);
  } else {
    const size_t slot = (size_t)(max_n + 1) * (max_n + 1);
    A = ws_eig + (size_t)blockIdx.x * 2 * slot;
    V = A + slot;
    cs = sm;
  }
  double* cc = cs;
  double* ss = cs + half;
  int* pp = reinterpret_cast<int*>(ss + half);
  int* qq = pp + half;
  int* rank = qq + half;
  double* lam = reinterpret_cast<double*>(rank + 2 * ((n + 1) / 2));
  double* T = lam + (n + 1);  // warm-start scratch (LDS path), [kNmax][kNmax + 1]

  const double* Fx = F + fi.off_C;
  const double* Cx = C + fi.off_C;
  for (int e = threadIdx.x; e < m * m; e += NT) {
    const int i = e / m, j = e - (e / m) * m;
    const bool in = i < n && j < n;
    A[i * lda + j] = in ? 0.5 * (Fx[i * n + j] + Fx[j * n + i]) : 0.0;
    V[i * lda + j] = kLds ? (in ? Cx[i * n + j] : 0.0) : ((in && i == j) ? 1.0 : 0.0);
  }
  __syncthreads();
  if (kLds) {
    // T = F C, then A = C^T T
    for (int e = threadIdx.x; e < n * n; e += NT) {
      const int i = e / n, j = e - (e / n) * n;
      double acc = 0.0;
      for (int k = 0; k < n; ++k) acc = fma(A[i * lda + k], V[k * lda + j], acc);
      T[i * lda + j] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += NT) {
      const int i = e / n, j = e - (e / n) * n;
      double acc = 0.0;
      for (int k = 0; k < n; ++k) acc = fma(V[k * lda + i], T[k * lda + j], acc);
      A[i * lda + j] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += NT) {  // exact symmetry
      const int i = e / n, j = e - (e / n) * n;
      if (i < j) {
        const double a = 0.5 * (A[i * lda + j] + A[j * lda + i]);
        A[i * lda + j] = a;
        A[j * lda + i] = a;
      }
    }
    __syncthreads();
  }

  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = threadIdx.x; e < n * n; e += NT) {
      const int i = e / n, j = e - (e / n) * n;
      const double a = A[i * lda + j];
      if (i == j) dia += a * a; else off += a * a;
    }
    off = block_sum(off, red);
    dia = block_sum(dia, red);
    if (off <= 1e-24 * dia || !(off == off)) break;
    for (int r = 0; r < m - 1; ++r) {
      for (int k = threadIdx.x; k < half; k += NT) {
        int p, q;
        round_robin_pair(r, k, m, p, q);
        double c, s;
        jacobi_rotation(A[p * lda + p], A[q * lda + q], A[p * lda + q], c, s);
        cc[k] = c;
        ss[k] = s;
        pp[k] = p;
        qq[k] = q;
      }
      __syncthreads();
      if (kLds) {
        // every 2x2 block (rows of pair k, columns of pair l) and every V
        // row pair: all loads first, then the arithmetic, then all stores
        double mb[kNB][4], vb[kNV][2];
        int ab[kNB][4], av[kNV][2];
        double cb[kNB][4], cv[kNV][2];
        bool ok[kNB], okv[kNV];
#pragma unroll
        for (int u = 0; u < kNB; ++u) {
          const int b = threadIdx.x + NT * u;
          const int k = b / kH, l = b - (b / kH) * kH;
          ok[u] = b < kH * kH && k < half && l < half;
          const int a0 = ok[u] ? pp[k] : 0, a1 = ok[u] ? qq[k] : 0;
          const int b0 = ok[u] ? pp[l] : 0, b1 = ok[u] ? qq[l] : 0;
          ab[u][0] = a0 * lda + b0; ab[u][1] = a0 * lda + b1;
          ab[u][2] = a1 * lda + b0; ab[u][3] = a1 * lda + b1;
          cb[u][0] = ok[u] ? cc[k] : 1.0; cb[u][1] = ok[u] ? ss[k] : 0.0;
          cb[u][2] = ok[u] ? cc[l] : 1.0; cb[u][3] = ok[u] ? ss[l] : 0.0;
#pragma unroll
          for (int z = 0; z < 4; ++z) mb[u][z] = A[ab[u][z]];
        }
#pragma unroll
        for (int u = 0; u < kNV; ++u) {
          const int e = threadIdx.x + NT * u;
          const int l = e / kNmax, i = e - (e / kNmax) * kNmax;
          okv[u] = e < kNmax * kH && i < n && l < half;
          const int p = okv[u] ? pp[l] : 0, q = okv[u] ? qq[l] : 0;
          const int row = okv[u] ? i : 0;
          av[u][0] = row * lda + p;
          av[u][1] = row * lda + q;
          cv[u][0] = okv[u] ? cc[l] : 1.0;
          cv[u][1] = okv[u] ? ss[l] : 0.0;
          vb[u][0] = V[av[u][0]];
          vb[u][1] = V[av[u][1]];
        }
#pragma unroll
        for (int u = 0; u < kNB; ++u) {
          const double ck = cb[u][0], sk = cb[u][1], cl = cb[u][2], sl = cb[u][3];
          const double t00 = ck * mb[u][0] - sk * mb[u][2], t01 = ck * mb[u][1] - sk * mb[u][3];
          const double t10 = sk * mb[u][0] + ck * mb[u][2], t11 = sk * mb[u][1] + ck * mb[u][3];
          mb[u][0] = cl * t00 - sl * t01;
          mb[u][1] = sl * t00 + cl * t01;
          mb[u][2] = cl * t10 - sl * t11;
          mb[u][3] = sl * t10 + cl * t11;
        }
#pragma unroll
        for (int u = 0; u < kNV; ++u) {
          const double c = cv[u][0], s = cv[u][1], vp = vb[u][0], vq = vb[u][1];
          vb[u][0] = c * vp - s * vq;
          vb[u][1] = s * vp + c * vq;
        }
#pragma unroll
        for (int u = 0; u < kNB; ++u)
          if (ok[u]) {
#pragma unroll
            for (int z = 0; z < 4; ++z) A[ab[u][z]] = mb[u][z];
          }
#pragma unroll
        for (int u = 0; u < kNV; ++u)
          if (okv[u]) {
            V[av[u][0]] = vb[u][0];
            V[av[u][1]] = vb[u][1];
          }
      } else {
        for (int b = threadIdx.x; b < half * half; b += NT) {
          const int k = b / half, l = b - (b / half) * half;
          const int a = pp[k], bb = qq[k], c = pp[l], d = qq[l];
          const double ck = cc[k], sk = ss[k], cl = cc[l], sl = ss[l];
          const double m00 = A[a * lda + c], m01 = A[a * lda + d];
          const double m10 = A[bb * lda + c], m11 = A[bb * lda + d];
          const double t00 = ck * m00 - sk * m10, t01 = ck * m01 - sk * m11;
          const double t10 = sk * m00 + ck * m10, t11 = sk * m01 + ck * m11;
          A[a * lda + c] = cl * t00 - sl * t01;
          A[a * lda + d] = sl * t00 + cl * t01;
          A[bb * lda + c] = cl * t10 - sl * t11;
          A[bb * lda + d] = sl * t10 + cl * t11;
        }
        for (int e = threadIdx.x; e < n * half; e += NT) {
          const int l = e / n, i = e - (e / n) * n;
          const int p = pp[l], q = qq[l];
          const double c = cc[l], s = ss[l];
          const double vp = V[i * lda + p], vq = V[i * lda + q];
          V[i * lda + p] = c * vp - s * vq;
          V[i * lda + q] = s * vp + c * vq;
        }
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

// ---------------------------------------------------------------------------
// Register-resident Jacobi for n <= 32: two matrices per wave, one per half
// (32 lanes).  Matrix size M (even, >= n; indices n..M-1 are decoupled zero
// rows/columns).  Lane t of a half holds row t of A and row t of V (AO row t)
// in registers, columns in "slot" order.  In every round the pairs are the
// slots (2k, 2k+1): each lane pair computes its rotation, the rotations are
// broadcast through LDS for the column updates (A <- A J, V <- V J, register
// pairs), and the row update (A <- J^T A) swaps rows between the two lanes of
// a pair with DPP.  Then the slots are relabelled by the circle-method
// permutation pi (a fixed slot stays, the others move one place round a
// circle), applied to A's rows (ds_bpermute straight into the permuted
// registers) and to the columns of A and V.  Over the M - 1 rounds of a
// sweep every pair of indices meets once and pi^(M-1) is the identity, so at
// the start of every sweep slot j holds index j again.  Same rotation
// formula, warm start (A = C^T F C, V = C) and stopping rule as above.
template <int M>
struct SlotPerm {
  // pi(s): the slot the contents of slot s move to after a round
  static constexpr int pi(int s) {
    return s == 0 ? 0
         : s == 1 ? (M > 2 ? 2 : 1)
         : (s % 2 == 0) ? (s / 2 + 1 <= M / 2 - 1 ? s + 2 : M - 1)
                        : (s / 2 >= 2 ? s - 2 : 1);
  }
  static constexpr int inv(int j) {
    int r = 0;
    for (int s = 0; s < M; ++s)
      if (pi(s) == j) r = s;
    return r;
  }
};

__device__ inline double dpp_swap_pair(double x) {  // value of lane ^ 1
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double bperm_d(int byte_addr, double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_bpermute(byte_addr, (int)b);
  const int hi = __builtin_amdgcn_ds_bpermute(byte_addr, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Bounded to two waves per SIMD (at most 256 registers): the 4000-matrix
// batches then fit on the chip at once, and the two waves of a SIMD hide
// each other's latency in the round's dependent chain.
// slices per group of the fused moments (the packed moments kernel's kMomQW)
constexpr int kMomQWave = 8;

template <int M>
__global__ __launch_bounds__(64, 2) void eigh_wave_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ list, int32_t count,
    const double* __restrict__ F, const double* __restrict__ Dold, double* __restrict__ C,
    double* __restrict__ eps, double* __restrict__ Dnew, double* __restrict__ dD_max,
    int32_t* __restrict__ flags, const int64_t* __restrict__ off_tri, double* __restrict__ Dw,
    const double* __restrict__ Bp, const int64_t* __restrict__ off_Bp,
    double* __restrict__ dmom) {
  static_assert(M % 2 == 0 && M >= 2 && M <= 32, "half-wave matrix size");
  constexpr int LD = M + 1;
  __shared__ double S1[2][M * LD];
  __shared__ double S2[2][M * LD];
  __shared__ double csb[2][M];      // (c, s) of the M/2 pairs
  __shared__ double lam[2][M];
  __shared__ int32_t rk[2][M];
  __shared__ int32_t occ[2][M];
  const int lane = threadIdx.x, h = lane >> 5, t = lane & 31;
  const int mi = blockIdx.x * 2 + h;
  const bool active = mi < count;
  const int f = active ? list[mi] : 0;
  const int n = active ? frag[f].nbf : 0;
  const int nocc = active ? frag[f].nocc : 0;
  const int64_t oc = active ? frag[f].off_C : 0;
  double* s1 = S1[h];
  double* s2 = S2[h];
  // ---- warm start: S1 = C, S2 = F_sym C, then A = C^T (F C).  Global
  // loads are unconditional (positions outside the matrix read its first
  // element and are replaced by zero), so that each lane's loads are in
  // flight together.
  // The Fock row and column of this lane are loaded together with the
  // orbitals, so that the two loads' latencies overlap.
  double frow[M], fcol[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const bool in = t < n && k < n;
    frow[k] = F[oc + (in ? t * n + k : 0)];
    fcol[k] = F[oc + (in ? k * n + t : 0)];
  }
  {
    constexpr int kPer = (M * M + 31) / 32;
    double cv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = t + 32 * u, i = e / M, j = e - (e / M) * M;
      const bool in = e < M * M && i < n && j < n;
      const double x = C[oc + (in ? i * n + j : 0)];
      cv[u] = in ? x : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = t + 32 * u, i = e / M, j = e - (e / M) * M;
      if (e < M * M) s1[i * LD + j] = cv[u];
    }
  }
  __syncthreads();
  if (t < M) {
#pragma unroll
    for (int k = 0; k < M; ++k) frow[k] = (t < n && k < n) ? 0.5 * (frow[k] + fcol[k]) : 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) acc = fma(frow[k], s1[k * LD + j], acc);
      s2[t * LD + j] = acc;
    }
  }
  __syncthreads();
  double a[M], v[M];
  if (t < M) {
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < M; ++i) acc = fma(s1[i * LD + t], s2[i * LD + j], acc);
      a[j] = acc;
      v[j] = s1[t * LD + j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) { a[j] = 0.0; v[j] = 0.0; }
  }
  __syncthreads();
  if (t < M)
#pragma unroll
    for (int j = 0; j < M; ++j) s2[t * LD + j] = a[j];
  __syncthreads();
  if (t < M)
#pragma unroll
    for (int j = 0; j < M; ++j) a[j] = 0.5 * (s2[t * LD + j] + s2[j * LD + t]);
  // lane t of this half receives the row of lane pi^-1(t) after each round
  int src = t;
#pragma unroll
  for (int s = 0; s < M; ++s)
    if (SlotPerm<M>::pi(s) == t) src = s;
  const int src_addr = 4 * (h * 32 + (t < M ? src : t));
  const bool odd = (t & 1) != 0;

  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const double q = a[j] * a[j];
      if (j == t) dia = q; else off += q;
    }
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 32);
      dia += __shfl_xor(dia, o, 32);
    }
    const bool done = off <= 1e-24 * dia || !(off == off);
    if (__all(done)) break;
    for (int r = 0; r < M - 1; ++r) {
      // this lane's pair (slots 2k, 2k+1): diagonal and off-diagonal entries
      double x0 = 0.0, x1 = 0.0;
#pragma unroll
      for (int k = 0; k < M / 2; ++k)
        if (2 * k == (t & ~1)) { x0 = a[2 * k]; x1 = a[2 * k + 1]; }
      const double d = odd ? x1 : x0, o = odd ? x0 : x1;
      const double dp = dpp_swap_pair(d), op = dpp_swap_pair(o);
      const double app = odd ? dp : d, aqq = odd ? d : dp, apq = odd ? op : o;
      double c, s;
      jacobi_rotation(app, aqq, apq, c, s);
      if (done) { c = 1.0; s = 0.0; }
      if (!odd && t < M) { csb[h][t] = c; csb[h][t + 1] = s; }
      __syncthreads();
      // columns of A and V
#pragma unroll
      for (int k = 0; k < M / 2; ++k) {
        const double ck = csb[h][2 * k], sk = csb[h][2 * k + 1];
        const double ap = a[2 * k], aq = a[2 * k + 1];
        a[2 * k] = ck * ap - sk * aq;
        a[2 * k + 1] = sk * ap + ck * aq;
        const double vp = v[2 * k], vq = v[2 * k + 1];
        v[2 * k] = ck * vp - sk * vq;
        v[2 * k + 1] = sk * vp + ck * vq;
      }
      // rows of A with the partner lane: p <- c p - s q, q <- s p + c q
      const double sg = odd ? s : -s;
#pragma unroll
      for (int j = 0; j < M; ++j) a[j] = fma(sg, dpp_swap_pair(a[j]), c * a[j]);
      // relabel the slots
      double na[M], nv[M];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        na[j] = bperm_d(src_addr, a[SlotPerm<M>::inv(j)]);
        nv[j] = v[SlotPerm<M>::inv(j)];
      }
#pragma unroll
      for (int j = 0; j < M; ++j) { a[j] = na[j]; v[j] = nv[j]; }
    }
  }

  // ---- eigenvalues (slot j = index j), ranks, outputs
  double lt = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j)
    if (j == t) lt = a[j];
  if (t < M) lam[h][t] = lt;
  __syncthreads();
  if (t < n) {
    int r0 = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = lam[h][j];
      r0 += (lj < lt) || (lj == lt && j < t);
    }
    rk[h][t] = r0;
    if (r0 < nocc) occ[h][r0] = t;
    eps[frag[f].off_eps + r0] = lt;
  }
  __syncthreads();
  if (t < n) {
#pragma unroll
    for (int j = 0; j < M; ++j)
      if (j < n) C[oc + t * n + rk[h][j]] = v[j];
#pragma unroll
    for (int j = 0; j < M; ++j) s1[t * LD + j] = v[j];
  }
  __syncthreads();
  double dmax = 0.0;
  if (t < n) {
    double dold[M];  // this lane's row of the previous density, loaded up front
#pragma unroll
    for (int j = 0; j < M; ++j) dold[j] = Dold[oc + t * n + (j < n ? j : 0)];
    // row t of the density, all columns at once: per occupied slot one
    // entry of this row and the slot's column (read by every lane of the
    // half alike), the products added in slot order as before
    double dacc[M];
#pragma unroll
    for (int j = 0; j < M; ++j) dacc[j] = 0.0;
    for (int k = 0; k < nocc; ++k) {
      const int sl = occ[h][k];
      const double ov = s1[t * LD + sl];
#pragma unroll
      for (int j = 0; j < M; ++j) dacc[j] = fma(ov, s1[j * LD + sl], dacc[j]);
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
      if (j < n) {
        const double acc = dacc[j];
        Dnew[oc + t * n + j] = acc;
        // the weighted packed copy, exactly as the density kernel forms it
        if (Dw && t <= j) {
          const int kk = t * n - t * (t - 1) / 2 + (j - t);
          const double w = (t == j ? 1.0 : 2.0) * acc;
          Dw[off_tri[f] + kk] = w;
          if (dmom) s2[kk] = w;
        }
        dmax = fmax(dmax, fabs(acc - dold[j]));
      }
    }
  }
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 32));
  if (dmom) {
    // Coulomb moments of the new densities for the next SCF step, d_Q =
    // sum_k Bp[Q][k] Dw[k], computed here as the packed moments kernel
    // computes them (the whole wave per matrix, lane l holding positions
    // 2 l + 128 c, c = 0..2, eight slices at a time, the same products in the
    // same order and the same wave sum), so the values are bitwise equal.
    // Only launched when every triangle is even-sized, at most 384 numbers
    // and starts at even offsets (the packed kernel's direct path).
    __syncthreads();
#pragma unroll 1
    for (int hh = 0; hh < 2; ++hh) {
      const int mj = blockIdx.x * 2 + hh;
      if (mj >= count) break;
      const int fj = list[mj];
      const FragInfo fi = frag[fj];
      const int nt = fi.nbf * (fi.nbf + 1) / 2;
      const double* dl = S2[hh];
      double2 dv[3];
      int kc[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int k = 2 * lane + 128 * c;
        kc[c] = min(k, nt - 2);
        dv[c] = k < nt ? double2{dl[k], dl[k + 1]} : double2{0.0, 0.0};
      }
#pragma unroll 1
      for (int q0 = 0; q0 < fi.naux; q0 += kMomQWave) {
        const int nq = min(kMomQWave, fi.naux - q0);
        const double* b = Bp + off_Bp[fj] + (int64_t)q0 * nt;
        double2 bv[kMomQWave][3];
#pragma unroll
        for (int q = 0; q < kMomQWave; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            bv[q][c] = *reinterpret_cast<const double2*>(b + (int64_t)min(q, nq - 1) * nt + kc[c]);
        double accm[kMomQWave];
#pragma unroll
        for (int q = 0; q < kMomQWave; ++q) {
          accm[q] = 0.0;
#pragma unroll
          for (int c = 0; c < 3; ++c)
            accm[q] = fma(bv[q][c].y, dv[c].y, fma(bv[q][c].x, dv[c].x, accm[q]));
        }
#pragma unroll
        for (int q = 0; q < kMomQWave; ++q) {
          const double tq = wave_sum_dpp(accm[q]);
          if (lane == 0 && q < nq) dmom[fi.off_aux + q0 + q] = tq;
        }
      }
    }
  }
  if (active && t == 0) {
    atomic_max_nonneg(dD_max, dmax);
    if (nocc > 0 && nocc < n) {
      double lh = 0.0, ll = 0.0;
      for (int j = 0; j < n; ++j) {
        if (rk[h][j] == nocc - 1) lh = lam[h][j];
        if (rk[h][j] == nocc) ll = lam[h][j];
      }
      if (!(ll > lh)) atomicOr(flags, FEF_FLAG_GAP);
    }
  }
}

// ---------------------------------------------------------------------------
// Jacobi for large fragments (48 < n <= 180): one workgroup of 1024 threads
// per matrix.  A's upper triangle (m (m + 1) / 2 numbers, m = n rounded up to
// even) lives in LDS; in each round every 2x2 block (rows of pair k, columns
// of pair l, k <= l) is transformed once, A_blk <- R_k^T A_blk R_l, so every
// stored element is written by exactly one thread.  V is kept transposed in
// a global workspace slot (row p = column p of V), so the column update of
// a pair touches two contiguous rows.  Warm start as above (A = C^T F C,
// V = C), same rotation formula and stopping rule.
__device__ inline int tri_at(int i, int j, int m) {  // packed index of (min, max)
  const int a = i < j ? i : j, b = i < j ? j : i;
  return a * m - a * (a - 1) / 2 + (b - a);
}
__device__ inline void tri_rc(int k, int m, int& i, int& j) {
  const double b = 2.0 * m + 1.0;
  int r = (int)((b - sqrt(b * b - 8.0 * (double)k)) * 0.5);
  if (r < 0) r = 0;
  if (r > m - 1) r = m - 1;
  while (r > 0 && r * m - r * (r - 1) / 2 > k) --r;
  while (r + 1 < m && (r + 1) * m - (r + 1) * r / 2 <= k) ++r;
  i = r;
  j = r + (k - (r * m - r * (r - 1) / 2));
}

constexpr int kLargeMax = 180;
size_t eigh_large_lds_bytes(int nmax) {
  const int m = nmax + (nmax & 1), half = m / 2;
  return (size_t)m * (m + 1) / 2 * sizeof(double) + 2 * (size_t)half * sizeof(double) +
         2 * (size_t)half * sizeof(int) + (size_t)m * sizeof(double) + 2 * (size_t)m * sizeof(int);
}

__global__ __launch_bounds__(1024) void eigh_large_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ list,
    const double* __restrict__ F, const double* __restrict__ Dold, double* __restrict__ C,
    double* __restrict__ eps, double* __restrict__ Dnew, double* __restrict__ dD_max,
    int32_t* __restrict__ flags, double* __restrict__ ws_eig, int max_n) {
  constexpr int NT = 1024;
  extern __shared__ double sm[];
  __shared__ double red[NT / 64];
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  const int n = fi.nbf, m = n + (n & 1), half = m / 2, ntri = m * (m + 1) / 2;
  double* Ap = sm;
  double* cc = Ap + ntri;
  double* ss = cc + half;
  int* pp = reinterpret_cast<int*>(ss + half);
  int* qq = pp + half;
  double* lam = reinterpret_cast<double*>(qq + half);  // 2 half ints: 8-byte aligned
  int* rank = reinterpret_cast<int*>(lam + m);
  int* occ = rank + m;
  const size_t slot = (size_t)(max_n + 1) * (max_n + 1);
  double* Vt = ws_eig + (size_t)blockIdx.x * eig_large_slot(max_n);  // [m][m]
  double* T = Vt + slot;                                 // [n][n]
  const double* Fx = F + fi.off_C;
  const double* Cx = C + fi.off_C;
  // T = F_sym C, then the upper triangle of A = C^T T, and V^T = C^T
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int i = e / n, j = e - (e / n) * n;
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc = fma(0.5 * (Fx[i * n + k] + Fx[k * n + i]), Cx[k * n + j], acc);
    T[e] = acc;
  }
  for (int e = threadIdx.x; e < m * m; e += NT) {
    const int p = e / m, i = e - (e / m) * m;
    Vt[e] = (p < n && i < n) ? Cx[i * n + p] : 0.0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < ntri; k += NT) {
    int i, j;
    tri_rc(k, m, i, j);
    double acc = 0.0;
    if (i < n && j < n)
      for (int q = 0; q < n; ++q) acc = fma(Cx[q * n + i], T[q * n + j], acc);
    Ap[k] = acc;
  }
  __syncthreads();
  // This thread's 2x2 blocks (at most kBlk: half (half + 1) / 2 <= 4096),
  // fixed for the whole solve.
  constexpr int kBlk = 4;
  static_assert((kLargeMax / 2) * (kLargeMax / 2 + 1) / 2 <= kBlk * NT, "block table");
  const int nblk = half * (half + 1) / 2;
  int blk[kBlk];
#pragma unroll
  for (int j = 0; j < kBlk; ++j) {
    const int b = threadIdx.x + j * NT;
    int k = 0, l = 0;
    if (b < nblk) tri_rc(b, half, k, l);
    blk[j] = b < nblk ? (k | (l << 16)) : -1;
  }
  // V^T update map: thread = (pair group vg, column vi); the pairs
  // vg, vg + ngrp, ... of a round, kVB of them per batch so that all their
  // loads are in flight together.
  constexpr int kVB = 6;
  const int ngrp = NT / n;  // >= 5
  const int vg = threadIdx.x / n, vi = threadIdx.x - (threadIdx.x / n) * n;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int k = threadIdx.x; k < ntri; k += NT) {
      int i, j;
      tri_rc(k, m, i, j);
      const double a = Ap[k];
      if (i == j) dia += a * a; else off += 2.0 * a * a;
    }
    off = block_sum(off, red);
    dia = block_sum(dia, red);
    if (off <= 1e-24 * dia || !(off == off)) break;
    for (int r = 0; r < m - 1; ++r) {
      for (int k = threadIdx.x; k < half; k += NT) {
        int p, q;
        round_robin_pair(r, k, m, p, q);
        double c, s;
        jacobi_rotation(Ap[tri_at(p, p, m)], Ap[tri_at(q, q, m)], Ap[tri_at(p, q, m)], c, s);
        cc[k] = c;
        ss[k] = s;
        pp[k] = p;
        qq[k] = q;
      }
      __syncthreads();
      // columns p, q of V (rows of V^T) of every pair: loads of a batch first
      if (vg < ngrp)
        for (int k0 = vg; k0 < half; k0 += kVB * ngrp) {
          double vp[kVB], vq[kVB];
#pragma unroll
          for (int u = 0; u < kVB; ++u) {
            const int k = k0 + u * ngrp;
            if (k < half) {
              vp[u] = Vt[(size_t)pp[k] * m + vi];
              vq[u] = Vt[(size_t)qq[k] * m + vi];
            }
          }
#pragma unroll
          for (int u = 0; u < kVB; ++u) {
            const int k = k0 + u * ngrp;
            if (k < half) {
              const double c = cc[k], s = ss[k];
              Vt[(size_t)pp[k] * m + vi] = c * vp[u] - s * vq[u];
              Vt[(size_t)qq[k] * m + vi] = s * vp[u] + c * vq[u];
            }
          }
        }
#pragma unroll
      for (int j = 0; j < kBlk; ++j) {
        if (blk[j] < 0) continue;
        const int k = blk[j] & 0xffff, l = blk[j] >> 16;
        const int a0 = pp[k], a1 = qq[k], b0 = pp[l], b1 = qq[l];
        const double ck = cc[k], sk = ss[k], cl = cc[l], sl = ss[l];
        const int i00 = tri_at(a0, b0, m), i01 = tri_at(a0, b1, m);
        const int i10 = tri_at(a1, b0, m), i11 = tri_at(a1, b1, m);
        const double m00 = Ap[i00], m01 = Ap[i01], m10 = Ap[i10], m11 = Ap[i11];
        const double t00 = ck * m00 - sk * m10, t01 = ck * m01 - sk * m11;
        const double t10 = sk * m00 + ck * m10, t11 = sk * m01 + ck * m11;
        const double n00 = cl * t00 - sl * t01, n01 = sl * t00 + cl * t01;
        const double n10 = cl * t10 - sl * t11, n11 = sl * t10 + cl * t11;
        Ap[i00] = n00;
        Ap[i01] = n01;  // for k == l, (a0, a1) = (p, q) with p < q and i10 == i01
        Ap[i11] = n11;
        if (k != l) Ap[i10] = n10;
      }
      __syncthreads();
    }
  }
  // ascending order, ties broken by index
  for (int i = threadIdx.x; i < n; i += NT) lam[i] = Ap[tri_at(i, i, m)];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) {
    const double li = lam[i];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = lam[j];
      rk += (lj < li) || (lj == li && j < i);
    }
    rank[i] = rk;
    if (rk < fi.nocc) occ[rk] = i;
    eps[fi.off_eps + rk] = li;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int p = e / n, i = e - (e / n) * n;
    C[fi.off_C + (size_t)i * n + rank[p]] = Vt[(size_t)p * m + i];
  }
  // occupied columns of V into LDS when they fit where A was, then D
  const bool vo_lds = fi.nocc * n <= ntri;
  double* Vo = Ap;  // [nocc][n]
  if (vo_lds)
    for (int e = threadIdx.x; e < fi.nocc * n; e += NT) {
      const int k = e / n, i = e - (e / n) * n;
      Vo[e] = Vt[(size_t)occ[k] * m + i];
    }
  __syncthreads();
  double dmax = 0.0;
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int l = e / n, s = e - (e / n) * n;
    double acc = 0.0;
    for (int k = 0; k < fi.nocc; ++k)
      acc = vo_lds ? fma(Vo[k * n + l], Vo[k * n + s], acc)
                   : fma(Vt[(size_t)occ[k] * m + l], Vt[(size_t)occ[k] * m + s], acc);
    Dnew[fi.off_C + e] = acc;
    dmax = fmax(dmax, fabs(acc - Dold[fi.off_C + e]));
  }
  dmax = block_max(dmax, red);
  if (threadIdx.x == 0) {
    atomic_max_nonneg(dD_max, dmax);
    if (fi.nocc > 0 && fi.nocc < n) {
      double lh = 0.0, ll = 0.0;
      for (int j = 0; j < n; ++j) {
        if (rank[j] == fi.nocc - 1) lh = lam[j];
        if (rank[j] == fi.nocc) ll = lam[j];
      }
      if (!(ll > lh)) atomicOr(flags, FEF_FLAG_GAP);
    }
  }
}

// rotation table (c, s, p, q per pair) + ranks + sorted eigenvalues
static size_t eig_scratch_bytes(int n) {
  const int half = (n + 1) / 2;
  return (size_t)2 * half * sizeof(double) + (size_t)2 * half * sizeof(int) +
         (size_t)2 * half * sizeof(int) + (size_t)(n + 1) * sizeof(double);
}

hipError_t launch_eigh(const fef_plan_s& p, const double* F, const double* Dold, double* C,
                       double* eps, double* Dnew, double* dD_max, int32_t* flags,
                       double* ws_eig, hipStream_t st, double* Dw, const double* Bp,
                       double* dmom) {
  // n <= 32: register-resident kernels, one size class per launch
  {
    const int sizes[4] = {8, 16, 24, 32};
    for (int c = 0; c < 4; ++c) {
      const int32_t b = p.eig_w_off[c], cnt = p.eig_w_off[c + 1] - b;
      if (cnt == 0) continue;
      const dim3 grid((unsigned)((cnt + 1) / 2));
      const int32_t* lst = p.d_eig_small + b;
#define FEF_EIGW(MM)                                                                          \
  hipLaunchKernelGGL((eigh_wave_kernel<MM>), grid, dim3(64), 0, st, p.d_frag, lst, cnt, F,    \
                     Dold, C, eps, Dnew, dD_max, flags, p.d_off_tri, Dw, Bp, p.d_off_Bp, dmom)
      switch (sizes[c]) {
        case 8: FEF_EIGW(8); break;
        case 16: FEF_EIGW(16); break;
        case 24: FEF_EIGW(24); break;
        default: FEF_EIGW(32); break;
      }
#undef FEF_EIGW
    }
  }
  if (!p.eig_mid.empty()) {
    const int nmax = 48;
    const size_t lds = 3 * (size_t)nmax * (nmax + 1) * sizeof(double) + eig_scratch_bytes(nmax);
    hipLaunchKernelGGL((eigh_kernel<256, 48>), dim3((unsigned)p.eig_mid.size()), dim3(256), lds,
                       st, p.d_frag, p.d_eig_mid, F, Dold, C, eps, Dnew, dD_max, flags, ws_eig,
                       nmax);
  }
  if (!p.eig_large.empty() && p.eig_large_max_nbf <= kTriMax) {
    hipError_t e = launch_eigh_tri(p, F, Dold, C, eps, Dnew, dD_max, flags, ws_eig, st);
    if (e != hipSuccess) return e;
  } else if (!p.eig_large.empty() && p.eig_large_max_nbf <= kLargeMax) {
    const int nmax = p.eig_large_max_nbf;
    static bool configured = false;
    if (!configured) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&eigh_large_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)eigh_large_lds_bytes(kLargeMax));
      (void)hipGetLastError();
      configured = true;
    }
    hipLaunchKernelGGL(eigh_large_kernel, dim3((unsigned)p.eig_large.size()), dim3(1024),
                       eigh_large_lds_bytes(nmax), st, p.d_frag, p.d_eig_large, F, Dold, C, eps,
                       Dnew, dD_max, flags, ws_eig, nmax);
  } else if (!p.eig_large.empty()) {
    const int nmax = p.eig_large_max_nbf;
    hipLaunchKernelGGL((eigh_kernel<1024, 0>), dim3((unsigned)p.eig_large.size()), dim3(1024),
                       eig_scratch_bytes(nmax), st, p.d_frag, p.d_eig_large, F, Dold, C, eps,
                       Dnew, dD_max, flags, ws_eig, nmax);
  }
  return hipGetLastError();
}

// One matrix n x n (for instance the coupling G_00 posed as a fragment with
// no occupied orbitals), global-memory path, cold start.
hipError_t launch_eigh_one(const FragInfo* d_fi, const int32_t* d_list, int n, const double* F,
                           const double* Dold, double* C, double* eps, double* Dnew,
                           double* dmax, int32_t* flags, double* ws_eig, hipStream_t st) {
  hipLaunchKernelGGL((eigh_kernel<1024, 0>), dim3(1), dim3(1024), eig_scratch_bytes(n), st, d_fi,
                     d_list, F, Dold, C, eps, Dnew, dmax, flags, ws_eig, n);
  return hipGetLastError();
}

}  // namespace fef
