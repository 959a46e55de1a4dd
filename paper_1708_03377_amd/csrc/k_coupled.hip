// Dimer doubles coupled through the inter-fragment part of the two-body
// zeroth-order operator (Sec. II.B: the particle-rank-conserving partition
// of Eq. partitioning0 keeps W^[0] in H0, so the dimer-doubles equation,
// Eq. dimDoubles, becomes a linear system instead of a division).
//
// For a pair (x, y) the amplitudes t[i,a,j,b] of the excitations i -> a on
// x and j -> b on y solve (D + W) t = -v with
//   v[i,a,j,b] = (ia|jb),   D = eps_a + eps_b - eps_i - eps_j,
//   (W t)[i,a,j,b] = + sum (aa'|bb') t[i,a',j,b']   particle ladder
//                    - sum (aa'|j'j) t[i,a',j',b]   hole line on y
//                    - sum (i'i|bb') t[i',a,j,b']   hole line on x
//                    + sum (i'i|j'j) t[i',a,j',b]   hole ladder
// and E2_xy = 4 sum v t.  The integrals come from the factored
// inter-fragment tensor,
//   (pq|rs)^{xy} = s_xy sum_Q X^x[Q][p][q] Y^y[Q][r][s],
//   Y^f[P] = C^f^T B^f[P] C^f (every slice of f's class, made exactly
//   symmetric), X^f[Q] = sum_P G_{c(f),0}[P][Q] Y^f[P] (Q < P_0);
// y is always a class-0 fragment.
//
// One workgroup solves one pair at a time in its slot of the workspace.  It
// builds v, D and the four operator blocks, each a matrix A[m][k] over its
// own index pairs,
//     pp  m = (a,b),  k = (a',b'):  (aa'|bb')
//     ph  m = (a,j),  k = (a',j'):  (aa'|j'j)
//     hp  m = (i,b),  k = (i',b'):  (i'i|bb')
//     hh  m = (i,j),  k = (i',j'):  (i'i|j'j)
// every one a sum over Q of Kronecker products, i.e. a GEMM over Q with rows
// (alpha, alpha') and columns (beta, beta'), run on FP64 MFMA and stored in
// 16 x 4 MFMA operand tiles.  Conjugate gradients preconditioned with D then
// apply W on FP64 MFMA too: the tiles stream from the slot, the search
// direction is gathered from LDS (from the slot when it does not fit).
//
// Amplitude vectors use the (a, b)-major order
//   idx(a,b,i,j) = (a vy + b) nO + i oy + j,        nO = ox oy,
// in which each block's row index m and column index n land on the vector
// position rowpart(m) + colpart(n):
//   pp: (a,b) -> (a vy + b) nO      n = (i,j) -> i oy + j
//   ph: (a,j) -> a vy nO + j        n = (b,i) -> b nO + i oy
//   hp: (i,b) -> b nO + i oy        n = (a,j) -> a vy nO + j
//   hh: (i,j) -> i oy + j           n = (a,b) -> (a vy + b) nO
// and the contraction index k, of the row kind, is gathered through the
// row map.  Each block covers every vector position exactly once.
#include <algorithm>
#include <cmath>

#include "fef_internal.h"
#include "fef_device.h"

namespace fef {

namespace {

constexpr int kCgThreads = 512;
constexpr int kCgWaves = kCgThreads / 64;
// LDS of one workgroup (the search direction p and the product W p held in
// LDS when 16 n bytes and the maps fit).
constexpr int64_t kCgLdsMax = 159 * 1024;
// device memory of the pair slots of one launch
constexpr int64_t kCgSlotBudget = (int64_t)8 << 30;

typedef double d4v __attribute__((ext_vector_type(4)));

// Two block-wide sums at once (fixed order: lanes, then waves); both results
// in every thread.
__device__ __attribute__((always_inline)) inline void block_sum_pair(double& a, double& b,
                                                                     double (*red2)[kCgWaves]) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red2[0][w] = a;
    red2[1][w] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int k = 0; k < kCgWaves; ++k) {
    sa += red2[0][k];
    sb += red2[1][k];
  }
  __syncthreads();
  a = sa;
  b = sb;
}

__device__ __attribute__((always_inline)) inline d4v mma64(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Offset of element (m, k) of an operator block stored in MFMA A-operand
// tiles: tile (m / 16, k / 4) holds 64 consecutive doubles, lane l = 16 (k %
// 4) + m % 16 reading element l (the FP64 16x16x4 A-operand layout).  A row
// of tiles holds tile_ks(M) tiles, ceil(M / 4) rounded up to a multiple of
// kApplyKC (the products load whole chunks of kApplyKC tiles; the padding
// is zero).
constexpr int kApplyKC = 8;
__host__ __device__ inline int tile_ks(int64_t M) {
  return (int)((((M + 3) / 4) + kApplyKC - 1) / kApplyKC * kApplyKC);
}
__device__ __attribute__((always_inline)) inline int64_t tile_off(int m, int k, int KS) {
  return ((int64_t)(m >> 4) * KS + (k >> 2)) * 64 + (k & 3) * 16 + (m & 15);
}
__host__ __device__ inline int64_t tiled_doubles(int64_t M) {
  return ((M + 15) / 16) * 16 * (4 * (int64_t)tile_ks(M));
}

// ---- MO blocks -------------------------------------------------------------

// H[P][mu][q] = sum_nu B[P][mu][nu] C[nu][q]
__global__ __launch_bounds__(256) void mo_left_kernel(const FragInfo* __restrict__ frag,
                                                      const double* __restrict__ B,
                                                      const double* __restrict__ C,
                                                      double* __restrict__ H) {
  const FragInfo fi = frag[blockIdx.x];
  const int n = fi.nbf;
  const int64_t nn = (int64_t)n * n;
  const double* Cf = C + fi.off_C;
  for (int P = blockIdx.y; P < fi.naux; P += gridDim.y) {
    const double* Bp = B + fi.off_B + P * nn;
    double* Hp = H + fi.off_B + P * nn;
    for (int64_t e = threadIdx.x; e < nn; e += blockDim.x) {
      const int mu = (int)(e / n), q = (int)(e - (int64_t)mu * n);
      double s = 0.0;
      for (int nu = 0; nu < n; ++nu) s = fma(Bp[(int64_t)mu * n + nu], Cf[(int64_t)nu * n + q], s);
      Hp[e] = s;
    }
  }
}

// Y[P][p][q] = Y[P][q][p] = sum_mu C[mu][p] H[P][mu][q] for p <= q (the
// block is symmetric; the upper triangle is computed and mirrored, so every
// operator block built from it is exactly symmetric).
__global__ __launch_bounds__(256) void mo_right_kernel(const FragInfo* __restrict__ frag,
                                                       const double* __restrict__ C,
                                                       const double* __restrict__ H,
                                                       double* __restrict__ Y) {
  const FragInfo fi = frag[blockIdx.x];
  const int n = fi.nbf;
  const int64_t nn = (int64_t)n * n;
  const double* Cf = C + fi.off_C;
  for (int P = blockIdx.y; P < fi.naux; P += gridDim.y) {
    const double* Hp = H + fi.off_B + P * nn;
    double* Yp = Y + fi.off_B + P * nn;
    for (int64_t e = threadIdx.x; e < nn; e += blockDim.x) {
      const int p = (int)(e / n), q = (int)(e - (int64_t)p * n);
      if (p > q) continue;
      double s = 0.0;
      for (int mu = 0; mu < n; ++mu) s = fma(Cf[(int64_t)mu * n + p], Hp[(int64_t)mu * n + q], s);
      Yp[(int64_t)p * n + q] = s;
      Yp[(int64_t)q * n + p] = s;
    }
  }
}

// X[Q][p][q] = sum_P G_{c,0}[P][Q] Y[P][p][q], Q < P_0 (fragment f's X block
// starts at P_0 * off_C)
__global__ __launch_bounds__(256) void x_fold_kernel(const FragInfo* __restrict__ frag,
                                                     const double* __restrict__ G,
                                                     const int64_t* __restrict__ off_G, int P0,
                                                     const double* __restrict__ Y,
                                                     double* __restrict__ X) {
  const FragInfo fi = frag[blockIdx.x];
  const int64_t nn = (int64_t)fi.nbf * fi.nbf;
  const double* Gc = G + off_G[fi.cls];
  for (int Q = blockIdx.y; Q < P0; Q += gridDim.y) {
    double* Xq = X + (int64_t)P0 * fi.off_C + Q * nn;
    for (int64_t e = threadIdx.x; e < nn; e += blockDim.x) {
      double s = 0.0;
      for (int P = 0; P < fi.naux; ++P) s = fma(Gc[(int64_t)P * P0 + Q], Y[fi.off_B + P * nn + e], s);
      Xq[e] = s;
    }
  }
}

// ---- pair solve --------------------------------------------------------------

// Exact quotient x / d for 0 <= x < 2^22, 1 <= d < 2^11 through the FP32
// reciprocal (the estimate is off by at most one, then corrected).
struct FastDiv {
  int d;
  float r;
  __device__ explicit FastDiv(int d_) : d(d_), r(1.0f / (float)d_) {}
  __device__ __attribute__((always_inline)) int div(int x) const {
    int q = (int)((float)x * r);
    const int rem = x - q * d;
    q += (rem >= d) - (rem < 0);
    return q;
  }
};

// One side of a Kronecker-sum GEMM: slice q of the block is
// T[q * slice + (r0 + row) * ld + c0 + col].
struct KronSide {
  const double* T;
  int64_t slice;
  int ld, r0, c0;
};

// C[(al, al2)][(be, be2)] = s sum_{q < nq} X_q[al][al2] Y_q[be][be2] for al <
// na, al2 < na2, be < nb, be2 < nb2 on FP64 MFMA; each element is handed to
// store(al, al2, be, be2, value).  Waves take 32 x 32 output blocks in turn.
// The q loop runs in chunks of kKronKC MFMA k steps, an even number of them,
// two register buffers deep (the next chunk's loads are in flight while the
// current one is multiplied).  Rows and columns past the block are clamped
// into it (their results are dropped); q >= nq loads slice nq - 1 and
// multiplies it by zero.
constexpr int kKronKC = 5;
template <class Store>
__device__ __attribute__((always_inline)) inline void kron_gemm(const KronSide X, int na, int na2,
                                                                const KronSide Y, int nb, int nb2,
                                                                int nq, double s, int wave,
                                                                int lane, Store store) {
  const int nR = na * na2, nS = nb * nb2;
  const int RT2 = (nR + 31) >> 5, ST2 = (nS + 31) >> 5;
  const int li = lane & 15, lk = lane >> 4;
  const int nks = (nq + 3) >> 2;
  const int nch = (((nks + kKronKC - 1) / kKronKC) + 1) & ~1;
  const FastDiv da(na2), db(nb2);
  for (int task = wave; task < RT2 * ST2; task += kCgWaves) {
    const int rt = task / ST2, st = task - (task / ST2) * ST2;
    int64_t oa[2], ob[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int R = min(rt * 32 + u * 16 + li, nR - 1);
      const int qa = da.div(R);
      oa[u] = (int64_t)(X.r0 + qa) * X.ld + X.c0 + (R - qa * na2);
      const int S = min(st * 32 + u * 16 + li, nS - 1);
      const int qb = db.div(S);
      ob[u] = (int64_t)(Y.r0 + qb) * Y.ld + Y.c0 + (S - qb * nb2);
    }
    d4v acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int w = 0; w < 2; ++w) acc[u][w] = d4v{0.0, 0.0, 0.0, 0.0};
    double a0[kKronKC][2], b0[kKronKC][2], a1[kKronKC][2], b1[kKronKC][2];
    auto load = [&](int ch, double (&a)[kKronKC][2], double (&b)[kKronKC][2])
                    __attribute__((always_inline)) {
#pragma unroll
      for (int j = 0; j < kKronKC; ++j) {
        const int q = 4 * (ch * kKronKC + j) + lk;
        const bool ok = q < nq;
        const int64_t qc = ok ? q : nq - 1;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const double av = X.T[qc * X.slice + oa[u]];
          a[j][u] = ok ? av : 0.0;
          b[j][u] = Y.T[qc * Y.slice + ob[u]];
        }
      }
    };
    auto mult = [&](const double (&a)[kKronKC][2], const double (&b)[kKronKC][2])
                    __attribute__((always_inline)) {
#pragma unroll
      for (int j = 0; j < kKronKC; ++j)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int w = 0; w < 2; ++w) acc[u][w] = mma64(a[j][u], b[j][w], acc[u][w]);
    };
    load(0, a0, b0);
    for (int ch = 0; ch < nch; ch += 2) {
      load(ch + 1, a1, b1);
      mult(a0, b0);
      if (ch + 2 < nch) load(ch + 2, a0, b0);
      mult(a1, b1);
    }
    // FP64 MFMA result: row lk + 4 r, column li of each 16 x 16 tile
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int w = 0; w < 2; ++w)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int R = rt * 32 + u * 16 + lk + 4 * r, S = st * 32 + w * 16 + li;
          if (R < nR && S < nS) {
            const int qa = da.div(R), qb = db.div(S);
            store(qa, R - qa * na2, qb, S - qb * nb2, s * acc[u][w][r]);
          }
        }
  }
}

// Zero the padding of a tiled M x M block: rows M .. 16 MT - 1 and columns
// M .. 4 KS - 1 (the products read every element of a tile).
__device__ __attribute__((always_inline)) inline void zero_tile_pad(double* A, int M) {
  const int MT = (M + 15) >> 4, KS = tile_ks(M);
  const int rows = MT * 16 - M, cols = KS * 4 - M;
  for (int e = threadIdx.x; e < rows * KS * 4; e += kCgThreads) {
    const int m = M + e / (KS * 4), k = e % (KS * 4);
    A[tile_off(m, k, KS)] = 0.0;
  }
  for (int e = threadIdx.x; e < M * cols; e += kCgThreads) {
    const int m = e / cols, k = M + e % cols;
    A[tile_off(m, k, KS)] = 0.0;
  }
}

// out (op)= A p for one operator block: A is M x M in MFMA tiles; the product
// B(k, n) = p[rp[k] + cp[n]] (n < N); each result goes to out[rp[m] + cp[n]]:
//   mode 0: out = result (the first block), 1: out += result, 2: out -= result.
// Waves take (row tile, two column tiles) tasks in turn.  The tiles stream
// in chunks of kApplyKC k steps, two register buffers deep; past the block,
// k and n are clamped into it (A's padding columns are zero, results of
// padding columns are dropped), so every load is unconditional.
template <typename PV>
__device__ __attribute__((always_inline)) inline void apply_block(
    const double* __restrict__ A, int M, int N, const int* rp, const int* cp, const PV* p,
    PV* out, int mode, int wave, int lane) {
  const int MT = (M + 15) >> 4, KS = tile_ks(M), NT2 = (N + 31) >> 5;
  const int li = lane & 15, lk = lane >> 4;
  for (int task = wave; task < MT * NT2; task += kCgWaves) {
    const int mt = task / NT2, nt = task - (task / NT2) * NT2;
    int cl[2];
    bool okc[2];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int n = nt * 32 + w * 16 + li;
      okc[w] = n < N;
      cl[w] = cp[min(n, N - 1)];
    }
    d4v acc[2] = {d4v{0.0, 0.0, 0.0, 0.0}, d4v{0.0, 0.0, 0.0, 0.0}};
    const double* At = A + (int64_t)mt * KS * 64 + lane;
    double a0[kApplyKC], a1[kApplyKC];
    auto load = [&](int ks0, double (&a)[kApplyKC]) __attribute__((always_inline)) {
#pragma unroll
      for (int j = 0; j < kApplyKC; ++j) a[j] = At[(int64_t)(ks0 + j) * 64];
    };
    auto mult = [&](int ks0, const double (&a)[kApplyKC]) __attribute__((always_inline)) {
      int rk[kApplyKC];
#pragma unroll
      for (int j = 0; j < kApplyKC; ++j) rk[j] = rp[min(4 * (ks0 + j) + lk, M - 1)];
      double b[kApplyKC][2];
#pragma unroll
      for (int j = 0; j < kApplyKC; ++j)
#pragma unroll
        for (int w = 0; w < 2; ++w) b[j][w] = (double)p[rk[j] + cl[w]];
#pragma unroll
      for (int j = 0; j < kApplyKC; ++j)
#pragma unroll
        for (int w = 0; w < 2; ++w) acc[w] = mma64(a[j], b[j][w], acc[w]);
    };
    load(0, a0);
    for (int ks0 = 0; ks0 < KS; ks0 += 2 * kApplyKC) {
      if (ks0 + kApplyKC < KS) load(ks0 + kApplyKC, a1);
      mult(ks0, a0);
      if (ks0 + kApplyKC >= KS) break;
      if (ks0 + 2 * kApplyKC < KS) load(ks0 + 2 * kApplyKC, a0);
      mult(ks0 + kApplyKC, a1);
    }
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      if (!okc[w]) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mt * 16 + lk + 4 * r;
        if (m >= M) continue;
        const int e = rp[m] + cl[w];
        if (mode == 0) out[e] = acc[w][r];
        else if (mode == 1) out[e] += acc[w][r];
        else out[e] -= acc[w][r];
      }
    }
  }
}

}  // namespace

namespace {

template <bool kLds>
__global__ __launch_bounds__(kCgThreads) void coupled_cg_kernel(
    const FragInfo* __restrict__ frag, const PairInfo* __restrict__ pairs,
    const int32_t* __restrict__ list, int32_t count, const double* __restrict__ X,
    const double* __restrict__ Y, int P0, const double* __restrict__ eps,
    double* __restrict__ slots, CgSlot L, double tol, int maxit, double* __restrict__ E2_pair,
    int32_t* __restrict__ iters, int32_t* __restrict__ flags, double* __restrict__ rec,
    const int64_t* __restrict__ rec_off) {
  extern __shared__ __align__(16) char lds_raw[];
  __shared__ double red[kCgWaves];
  __shared__ double red2[2][kCgWaves];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int tid = threadIdx.x;
  double* slot = slots + (int64_t)blockIdx.x * L.size;
  double* v = slot + L.v;
  double* D = slot + L.d;
  double* t = slot + L.t;
  double* r = slot + L.r;
  double* Aq = slot + L.q;
  double* Aph = slot + L.ph;
  double* Ahp = slot + L.hp;
  double* Ahh = slot + L.hh;
  double* pb;
  double* apb;
  int* tab;
  if constexpr (kLds) {
    pb = reinterpret_cast<double*>(lds_raw);
    apb = pb + L.npb;
    tab = reinterpret_cast<int*>(apb + L.nmax + kCgThreads);  // after the partial-sum room
  } else {
    pb = slot + L.p;
    apb = slot + L.ap;
    tab = reinterpret_cast<int*>(lds_raw);
  }
  for (int q = blockIdx.x; q < count; q += gridDim.x) {
    const int k = list[q];
    const PairInfo pr = pairs[k];
    const FragInfo fx = frag[pr.x], fy = frag[pr.y];
    const int ox = fx.nocc, vx = fx.nvir, oy = fy.nocc, vy = fy.nvir;
    const int nO = ox * oy, nV = vx * vy, nPH = vx * oy, nHP = ox * vy;
    const int n = nV * nO;
    if (n == 0) {
      if (tid == 0) {
        E2_pair[k] = 0.0;
        if (iters) iters[k] = 0;
      }
      if (rec) {
        const int nr = ox * ox + vx * vx + oy * oy + vy * vy;
        for (int u = tid; u < nr; u += kCgThreads) rec[rec_off[k] + u] = 0.0;
      }
      continue;
    }
    const double s = pr.s;
    // row and column maps of the four blocks
    int* rp_pp = tab;
    int* cp_pp = rp_pp + nV;
    int* rp_ph = cp_pp + nO;
    int* cp_ph = rp_ph + nPH;
    int* rp_hp = cp_ph + nHP;
    int* cp_hp = rp_hp + nHP;
    int* rp_hh = cp_hp + nPH;
    int* cp_hh = rp_hh + nO;
    for (int u = tid; u < nV; u += kCgThreads) { rp_pp[u] = u * nO; cp_hh[u] = u * nO; }
    for (int u = tid; u < nO; u += kCgThreads) { cp_pp[u] = u; rp_hh[u] = u; }
    for (int u = tid; u < nPH; u += kCgThreads) {
      const int a = u / oy, j = u - (u / oy) * oy;  // u = a oy + j
      rp_ph[u] = a * vy * nO + j;
      cp_hp[u] = a * vy * nO + j;
    }
    for (int u = tid; u < nHP; u += kCgThreads) {
      const int b = u / ox, i = u - (u / ox) * ox;  // u = b ox + i (ph columns)
      cp_ph[u] = b * nO + i * oy;
      const int i2 = u / vy, b2 = u - (u / vy) * vy;  // u = i vy + b (hp rows)
      rp_hp[u] = b2 * nO + i2 * oy;
    }
    // v, D
    const int64_t nnx = (int64_t)fx.nbf * fx.nbf, nny = (int64_t)fy.nbf * fy.nbf;
    const double* Xx = X + (int64_t)P0 * fx.off_C;
    const double* Yy = Y + fy.off_B;
    kron_gemm(KronSide{Xx, nnx, fx.nbf, 0, ox}, ox, vx, KronSide{Yy, nny, fy.nbf, 0, oy}, oy, vy,
              P0, s, wave, lane,
              [&](int i, int a, int j, int b, double val) __attribute__((always_inline)) {
                v[(int64_t)(a * vy + b) * nO + i * oy + j] = val;
              });
    const double* ex = eps + fx.off_eps;
    const double* ey = eps + fy.off_eps;
    for (int e = tid; e < n; e += kCgThreads) {
      const int ab = e / nO, ij = e - (e / nO) * nO;
      const int a = ab / vy, b = ab - (ab / vy) * vy;
      const int i = ij / oy, j = ij - (ij / oy) * oy;
      D[e] = (ex[ox + a] - ex[i]) + (ey[oy + b] - ey[j]);
    }
    // operator blocks (not needed for maxit = 0: t = -v / D)
    if (maxit > 0) {
      const int KS = tile_ks(nV);
      kron_gemm(KronSide{Xx, nnx, fx.nbf, ox, ox}, vx, vx, KronSide{Yy, nny, fy.nbf, oy, oy}, vy,
                vy, P0, s, wave, lane,
                [&](int a, int a2, int b, int b2, double val) __attribute__((always_inline)) {
                  Aq[tile_off(a * vy + b, a2 * vy + b2, KS)] = val;
                });
      zero_tile_pad(Aq, nV);
    }
    if (maxit > 0) {
      const int KS = tile_ks(nPH);
      kron_gemm(KronSide{Xx, nnx, fx.nbf, ox, ox}, vx, vx, KronSide{Yy, nny, fy.nbf, 0, 0}, oy,
                oy, P0, s, wave, lane,
                [&](int a, int a2, int j, int j2, double val) __attribute__((always_inline)) {
                  Aph[tile_off(a * oy + j, a2 * oy + j2, KS)] = val;
                });
      zero_tile_pad(Aph, nPH);
    }
    if (maxit > 0) {
      const int KS = tile_ks(nHP);
      kron_gemm(KronSide{Xx, nnx, fx.nbf, 0, 0}, ox, ox, KronSide{Yy, nny, fy.nbf, oy, oy}, vy,
                vy, P0, s, wave, lane,
                [&](int i, int i2, int b, int b2, double val) __attribute__((always_inline)) {
                  Ahp[tile_off(i * vy + b, i2 * vy + b2, KS)] = val;
                });
      zero_tile_pad(Ahp, nHP);
    }
    if (maxit > 0) {
      const int KS = tile_ks(nO);
      kron_gemm(KronSide{Xx, nnx, fx.nbf, 0, 0}, ox, ox, KronSide{Yy, nny, fy.nbf, 0, 0}, oy,
                oy, P0, s, wave, lane,
                [&](int i, int i2, int j, int j2, double val) __attribute__((always_inline)) {
                  Ahh[tile_off(i * oy + j, i2 * oy + j2, KS)] = val;
                });
      zero_tile_pad(Ahh, nO);
    }
    __syncthreads();

    // W p into apb (the owner of each element adds D p)
    auto apply = [&]() __attribute__((always_inline)) {
      apply_block(Aq, nV, nO, rp_pp, cp_pp, pb, apb, 0, wave, lane);
      __syncthreads();
      apply_block(Aph, nPH, nHP, rp_ph, cp_ph, pb, apb, 2, wave, lane);
      __syncthreads();
      apply_block(Ahp, nHP, nPH, rp_hp, cp_hp, pb, apb, 2, wave, lane);
      __syncthreads();
      apply_block(Ahh, nO, nV, rp_hh, cp_hh, pb, apb, 1, wave, lane);
      __syncthreads();
    };

    // start: t = b / D with b = -v; r = b - (D + W) t; p = z = r / D.
    // Conjugate gradients as the oracle takes them; t, r and D live in the
    // slot, p and W p in LDS when they fit.
    double nb = 0.0, rr = 0.0, vt = 0.0;
    int it = 0;
    double bb = 0.0;
#pragma unroll 4
    for (int e = tid; e < n; e += kCgThreads) {
      const double b = -v[e];
      const double t0 = b / D[e];
      t[e] = t0;
      pb[e] = t0;
      bb = fma(b, b, bb);
      if (maxit == 0) vt = fma(v[e], t0, vt);
    }
    nb = sqrt(block_sum(bb, red));
    if (maxit > 0) {
      apply();
      double rz = 0.0;
      rr = 0.0;
#pragma unroll 4
      for (int e = tid; e < n; e += kCgThreads) {
        const double re = -v[e] - fma(D[e], pb[e], apb[e]);
        const double z = re / D[e];
        r[e] = re;
        pb[e] = z;
        rz = fma(re, z, rz);
        rr = fma(re, re, rr);
      }
      block_sum_pair(rz, rr, red2);
      while (it < maxit && !(sqrt(rr) <= tol * nb)) {
        apply();
        double pap = 0.0;
#pragma unroll 4
        for (int e = tid; e < n; e += kCgThreads) {
          const double pe = pb[e];
          pap = fma(pe, fma(D[e], pe, apb[e]), pap);
        }
        pap = block_sum(pap, red);
        const double alpha = rz / pap;
        double rzn = 0.0;
        rr = 0.0;
#pragma unroll 4
        for (int e = tid; e < n; e += kCgThreads) {
          const double pe = pb[e];
          t[e] = fma(alpha, pe, t[e]);
          const double re = fma(-alpha, fma(D[e], pe, apb[e]), r[e]);
          r[e] = re;
          const double z = re / D[e];
          rzn = fma(re, z, rzn);
          rr = fma(re, re, rr);
        }
        block_sum_pair(rzn, rr, red2);
        const double beta = rzn / rz;
#pragma unroll 4
        for (int e = tid; e < n; e += kCgThreads) pb[e] = fma(beta, pb[e], r[e] / D[e]);
        rz = rzn;
        ++it;
        __syncthreads();
      }
#pragma unroll 4
      for (int e = tid; e < n; e += kCgThreads) vt = fma(v[e], t[e], vt);
    }
    const double E = 4.0 * block_sum(vt, red);
    if (tid == 0) {
      E2_pair[k] = E;
      if (iters) iters[k] = it;
      if (!isfinite(E)) atomicOr(flags, FEF_FLAG_NONFINITE);
      // maxit = 0 stops at the start, the residual of t = -v / D unformed
      if (maxit == 0 || !(sqrt(rr) <= tol * nb)) atomicOr(flags, FEF_FLAG_NOCONV);
    }
    if (rec) {
      // the pair's one-body dressings (Eqs. MPij, MPab, doubles terms) into
      // its record [Hoo^x][Hvv^x][Hoo^y][Hvv^y]; p's storage, free after the
      // solve, holds the partial sums of short outputs
      double* R = rec + rec_off[k];
      double* scratch = pb;
      const double* vd = v;
      const double* td = t;
      if constexpr (kLds) {
        // v and t into LDS (p and W p are free after the solve), partial
        // sums in the room behind them
        __syncthreads();
        for (int e = tid; e < n; e += kCgThreads) {
          pb[e] = v[e];
          apb[e] = t[e];
        }
        vd = pb;
        td = apb;
        scratch = apb + L.nmax;
      }
      const int64_t vyn = (int64_t)vy * nO;
      // nout outputs, each sum over kk < K of term(o, kk), times scale:
      // outputs fewer than the threads are split over parts summed in order
      auto split_sum = [&](int nout, int K, double scale, double* dst, auto term)
                           __attribute__((always_inline)) {
        if (nout >= kCgThreads) {
          for (int o = tid; o < nout; o += kCgThreads) {
            double acc = 0.0;
            for (int kk = 0; kk < K; ++kk) acc += term(o, kk);
            dst[o] = scale * acc;
          }
          return;
        }
        const int np = kCgThreads / nout;
        if (tid < np * nout) {
          const int o = tid % nout, part = tid / nout;
          double acc = 0.0;
          for (int kk = part; kk < K; kk += np) acc += term(o, kk);
          scratch[part * nout + o] = acc;
        }
        __syncthreads();
        for (int o = tid; o < nout; o += kCgThreads) {
          double acc = 0.0;
          for (int part = 0; part < np; ++part) acc += scratch[part * nout + o];
          dst[o] = scale * acc;
        }
        __syncthreads();
      };
      __syncthreads();
      // Hoo^x[i][i1] = 2 sum_{a b, j} v[a b, i, j] t[a b, i1, j]
      split_sum(ox * ox, nV, 2.0, R, [&](int o, int ab) __attribute__((always_inline)) {
        const int i = o / ox, i1 = o - (o / ox) * ox;
        const double* vr = vd + (int64_t)ab * nO + i * oy;
        const double* tr = td + (int64_t)ab * nO + i1 * oy;
        double q = 0.0;
        for (int j = 0; j < oy; ++j) q = fma(vr[j], tr[j], q);
        return q;
      });
      // Hvv^x[a][a1] = -2 sum_{b, i j} v[a1 b, i j] t[a b, i j]
      split_sum(vx * vx, (int)vyn, -2.0, R + ox * ox,
                [&](int o, int m) __attribute__((always_inline)) {
                  const int a = o / vx, a1 = o - (o / vx) * vx;
                  return vd[a1 * vyn + m] * td[a * vyn + m];
                });
      // Hoo^y[j][j1] = 2 sum_{a b, i} v[a b, i, j] t[a b, i, j1]
      split_sum(oy * oy, nV, 2.0, R + ox * ox + vx * vx,
                [&](int o, int ab) __attribute__((always_inline)) {
                  const int j = o / oy, j1 = o - (o / oy) * oy;
                  const double* vr = vd + (int64_t)ab * nO + j;
                  const double* tr = td + (int64_t)ab * nO + j1;
                  double q = 0.0;
                  for (int i = 0; i < ox; ++i) q = fma(vr[i * oy], tr[i * oy], q);
                  return q;
                });
      // Hvv^y[b][b1] = -2 sum_{a, i j} v[a b1, i j] t[a b, i j]
      split_sum(vy * vy, vx, -2.0, R + ox * ox + vx * vx + oy * oy,
                [&](int o, int a) __attribute__((always_inline)) {
                  const int b = o / vy, b1 = o - (o / vy) * vy;
                  const double* vr = vd + (int64_t)(a * vy + b1) * nO;
                  const double* tr = td + (int64_t)(a * vy + b) * nO;
                  double q = 0.0;
                  for (int ij = 0; ij < nO; ++ij) q = fma(vr[ij], tr[ij], q);
                  return q;
                });
    }
    __syncthreads();
  }
}

// Per-fragment dressings: the sum, in pair order, of the fragment's parts of
// the records of its pairs (inc_base: where each part starts).
__global__ __launch_bounds__(256) void dressing_reduce_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ inc_ptr,
    const int64_t* __restrict__ inc_base, const int64_t* __restrict__ off_oo,
    const int64_t* __restrict__ off_vv, const double* __restrict__ rec, double* __restrict__ Hoo,
    double* __restrict__ Hvv) {
  const int f = blockIdx.x;
  const FragInfo fi = frag[f];
  const int noo = fi.nocc * fi.nocc, nvv = fi.nvir * fi.nvir;
  const int b0 = inc_ptr[f], b1 = inc_ptr[f + 1];
  for (int e = blockIdx.y * 256 + threadIdx.x; e < noo + nvv; e += 256 * gridDim.y) {
    double acc = 0.0;
    for (int m = b0; m < b1; ++m) acc += rec[inc_base[m] + e];
    if (e < noo) Hoo[off_oo[f] + e] = acc;
    else Hvv[off_vv[f] + (e - noo)] = acc;
  }
}

// E2_total = sum of E2_pair in a fixed order (one block: strided lane sums,
// then lane and wave order)
__global__ __launch_bounds__(256) void coupled_total_kernel(const double* __restrict__ E2_pair,
                                                            int64_t npair,
                                                            double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < npair; k += 256) s += E2_pair[k];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) *out = t;
}

}  // namespace

template <typename T>
static hipError_t upload_vec(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return hipSuccess;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Pair groups by the class of x: one launch each, slots sized for the
// group's largest pair.  Dressing tables: each pair's record [Hoo^x][Hvv^x]
// [Hoo^y][Hvv^y] (oriented x, y), the output offsets of every fragment, and
// each fragment's record parts in pair order.
hipError_t coupled_setup(fef_plan_s& p) {
  p.cp_groups.clear();
  p.cp_list.clear();
  const int ncu = compute_units();
  std::vector<std::vector<int32_t>> by_cls(std::max(p.nclass, 1));
  for (int64_t k = 0; k < p.npair; ++k) by_cls[p.frag[p.pairs[k].x].cls].push_back((int32_t)k);
  auto amp = [&](int32_t k) {
    const FragInfo& fx = p.frag[p.pairs[k].x];
    const FragInfo& fy = p.frag[p.pairs[k].y];
    return (int64_t)fx.ov * fy.ov;
  };
  for (auto& lst : by_cls) {
    if (lst.empty()) continue;
    // largest first, so the static round robin over slots ends evenly
    std::stable_sort(lst.begin(), lst.end(), [&](int32_t a, int32_t b) { return amp(a) > amp(b); });
    CoupledGroup g;
    g.first = (int32_t)p.cp_list.size();
    g.count = (int32_t)lst.size();
    int64_t nmax = 0, nV = 0, nO = 0, nPH = 0, nHP = 0;
    for (int32_t k : lst) {
      const FragInfo& fx = p.frag[p.pairs[k].x];
      const FragInfo& fy = p.frag[p.pairs[k].y];
      nmax = std::max<int64_t>(nmax, (int64_t)fx.ov * fy.ov);
      nV = std::max<int64_t>(nV, (int64_t)fx.nvir * fy.nvir);
      nO = std::max<int64_t>(nO, (int64_t)fx.nocc * fy.nocc);
      nPH = std::max<int64_t>(nPH, (int64_t)fx.nvir * fy.nocc);
      nHP = std::max<int64_t>(nHP, (int64_t)fx.nocc * fy.nvir);
      p.cp_list.push_back(k);
    }
    const int64_t tab_bytes = 8 * (nV + nO + nPH + nHP);
    const int64_t npb = std::max<int64_t>(nmax, kCgThreads);
    const int64_t lds_bytes = 8 * (npb + nmax + kCgThreads) + tab_bytes;
    g.lds = lds_bytes <= kCgLdsMax - 1024;
    g.lds_bytes = (size_t)(g.lds ? lds_bytes : tab_bytes);
    auto al = [](int64_t x) { return round_up(std::max<int64_t>(x, 1), 64); };
    CgSlot& L = g.L;
    int64_t o = 0;
    L.nmax = nmax;
    L.npb = npb;
    L.v = o; o += al(nmax);
    L.d = o; o += al(nmax);
    L.t = o; o += al(nmax);
    L.r = o; o += al(nmax);
    L.p = o; o += g.lds ? 0 : al(npb);
    L.ap = o; o += g.lds ? 0 : al(nmax);
    L.q = o; o += al(tiled_doubles(nV));
    L.ph = o; o += al(tiled_doubles(nPH));
    L.hp = o; o += al(tiled_doubles(nHP));
    L.hh = o; o += al(tiled_doubles(nO));
    L.size = o;
    const int64_t per_cu = g.lds_bytes > (size_t)(kCgLdsMax / 2) ? 1 : 2;
    int64_t ns = std::min<int64_t>(g.count, (int64_t)ncu * per_cu);
    ns = std::min<int64_t>(ns, std::max<int64_t>(1, kCgSlotBudget / (8 * L.size)));
    g.nslots = (int32_t)ns;
    p.cp_groups.push_back(g);
  }
  std::vector<int64_t> rec_off(std::max<int64_t>(p.npair, 1), 0), off_oo(p.nfrag), off_vv(p.nfrag);
  std::vector<std::vector<std::pair<int32_t, int64_t>>> parts(p.nfrag);
  int64_t o = 0;
  for (int64_t k = 0; k < p.npair; ++k) {
    const FragInfo& fx = p.frag[p.pairs[k].x];
    const FragInfo& fy = p.frag[p.pairs[k].y];
    rec_off[k] = o;
    const int64_t xpart = (int64_t)fx.nocc * fx.nocc + (int64_t)fx.nvir * fx.nvir;
    parts[p.pairs[k].x].push_back({(int32_t)k, o});
    parts[p.pairs[k].y].push_back({(int32_t)k, o + xpart});
    o += xpart + (int64_t)fy.nocc * fy.nocc + (int64_t)fy.nvir * fy.nvir;
  }
  p.n_rec = o;
  int64_t noo = 0, nvv = 0;
  std::vector<int32_t> inc_ptr(p.nfrag + 1, 0);
  std::vector<int64_t> inc_base;
  for (int f = 0; f < p.nfrag; ++f) {
    off_oo[f] = noo;
    off_vv[f] = nvv;
    noo += (int64_t)p.frag[f].nocc * p.frag[f].nocc;
    nvv += (int64_t)p.frag[f].nvir * p.frag[f].nvir;
    auto& v = parts[f];
    std::sort(v.begin(), v.end());
    for (auto& e : v) inc_base.push_back(e.second);
    inc_ptr[f + 1] = (int32_t)inc_base.size();
  }
  p.n_oo = noo;
  p.n_vv = nvv;
  hipError_t e = upload_vec(&p.d_cp_list, p.cp_list);
  if (e == hipSuccess) e = upload_vec(&p.d_rec_off, rec_off);
  if (e == hipSuccess) e = upload_vec(&p.d_off_oo, off_oo);
  if (e == hipSuccess) e = upload_vec(&p.d_off_vv, off_vv);
  if (e == hipSuccess) e = upload_vec(&p.d_inc_ptr, inc_ptr);
  if (e == hipSuccess) e = upload_vec(&p.d_inc_base, inc_base);
  return e;
}

// The coupled solve's workspace, then the pair records.
int64_t dressing_ws_bytes(const fef_plan_s& p) {
  return coupled_ws_bytes(p) + 8 * round_up(std::max<int64_t>(p.n_rec, 1), 32);
}

// Workspace: Y (B-pool sized), X (P_0 per C-pool element), then a region
// shared by the first half-transform product H (B-pool sized) and the pair
// slots of whichever group runs.
int64_t coupled_ws_bytes(const fef_plan_s& p) {
  int64_t slots = 0;
  for (const auto& g : p.cp_groups) slots = std::max<int64_t>(slots, (int64_t)g.nslots * g.L.size);
  const int64_t y = round_up(std::max<int64_t>(p.nB, 1), 32);
  const int64_t x = round_up(std::max<int64_t>((int64_t)p.P0 * p.nC, 1), 32);
  return 8 * (y + x + std::max<int64_t>(round_up(std::max<int64_t>(p.nB, 1), 32), slots));
}

// rec non-null: the solve kernels also write each pair's dressing record
// (the workspace part after the coupled solve's, see dressing_ws_bytes)
static hipError_t launch_coupled(const fef_plan_s& p, const double* B, const double* C,
                                 const double* eps, const double* G, double tol, int maxit,
                                 double* E2_pair, double* E2_total, int32_t* iters,
                                 int32_t* flags, void* ws, hipStream_t st,
                                 double* rec = nullptr) {
  double* Y = static_cast<double*>(ws);
  double* X = Y + round_up(std::max<int64_t>(p.nB, 1), 32);
  double* H = X + round_up(std::max<int64_t>((int64_t)p.P0 * p.nC, 1), 32);
  double* slots = H;
  if (p.npair > 0 && p.nfrag > 0) {
    const unsigned gy = (unsigned)std::min(std::max(p.max_naux, 1), 64);
    hipLaunchKernelGGL(mo_left_kernel, dim3(p.nfrag, gy), dim3(256), 0, st, p.d_frag, B, C, H);
    hipLaunchKernelGGL(mo_right_kernel, dim3(p.nfrag, gy), dim3(256), 0, st, p.d_frag, C, H, Y);
    const unsigned gq = (unsigned)std::min(std::max(p.P0, 1), 64);
    hipLaunchKernelGGL(x_fold_kernel, dim3(p.nfrag, gq), dim3(256), 0, st, p.d_frag, G,
                       p.d_off_G, p.P0, Y, X);
    for (const auto& g : p.cp_groups) {
      const int32_t* list = p.d_cp_list + g.first;
      if (g.lds) {
        hipLaunchKernelGGL(coupled_cg_kernel<true>, dim3(g.nslots), dim3(kCgThreads), g.lds_bytes,
                           st, p.d_frag, p.d_pair, list, g.count, X, Y, p.P0, eps, slots, g.L,
                           tol, maxit, E2_pair, iters, flags, rec, p.d_rec_off);
      } else {
        hipLaunchKernelGGL(coupled_cg_kernel<false>, dim3(g.nslots), dim3(kCgThreads),
                           g.lds_bytes, st, p.d_frag, p.d_pair, list, g.count, X, Y, p.P0, eps,
                           slots, g.L, tol, maxit, E2_pair, iters, flags, rec, p.d_rec_off);
      }
    }
  }
  hipLaunchKernelGGL(coupled_total_kernel, dim3(1), dim3(256), 0, st, E2_pair, p.npair, E2_total);
  return hipGetLastError();
}

static hipError_t launch_dressing_reduce(const fef_plan_s& p, const double* rec, double* Hoo,
                                         double* Hvv, hipStream_t st) {
  if (p.nfrag == 0) return hipSuccess;
  int64_t mx = 1;
  for (const FragInfo& fi : p.frag)
    mx = std::max<int64_t>(mx, (int64_t)fi.nocc * fi.nocc + (int64_t)fi.nvir * fi.nvir);
  const unsigned gy = (unsigned)std::min<int64_t>((mx + 255) / 256, 64);
  hipLaunchKernelGGL(dressing_reduce_kernel, dim3(p.nfrag, gy), dim3(256), 0, st, p.d_frag,
                     p.d_inc_ptr, p.d_inc_base, p.d_off_oo, p.d_off_vv, rec, Hoo, Hvv);
  return hipGetLastError();
}

// Lifts the dynamic-LDS limit of the solve kernels once per process (as the
// other large-LDS kernels of this library do, a refusal is left to the
// launch to report).
static void coupled_prepare() {
  static bool configured = false;
  if (configured) return;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&coupled_cg_kernel<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCgLdsMax);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&coupled_cg_kernel<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCgLdsMax);
  (void)hipGetLastError();
  configured = true;
}

}  // namespace fef

using namespace fef;

extern "C" {

fef_status fef_coupled_pair_energies(fef_plan p, const double* B, const double* C,
                                     const double* eps, const double* G, double tol,
                                     int32_t maxit, double* E2_pair, double* E2_total,
                                     int32_t* iters, int32_t* flags, void* ws, size_t ws_bytes,
                                     void* stream) {
  if (!p) return FEF_E_ARG;
  if (!E2_total || !flags) return FEF_E_ARG;
  if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 0) return FEF_E_ARG;
  if (p->npair > 0 && (!B || !C || !eps || !G || !E2_pair || !ws)) return FEF_E_ARG;
  if (p->npair > 0 && ws_bytes < (size_t)coupled_ws_bytes(*p)) return FEF_E_WORKSPACE;
  // index arithmetic of the blocks is exact below nbf = 2048
  if (p->max_nbf >= 2048) return FEF_E_UNSUPPORTED;
  for (const auto& g : p->cp_groups)
    if (g.lds_bytes > (size_t)kCgLdsMax) return FEF_E_UNSUPPORTED;
  coupled_prepare();
  return launch_coupled(*p, B, C, eps, G, tol, maxit, E2_pair, E2_total, iters, flags, ws,
                        static_cast<hipStream_t>(stream)) == hipSuccess
             ? FEF_OK
             : FEF_E_HIP;
}

fef_status fef_dimer_dressing(fef_plan p, const double* B, const double* C, const double* eps,
                              const double* G, double tol, int32_t maxit, double* E2_pair,
                              double* E2_total, double* Hoo, double* Hvv, int32_t* flags,
                              void* ws, size_t ws_bytes, void* stream) {
  if (!p) return FEF_E_ARG;
  if (!E2_total || !flags) return FEF_E_ARG;
  if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 0) return FEF_E_ARG;
  if (p->npair > 0 && (!B || !C || !eps || !G || !E2_pair || !ws)) return FEF_E_ARG;
  if ((p->n_oo > 0 && !Hoo) || (p->n_vv > 0 && !Hvv)) return FEF_E_ARG;
  if (p->npair > 0 && ws_bytes < (size_t)dressing_ws_bytes(*p)) return FEF_E_WORKSPACE;
  if (p->max_nbf >= 2048) return FEF_E_UNSUPPORTED;
  for (const auto& g : p->cp_groups)
    if (g.lds_bytes > (size_t)kCgLdsMax) return FEF_E_UNSUPPORTED;
  coupled_prepare();
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* rec = ws ? reinterpret_cast<double*>(static_cast<char*>(ws) + coupled_ws_bytes(*p))
                  : nullptr;
  hipError_t e = launch_coupled(*p, B, C, eps, G, tol, maxit, E2_pair, E2_total, nullptr, flags,
                                ws, st, p->npair > 0 ? rec : nullptr);
  if (e == hipSuccess && p->npair > 0) e = launch_dressing_reduce(*p, rec, Hoo, Hvv, st);
  else if (e == hipSuccess && p->nfrag > 0) {
    // no pairs: every dressing is zero (a kernel, not a memset)
    e = launch_dressing_reduce(*p, rec, Hoo, Hvv, st);
  }
  return e == hipSuccess ? FEF_OK : FEF_E_HIP;
}

}  // extern "C"
