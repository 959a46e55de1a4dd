// Effective Coulomb field of the polarisation-screened fragment Fock matrix
// (the "bubble" integrals 2 v^{mu j}_{nu j} summed over every other fragment
// inside the cutoff), through the factored integrals:
//   D^y      = C^y_occ C^y_occ^T                     (density, no factor 2)
//   d^y_Q    = sum_{lambda sigma} B^y[Q][lambda sigma] D^y[lambda sigma]
//   phi^x    = sum_{y in nbr(x)} s_xy G_{c(x) c(y)} d^y
//   J^x      = 2 sum_P B^x[P] phi^x_P ;  F~^x = F0^x + h~^x + J^x
// Moments and J each stream B once (HBM bound); the neighbour sum gathers
// P-vectors of the neighbours (L2 resident).
#include <algorithm>

#include "fef_internal.h"
#include "fef_device.h"

namespace fef {

// D = C_occ C_occ^T, one block per chunk of the flat density pool;
// optionally also its upper triangle, off-diagonal entries doubled
// (Dw[k] = w_k D[mu][nu], the weights of the packed moments).
__global__ __launch_bounds__(256) void density_kernel(const FragInfo* __restrict__ frag,
                                                      const Chunk* __restrict__ chunks,
                                                      const int64_t* __restrict__ off_tri,
                                                      const double* __restrict__ C,
                                                      double* __restrict__ D,
                                                      double* __restrict__ Dw,
                                                      double* __restrict__ dD_max) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && dD_max) *dD_max = 0.0;
  const Chunk ch = chunks[blockIdx.x];
  const FragInfo fi = frag[ch.frag];
  const int n = fi.nbf, o = fi.nocc;
  const double* c = C + fi.off_C;
  const int e0 = (int)(ch.begin - fi.off_C), e1 = (int)(ch.end - fi.off_C);
  for (int e = e0 + threadIdx.x; e < e1; e += 256) {
    const int l = e / n, s = e - (e / n) * n;
    double acc = 0.0;
    for (int k = 0; k < o; ++k) acc = fma(c[l * n + k], c[s * n + k], acc);
    D[fi.off_C + e] = acc;
    if (Dw && l <= s)
      Dw[off_tri[ch.frag] + l * n - l * (l - 1) / 2 + (s - l)] = (l == s ? 1.0 : 2.0) * acc;
  }
}

__global__ void zero_scalar_kernel(double* p) { *p = 0.0; }

// d^x_Q: each wave reduces four Q against one pass over D, sixteen Q per
// block (fixed summation order: lane-strided partial sums, then the wave).
constexpr int kMomQ = 4;
__global__ __launch_bounds__(256) void moments_kernel(const FragInfo* __restrict__ frag,
                                                      const double* __restrict__ B,
                                                      const double* __restrict__ D,
                                                      double* __restrict__ dmom) {
  const FragInfo fi = frag[blockIdx.x];
  const int q0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * kMomQ;
  if (q0 >= fi.naux) return;
  const int lane = threadIdx.x & 63;
  const int nq = min(kMomQ, fi.naux - q0);
  const int nn = fi.nbf * fi.nbf;
  const double* b = B + fi.off_B + (int64_t)q0 * nn;
  const double* d = D + fi.off_C;
  double acc[kMomQ] = {0.0, 0.0, 0.0, 0.0};
  for (int e = lane; e < nn; e += 64) {
    const double dv = d[e];
#pragma unroll
    for (int k = 0; k < kMomQ; ++k)
      if (k < nq) acc[k] = fma(b[(int64_t)k * nn + e], dv, acc[k]);
  }
#pragma unroll
  for (int k = 0; k < kMomQ; ++k) {
    const double t = wave_sum_dpp(acc[k]);
    if (lane == 0 && k < nq) dmom[fi.off_aux + q0 + k] = t;
  }
}

// phi^x.  The neighbour moments are first summed per class,
// e_c = sum_{y in nbr(x), c(y) = c} s_xy d^y, then phi^x = sum_c G_{c(x) c} e_c
// with G_{c,0} stored and G_{0,c} = G_{c,0}^T.  Wave w takes the chunks of 64
// neighbours w, w + 4, ... in list order: each lane first loads one
// neighbour's index, coupling and table entries (one memory round trip for 64
// neighbours), then the wave walks the chunk in order, taking each
// neighbour's entries from its lane, so the moment loads of successive
// neighbours are independent and overlap.  Class-0 sums stay in registers
// (rows lane, lane + 64 of the P0 vector); the four wave partials are added
// in wave order, so the result is deterministic.
__global__ __launch_bounds__(256) void field_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ nbr_ptr,
    const int32_t* __restrict__ nbr_idx, const double* __restrict__ nbr_s,
    const double* __restrict__ G, const int64_t* __restrict__ off_G, int P0, int nclass,
    const int32_t* __restrict__ naux_cls_off, const double* __restrict__ dmom,
    double* __restrict__ phi) {
  extern __shared__ double part[];  // [4][etot] per-wave partial e_c, then e
  const int x = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int etot = naux_cls_off[nclass];
  for (int t = threadIdx.x; t < 4 * etot; t += blockDim.x) part[t] = 0.0;
  __syncthreads();
  double* mine = part + wave * etot;
  const int beg = nbr_ptr[x], end = nbr_ptr[x + 1];
  double e0 = 0.0, e1 = 0.0;
  for (int c0 = beg + 64 * wave; c0 < end; c0 += 256) {
    const int k = c0 + lane;
    int y_cls = 0, y_naux = 0;
    int64_t y_off = 0;
    double y_s = 0.0;
    if (k < end) {
      const int y = nbr_idx[k];
      y_s = nbr_s[k];
      y_cls = frag[y].cls;
      y_naux = frag[y].naux;
      y_off = frag[y].off_aux;
    }
    const int cnt = min(64, end - c0);
    // class-0 neighbours, eight at a time: the weight of any other class is
    // zeroed and its moments pointer parked at the pool start, so the loop
    // has no branches and the eight neighbours' loads are in flight together
    for (int j0 = 0; j0 < cnt; j0 += 8) {
      double s8[8], v0[8], v1[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = min(j0 + u, cnt - 1);
        const bool use = j0 + u < cnt && __builtin_amdgcn_readlane(y_cls, j) == 0;
        const int lo = __builtin_amdgcn_readlane((int)y_off, j);
        const int hi = __builtin_amdgcn_readlane((int)(y_off >> 32), j);
        const int64_t off = use ? (((int64_t)hi << 32) | (uint32_t)lo) : 0;
        const long long sb = __builtin_amdgcn_readlane((int)__double_as_longlong(y_s), j) &
                             0xffffffffLL;
        const long long sh =
            __builtin_amdgcn_readlane((int)(__double_as_longlong(y_s) >> 32), j);
        s8[u] = use ? __longlong_as_double((sh << 32) | sb) : 0.0;
        const double* dy = dmom + off;
        v0[u] = lane < P0 ? dy[lane] : 0.0;
        v1[u] = lane + 64 < P0 ? dy[lane + 64] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        e0 = fma(s8[u], v0[u], e0);
        e1 = fma(s8[u], v1[u], e1);
      }
    }
    // neighbours of other classes (rare): per-class sums in LDS
    if (__any(k < end && y_cls != 0)) {
      for (int j = 0; j < cnt; ++j) {
        const int cy = __builtin_amdgcn_readlane(y_cls, j);
        if (cy == 0) continue;
        const int lo = __builtin_amdgcn_readlane((int)y_off, j);
        const int hi = __builtin_amdgcn_readlane((int)(y_off >> 32), j);
        const int64_t off = ((int64_t)hi << 32) | (uint32_t)lo;
        const long long sb = __builtin_amdgcn_readlane((int)__double_as_longlong(y_s), j) &
                             0xffffffffLL;
        const long long sh =
            __builtin_amdgcn_readlane((int)(__double_as_longlong(y_s) >> 32), j);
        const double s = __longlong_as_double((sh << 32) | sb);
        const double* dy = dmom + off;
        const int base = naux_cls_off[cy], pc = __builtin_amdgcn_readlane(y_naux, j);
        for (int q = lane; q < pc; q += 64) mine[base + q] = fma(s, dy[q], mine[base + q]);
      }
    }
  }
  if (lane < P0) mine[lane] += e0;
  if (lane + 64 < P0) mine[lane + 64] += e1;
  __syncthreads();
  for (int q = threadIdx.x; q < etot; q += blockDim.x)
    part[q] = ((part[q] + part[etot + q]) + part[2 * etot + q]) + part[3 * etot + q];
  __syncthreads();
  const FragInfo fx = frag[x];
  const int cx = fx.cls;
  for (int p = threadIdx.x; p < fx.naux; p += blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < nclass; ++c) {
      const int pc = naux_cls_off[c + 1] - naux_cls_off[c];
      const double* ec = part + naux_cls_off[c];
      if (c == 0 && cx == 0) {
        // G_{0,0} is symmetric: read it by columns, so that consecutive
        // threads (rows p) load consecutive addresses; eight columns' loads
        // in flight at a time
        int q = 0;
        for (; q + 8 <= pc; q += 8) {
          double g8[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) g8[u] = G[(int64_t)(q + u) * P0 + p];
#pragma unroll
          for (int u = 0; u < 8; ++u) acc = fma(g8[u], ec[q + u], acc);
        }
        for (; q < pc; ++q) acc = fma(G[(int64_t)q * P0 + p], ec[q], acc);
      } else if (c == 0) {
        const double* g = G + off_G[cx];  // G_{cx,0}: [P_cx][P0]
        for (int q = 0; q < pc; ++q) acc = fma(g[(int64_t)p * P0 + q], ec[q], acc);
      } else if (cx == 0) {
        const double* g = G + off_G[c];   // G_{c,0}: [P_c][P0]; use its transpose
        for (int q = 0; q < pc; ++q) acc = fma(g[(int64_t)q * P0 + p], ec[q], acc);
      }
    }
    phi[fx.off_aux + p] = acc;
  }
}

// out^x[mu nu] = (F0 + h~)[mu nu] + 2 sum_P B^x[P][mu nu] phi^x_P.  Each
// thread takes two neighbouring elements (16-byte loads when nbf^2 and the
// fragment's B offset are even).
__global__ __launch_bounds__(256) void jbuild_kernel(const FragInfo* __restrict__ frag,
                                                     const double* __restrict__ B,
                                                     const double* __restrict__ phi,
                                                     const double* __restrict__ F0,
                                                     const double* __restrict__ htilde,
                                                     double* __restrict__ out) {
  const FragInfo fi = frag[blockIdx.x];
  const int nn = fi.nbf * fi.nbf;
  const int e = 2 * (blockIdx.y * blockDim.x + threadIdx.x);
  if (e >= nn) return;
  const double* b = B + fi.off_B + e;
  const double* ph = phi + fi.off_aux;
  double a0 = 0.0, a1 = 0.0;
  if ((nn & 1) == 0 && (fi.off_B & 1) == 0) {
#pragma unroll 8
    for (int P = 0; P < fi.naux; ++P) {
      const double2 v = *reinterpret_cast<const double2*>(b + (int64_t)P * nn);
      const double f = ph[P];
      a0 = fma(v.x, f, a0);
      a1 = fma(v.y, f, a1);
    }
  } else {
    const bool two = e + 1 < nn;
    for (int P = 0; P < fi.naux; ++P) {
      const double f = ph[P];
      a0 = fma(b[(int64_t)P * nn], f, a0);
      if (two) a1 = fma(b[(int64_t)P * nn + 1], f, a1);
    }
  }
  const int64_t o = fi.off_C + e;
  double v0 = 2.0 * a0, v1 = 2.0 * a1;
  if (F0) { v0 += F0[o]; if (e + 1 < nn) v1 += F0[o + 1]; }
  if (htilde) { v0 += htilde[o]; if (e + 1 < nn) v1 += htilde[o + 1]; }
  out[o] = v0;
  if (e + 1 < nn) out[o + 1] = v1;
}

// ---------------------------------------------------------------------------
// Packed coefficients: B^x[P] is symmetric, so only its upper triangle
// (mu <= nu, row-major, nbf (nbf + 1) / 2 numbers per slice) is kept.  The
// moments then weight off-diagonal entries by 2 and the J build writes both
// mirror images, halving the bytes both kernels stream per SCF step.
__device__ inline void tri_row_col(int k, int n, int& mu, int& nu) {
  // float guess of the row (the loops below correct it)
  const float b = 2.0f * n + 1.0f;
  int m = (int)((b - sqrtf(fmaxf(b * b - 8.0f * (float)k, 0.0f))) * 0.5f);
  if (m < 0) m = 0;
  if (m > n - 1) m = n - 1;
  while (m > 0 && m * n - m * (m - 1) / 2 > k) --m;
  while (m + 1 < n && (m + 1) * n - (m + 1) * m / 2 <= k) ++m;
  mu = m;
  nu = m + (k - (m * n - m * (m - 1) / 2));
}

// Bp = upper triangles of the B slices, one block per chunk of the packed pool.
__global__ __launch_bounds__(256) void pack_coefficients_kernel(const FragInfo* __restrict__ frag,
                                                                const Chunk* __restrict__ chunks,
                                                                const int64_t* __restrict__ off_Bp,
                                                                const double* __restrict__ B,
                                                                double* __restrict__ Bp) {
  const Chunk ch = chunks[blockIdx.x];
  const FragInfo fi = frag[ch.frag];
  const int n = fi.nbf, nt = n * (n + 1) / 2;
  const double* b = B + fi.off_B;
  const int64_t base = off_Bp[ch.frag];
  const int e0 = (int)(ch.begin - base), e1 = (int)(ch.end - base);
  // eight loads per thread in flight: addresses of elements past the chunk
  // are clamped to its last element and their values are not stored
  for (int eb = e0 + threadIdx.x; eb < e1; eb += 256 * 8) {
    double v8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = min(eb + 256 * u, e1 - 1);
      const int P = e / nt, k = e - (e / nt) * nt;
      int mu, nu;
      tri_row_col(k, n, mu, nu);
      v8[u] = b[P * n * n + mu * n + nu];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (eb + 256 * u < e1) Bp[base + eb + 256 * u] = v8[u];
  }
}

// d^x_Q = sum_k Bp[Q][k] Dw[k] from the packed slices and the weighted
// packed density.  Each wave takes kMomQW consecutive Q (four waves per
// block); with triangles of at most 384 numbers (up to 27 basis functions)
// the k loop is unrolled and every load is unconditional, so that all of a
// wave's loads are in flight together.  kPack: the slice values are read
// from B at their triangle positions and also written to Bp (the packing
// of the first SCF step of a pass), in the same order as the packed
// variant, so that Bp and d are bitwise those of packing then moments.
// Blocks run fragment-major (the nqb Q blocks of a fragment are adjacent in
// the 1-D grid), so the kernel streams the pool from its start to its end;
// the fused field and J kernel (small fragments) walks the fragments
// backwards and so starts on the slices this kernel read last, which the
// memory-side cache still holds, and ends on the first ones, where the next
// step's moments start again.  zero_out non-null: one thread clears it
// (a maximum that a later kernel of the same step accumulates).
constexpr int kMomQW = 8;
template <bool kPack>
__global__ __launch_bounds__(256) void moments_packed_kernel(const FragInfo* __restrict__ frag,
                                                             const int64_t* __restrict__ off_Bp,
                                                             const int64_t* __restrict__ off_tri,
                                                             const double* __restrict__ Bsrc,
                                                             const double* __restrict__ Dw,
                                                             double* __restrict__ dmom,
                                                             const double* __restrict__ Bfull,
                                                             double* __restrict__ Bp_out,
                                                             int nqb, double* __restrict__ zero_out) {
  if (zero_out && blockIdx.x == 0 && threadIdx.x == 0) *zero_out = 0.0;
  const int fx = blockIdx.x / nqb, qb = blockIdx.x - fx * nqb;
  const FragInfo fi = frag[fx];
  const int q0 = (qb * 4 + (threadIdx.x >> 6)) * kMomQW;
  if (q0 >= fi.naux) return;
  const int lane = threadIdx.x & 63;
  const int nq = min(kMomQW, fi.naux - q0);
  const int n = fi.nbf, nt = n * (n + 1) / 2, nn = n * n;
  const int64_t ob = off_Bp[fx] + (int64_t)q0 * nt, od = off_tri[fx];
  const double* b = kPack ? nullptr : Bsrc + ob;
  const double* bf = kPack ? Bfull + fi.off_B + (int64_t)q0 * nn : nullptr;
  double* bo = kPack ? Bp_out + ob : nullptr;
  const double* d = Dw + od;
  double acc[kMomQW];
#pragma unroll
  for (int q = 0; q < kMomQW; ++q) acc[q] = 0.0;
  if ((nt & 1) == 0 && (ob & 1) == 0 && (od & 1) == 0 && nt <= 384) {
    // rows past nq re-read row nq - 1 (their sums are not stored), and
    // positions past nt re-read the row's last pair with density weight 0
    // (adding +-0 leaves the sum unchanged)
    double2 dv[3];
    int kc[3], s0[3], s1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = 2 * lane + 128 * c;
      kc[c] = min(k, nt - 2);
      dv[c] = k < nt ? *reinterpret_cast<const double2*>(d + k) : double2{0.0, 0.0};
      if (kPack) {
        int mu, nu;
        tri_row_col(kc[c], n, mu, nu);
        s0[c] = mu * n + nu;
        tri_row_col(kc[c] + 1, n, mu, nu);
        s1[c] = mu * n + nu;
      }
    }
    double2 bv[kMomQW][3];
#pragma unroll
    for (int q = 0; q < kMomQW; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t row = min(q, nq - 1);
        if (kPack) {
          bv[q][c].x = bf[row * nn + s0[c]];
          bv[q][c].y = bf[row * nn + s1[c]];
        } else {
          bv[q][c] = *reinterpret_cast<const double2*>(b + row * nt + kc[c]);
        }
      }
    __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the arithmetic
#pragma unroll
    for (int q = 0; q < kMomQW; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[q] = fma(bv[q][c].y, dv[c].y, fma(bv[q][c].x, dv[c].x, acc[q]));
    if (kPack)
#pragma unroll
      for (int q = 0; q < kMomQW; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          if (q < nq && 2 * lane + 128 * c < nt)
            *reinterpret_cast<double2*>(bo + (int64_t)q * nt + 2 * lane + 128 * c) = bv[q][c];
  } else {
    // large or odd triangles: kMomU positions per lane at a time, all of
    // their loads in flight before the products (rows past nq re-read row
    // nq - 1 and positions past nt are clamped, their density weight 0; the
    // products are added in the same k order as one position at a time)
    constexpr int kMomU = 4;
    for (int k0 = lane; k0 < nt; k0 += 64 * kMomU) {
      double dk[kMomU], v[kMomQW][kMomU];
      int kc[kMomU];
#pragma unroll
      for (int u = 0; u < kMomU; ++u) {
        const int k = k0 + 64 * u;
        kc[u] = min(k, nt - 1);
        dk[u] = k < nt ? d[kc[u]] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kMomU; ++u) {
        int s = 0;
        if (kPack) {
          int mu, nu;
          tri_row_col(kc[u], n, mu, nu);
          s = mu * n + nu;
        }
#pragma unroll
        for (int q = 0; q < kMomQW; ++q) {
          const int64_t row = min(q, nq - 1);
          v[q][u] = kPack ? bf[row * nn + s] : b[row * nt + kc[u]];
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // every load ahead of the arithmetic
#pragma unroll
      for (int u = 0; u < kMomU; ++u)
#pragma unroll
        for (int q = 0; q < kMomQW; ++q) {
          if (k0 + 64 * u < nt) acc[q] = fma(v[q][u], dk[u], acc[q]);
          if (kPack && q < nq && k0 + 64 * u < nt) bo[(int64_t)q * nt + k0 + 64 * u] = v[q][u];
        }
    }
  }
#pragma unroll
  for (int q = 0; q < kMomQW; ++q) {
    const double t = wave_sum_dpp(acc[q]);
    if (lane == 0 && q < nq) dmom[fi.off_aux + q0 + q] = t;
  }
}

// out = F0 + h~ + 2 sum_P B[P] phi_P from the packed slices, both mirror
// elements written.  A workgroup takes 64 triangle positions; its four
// waves take the slices P = g mod 4 (four partial sums each, so that loads
// of several slices are in flight), and the four wave sums meet in LDS in a
// fixed order.  Large fragments (the nucleobase's triangle of 11,325
// positions over 450 slices) so spread over many workgroups.
constexpr int kJbK = 64;
__global__ __launch_bounds__(256) void jbuild_packed_kernel(const FragInfo* __restrict__ frag,
                                                           const int64_t* __restrict__ off_Bp,
                                                           const double* __restrict__ Bp,
                                                           const double* __restrict__ phi,
                                                           const double* __restrict__ F0,
                                                           const double* __restrict__ htilde,
                                                           double* __restrict__ out) {
  __shared__ double part[4][kJbK];
  const FragInfo fi = frag[blockIdx.x];
  const int n = fi.nbf, nt = n * (n + 1) / 2;
  if ((int)blockIdx.y * kJbK >= nt) return;  // uniform over the workgroup
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int k = blockIdx.y * kJbK + lane;
  const int kc = min(k, nt - 1);  // every load in bounds; the sum of k >= nt is not stored
  const double* b = Bp + off_Bp[blockIdx.x] + kc;
  const double* ph = phi + fi.off_aux;
  double a4[4] = {0.0, 0.0, 0.0, 0.0};
  int P = g;
#pragma unroll 2
  for (; P + 12 < fi.naux; P += 16)
#pragma unroll
    for (int u = 0; u < 4; ++u) a4[u] = fma(b[(int64_t)(P + 4 * u) * nt], ph[P + 4 * u], a4[u]);
  for (; P < fi.naux; P += 4) a4[0] = fma(b[(int64_t)P * nt], ph[P], a4[0]);
  part[g][lane] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  __syncthreads();
  if (g != 0 || k >= nt) return;
  const double acc = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
  int mu, nu;
  tri_row_col(k, n, mu, nu);
  const double j2 = 2.0 * acc;
  const int64_t o1 = fi.off_C + (int64_t)mu * n + nu, o2 = fi.off_C + (int64_t)nu * n + mu;
  double v1 = j2, v2 = j2;
  if (F0) { v1 += F0[o1]; v2 += F0[o2]; }
  if (htilde) { v1 += htilde[o1]; v2 += htilde[o2]; }
  out[o1] = v1;
  if (mu != nu) out[o2] = v2;
}

// Field and J in one kernel, one workgroup per fragment (every fragment
// small enough that its packed triangle fits one workgroup): the field
// gather of one fragment is latency-bound and its J build streams the
// fragment's coefficients, so workgroups in different phases overlap, and
// phi stays in LDS.
// Staged neighbour entries past a chunk of blockDim (the gather reads up to
// 8 NG - 1 entries beyond a chunk's last, NG <= 8 groups)
constexpr int kStageExtra = 64;
__global__ __launch_bounds__(512) void field_jbuild_packed_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ nbr_ptr,
    const int32_t* __restrict__ nbr_idx, const double* __restrict__ nbr_s,
    const double* __restrict__ G, const int64_t* __restrict__ off_G, int P0, int nclass,
    const int32_t* __restrict__ naux_cls_off, const double* __restrict__ dmom,
    const int64_t* __restrict__ off_Bp, const double* __restrict__ Bp,
    const double* __restrict__ F0, const double* __restrict__ htilde, double* __restrict__ out,
    double* __restrict__ zero_out) {
  // LDS: the staged neighbour chunk (weights [NT + 64], pool offsets
  // [NT + 64]), then [NW][etot] partial e_c (e after the reduction), then
  // phi^x
  extern __shared__ double smem[];
  const int NT = blockDim.x, NW = NT >> 6;
  double* st_s = smem;
  int32_t* st_o = reinterpret_cast<int32_t*>(smem + NT + kStageExtra);
  double* part = smem + NT + kStageExtra + (NT + kStageExtra) / 2;
  __shared__ int32_t other_cls;
  // zero_out non-null: one thread clears it (a maximum that a later kernel
  // of the same step accumulates; set when no moments kernel runs)
  if (zero_out && blockIdx.x == 0 && threadIdx.x == 0) *zero_out = 0.0;
  // fragments in reverse order: the moments kernel before it streamed the
  // slices forwards, so the last ones it read are the first ones read here
  const int x = gridDim.x - 1 - blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int etot = naux_cls_off[nclass];
  for (int t = threadIdx.x; t < NW * etot; t += NT) part[t] = 0.0;
  const int beg = nbr_ptr[x], end = nbr_ptr[x + 1];
  // class-0 neighbours: NG groups of P0 threads, thread (g, q) sums
  // s_xy d^y_q over the chunk's neighbours j = g, g + NG, ..., eight loads
  // in flight; entries past the chunk carry weight 0 and offset 0, and a
  // neighbour of another class is parked the same way (its sum is formed
  // below), so the loop has no branches
  const int NG = NT >= P0 ? min(NW, NT / P0) : 1;
  for (int c0 = beg; c0 < end; c0 += NT) {
    const int cnt = min(NT, end - c0);
    if (threadIdx.x == 0) other_cls = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < NT + kStageExtra; t += NT) {
      double s = 0.0;
      int32_t o = 0;
      if (t < cnt) {
        const int y = nbr_idx[c0 + t];
        const FragInfo fy = frag[y];
        if (fy.cls == 0) {
          s = nbr_s[c0 + t];
          o = (int32_t)fy.off_aux;
        } else {
          other_cls = 1;
        }
      }
      st_s[t] = s;
      st_o[t] = o;
    }
    __syncthreads();
    const int per = (cnt + NG - 1) / NG;
    const int nb8 = (per + 7) / 8;
    for (int u = threadIdx.x; u < NG * P0; u += NT) {
      const int g = u / P0, q = u - g * P0;
      double acc = 0.0;
      for (int b = 0; b < nb8; ++b) {
        const int j = g + 8 * NG * b;
        double sv[8], dv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          sv[k] = st_s[j + k * NG];
          dv[k] = dmom[st_o[j + k * NG] + q];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) acc = fma(sv[k], dv[k], acc);
      }
      part[g * etot + q] += acc;
    }
    // neighbours of other classes (rare): wave 0, one neighbour at a time,
    // into the class sums of group 0
    if (wave == 0 && other_cls) {
      for (int j = 0; j < cnt; ++j) {
        const int y = nbr_idx[c0 + j];
        const FragInfo fy = frag[y];
        if (fy.cls == 0) continue;
        const double s = nbr_s[c0 + j];
        const double* dy = dmom + fy.off_aux;
        const int base = naux_cls_off[fy.cls];
        for (int q = lane; q < fy.naux; q += 64) part[base + q] = fma(s, dy[q], part[base + q]);
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < etot; q += NT) {
    double s = part[q];
    for (int w = 1; w < NW; ++w) s += part[w * etot + q];
    part[q] = s;
  }
  __syncthreads();
  double* phis = part + NW * etot;
  const FragInfo fx = frag[x];
  const int cx = fx.cls, naux = fx.naux;
  const int pc0 = naux_cls_off[1] - naux_cls_off[0], qs = (pc0 + 3) / 4;
  double* red4 = part + etot;
  const bool quarter = cx == 0 && 4 * naux <= (int)blockDim.x && 4 * naux <= (NW - 1) * etot;
  if (quarter) {
    const int g = threadIdx.x / naux, p = threadIdx.x - g * naux;
    if (g < 4) {
      const double* e0c = part + naux_cls_off[0];
      const int q1 = min(pc0, (g + 1) * qs);
      double acc = 0.0;
      int q = g * qs;
      for (; q + 8 <= q1; q += 8) {
        double g8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) g8[u] = G[(int64_t)(q + u) * P0 + p];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(g8[u], e0c[q + u], acc);
      }
      for (; q < q1; ++q) acc = fma(G[(int64_t)q * P0 + p], e0c[q], acc);
      red4[g * naux + p] = acc;
    }
    __syncthreads();
  }
  for (int p = threadIdx.x; p < naux; p += blockDim.x) {
    double acc = quarter ? (red4[p] + red4[naux + p]) + (red4[2 * naux + p] + red4[3 * naux + p]) : 0.0;
    for (int c = 0; c < nclass; ++c) {
      const int pc = naux_cls_off[c + 1] - naux_cls_off[c];
      const double* ec = part + naux_cls_off[c];
      if (c == 0 && cx == 0 && quarter) {
        continue;
      } else if (c == 0 && cx == 0) {
        // G_{0,0} is symmetric: read it by columns, so that consecutive
        // threads (rows p) load consecutive addresses; eight columns' loads
        // in flight at a time
        int q = 0;
        for (; q + 8 <= pc; q += 8) {
          double g8[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) g8[u] = G[(int64_t)(q + u) * P0 + p];
#pragma unroll
          for (int u = 0; u < 8; ++u) acc = fma(g8[u], ec[q + u], acc);
        }
        for (; q < pc; ++q) acc = fma(G[(int64_t)q * P0 + p], ec[q], acc);
      } else if (c == 0) {
        const double* g = G + off_G[cx];  // G_{cx,0}: [P_cx][P0]
        for (int q = 0; q < pc; ++q) acc = fma(g[(int64_t)p * P0 + q], ec[q], acc);
      } else if (cx == 0) {
        const double* g = G + off_G[c];   // G_{c,0}: [P_c][P0]; use its transpose
        for (int q = 0; q < pc; ++q) acc = fma(g[(int64_t)q * P0 + p], ec[q], acc);
      }
    }
    phis[p] = acc;
  }
  __syncthreads();
  // J = 2 sum_P B[P] phi_P from the packed slices; F~ = F0 + h~ + J, both
  // mirror elements written (as jbuild_packed_kernel)
  const int n = fx.nbf, nt = n * (n + 1) / 2;
  const double* bx = Bp + off_Bp[x];
  const int H = nt / 2;
  if ((nt & 1) == 0 && (off_Bp[x] & 1) == 0 && 2 * H <= (int)blockDim.x && nt <= NW * etot) {
    // pairs of elements with 16-byte loads: threads [0, H) take the even
    // slices, [H, 2H) the odd ones, and the two partial sums meet in LDS
    // (the e_c area is free now)
    double* jbuf = part;
    const int tid = threadIdx.x, half = tid >= H ? 1 : 0, m = tid - half * H;
    double2 acc2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc2[u] = double2{0.0, 0.0};
    if (tid < 2 * H) {
      const double* b = bx + 2 * m;
      int P = half;
      for (; P + 14 < fx.naux; P += 16) {
        double2 bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) bv[u] = *reinterpret_cast<const double2*>(b + (int64_t)(P + 2 * u) * nt);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double ph = phis[P + 2 * u];
          acc2[u & 3].x = fma(bv[u].x, ph, acc2[u & 3].x);
          acc2[u & 3].y = fma(bv[u].y, ph, acc2[u & 3].y);
        }
      }
      for (; P < fx.naux; P += 2) {
        const double2 bv = *reinterpret_cast<const double2*>(b + (int64_t)P * nt);
        acc2[0].x = fma(bv.x, phis[P], acc2[0].x);
        acc2[0].y = fma(bv.y, phis[P], acc2[0].y);
      }
    }
    const double sx = (acc2[0].x + acc2[1].x) + (acc2[2].x + acc2[3].x);
    const double sy = (acc2[0].y + acc2[1].y) + (acc2[2].y + acc2[3].y);
    if (half == 1 && m < H) { jbuf[2 * m] = sx; jbuf[2 * m + 1] = sy; }
    __syncthreads();
    if (half == 0 && m < H) {
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const int kk = 2 * m + w;
        const double j2 = 2.0 * ((w ? sy : sx) + jbuf[kk]);
        int mu, nu;
        tri_row_col(kk, n, mu, nu);
        const int64_t o1 = fx.off_C + (int64_t)mu * n + nu, o2 = fx.off_C + (int64_t)nu * n + mu;
        double v1 = j2, v2 = j2;
        if (F0) { v1 += F0[o1]; v2 += F0[o2]; }
        if (htilde) { v1 += htilde[o1]; v2 += htilde[o2]; }
        out[o1] = v1;
        if (mu != nu) out[o2] = v2;
      }
    }
    return;
  }
  for (int kk = threadIdx.x; kk < nt; kk += blockDim.x) {
    const double* b = bx + kk;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    int P = 0;
#pragma unroll 4
    for (; P + 4 <= fx.naux; P += 4)
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u] = fma(b[(int64_t)(P + u) * nt], phis[P + u], a4[u]);
    for (; P < fx.naux; ++P) a4[0] = fma(b[(int64_t)P * nt], phis[P], a4[0]);
    const double j2 = 2.0 * ((a4[0] + a4[1]) + (a4[2] + a4[3]));
    int mu, nu;
    tri_row_col(kk, n, mu, nu);
    const int64_t o1 = fx.off_C + (int64_t)mu * n + nu, o2 = fx.off_C + (int64_t)nu * n + mu;
    double v1 = j2, v2 = j2;
    if (F0) { v1 += F0[o1]; v2 += F0[o2]; }
    if (htilde) { v1 += htilde[o1]; v2 += htilde[o2]; }
    out[o1] = v1;
    if (mu != nu) out[o2] = v2;
  }
}

hipError_t launch_pack_coefficients(const fef_plan_s& p, const double* B, double* Bp,
                                    hipStream_t st) {
  if (p.nfrag == 0) return hipSuccess;
  hipLaunchKernelGGL(pack_coefficients_kernel, dim3((unsigned)p.n_chunk_Bp), dim3(256), 0, st,
                     p.d_frag, p.d_chunk_Bp, p.d_off_Bp, B, Bp);
  return hipGetLastError();
}

hipError_t launch_field_packed(const fef_plan_s& p, const double* Bp, const double* G,
                               const double* Dw, const double* F0, const double* htilde,
                               double* out, double* ws_d, double* ws_phi, hipStream_t st,
                               const double* B_pack, double* Bp_out, double* zero_out,
                               bool moments_given) {
  const int nqb = (p.max_naux + 4 * kMomQW - 1) / (4 * kMomQW);
  const dim3 mgrid((unsigned)((int64_t)p.nfrag * nqb));
  if (moments_given) {
    // ws_d already holds the moments (left there by the previous step's
    // eigensolver); the fused field kernel clears zero_out instead
  } else if (B_pack)
    hipLaunchKernelGGL(moments_packed_kernel<true>, mgrid, dim3(256), 0, st, p.d_frag, p.d_off_Bp,
                       p.d_off_tri, nullptr, Dw, ws_d, B_pack, Bp_out, nqb, zero_out);
  else
    hipLaunchKernelGGL(moments_packed_kernel<false>, mgrid, dim3(256), 0, st, p.d_frag, p.d_off_Bp,
                       p.d_off_tri, Bp, Dw, ws_d, nullptr, nullptr, nqb, zero_out);
  stage_mark(p, 2, st);
  if (moments_given && !small_fragments(p)) return hipErrorInvalidValue;
  const int etot = p.naux_cls_off.back();
  const int ntmax = p.max_nbf * (p.max_nbf + 1) / 2;
  if (small_fragments(p)) {
    // all fragments small: field and J fused (water: 320 threads)
    const int jt = std::min(512, (ntmax + 63) / 64 * 64);
    // the staged neighbour offsets are 32-bit
    if (naux_total(p) > INT32_MAX) return hipErrorInvalidValue;
    const size_t lds = ((size_t)(jt / 64) * etot + p.max_naux + (jt + kStageExtra) +
                        (jt + kStageExtra) / 2) * sizeof(double);
    hipLaunchKernelGGL(field_jbuild_packed_kernel, dim3(p.nfrag), dim3(jt), lds, st, p.d_frag,
                       p.d_nbr_ptr, p.d_nbr_idx, p.d_nbr_s, G, p.d_off_G, p.P0, p.nclass,
                       p.d_naux_cls_off, ws_d, p.d_off_Bp, Bp, F0, htilde, out,
                       moments_given ? zero_out : nullptr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(field_kernel, dim3(p.nfrag), dim3(256), 4 * etot * sizeof(double), st, p.d_frag,
                     p.d_nbr_ptr, p.d_nbr_idx, p.d_nbr_s, G, p.d_off_G, p.P0, p.nclass,
                     p.d_naux_cls_off, ws_d, ws_phi);
  hipLaunchKernelGGL(jbuild_packed_kernel, dim3(p.nfrag, (ntmax + kJbK - 1) / kJbK), dim3(256), 0,
                     st, p.d_frag, p.d_off_Bp, Bp, ws_phi, F0, htilde, out);
  return hipGetLastError();
}

bool small_fragments(const fef_plan_s& p) { return p.max_nbf <= 32 && p.max_naux <= 80; }

hipError_t launch_zero_scalar(double* x, hipStream_t st) {
  hipLaunchKernelGGL(zero_scalar_kernel, dim3(1), dim3(1), 0, st, x);
  return hipGetLastError();
}

hipError_t launch_density(const fef_plan_s& p, const double* C, double* D, double* Dw,
                          double* dD_max, hipStream_t st) {
  if (p.nfrag == 0) {
    hipLaunchKernelGGL(zero_scalar_kernel, dim3(1), dim3(1), 0, st, dD_max);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(density_kernel, dim3((unsigned)p.n_chunk_C), dim3(256), 0, st, p.d_frag,
                     p.d_chunk_C, p.d_off_tri, C, D, Dw, dD_max);
  return hipGetLastError();
}

hipError_t launch_moments(const fef_plan_s& p, const double* B, const double* D, double* dmom,
                          hipStream_t st) {
  hipLaunchKernelGGL(moments_kernel, dim3(p.nfrag, (p.max_naux + 4 * kMomQ - 1) / (4 * kMomQ)),
                     dim3(256), 0, st, p.d_frag, B, D, dmom);
  return hipGetLastError();
}

hipError_t launch_field(const fef_plan_s& p, const double* B, const double* G, const double* D,
                        const double* F0, const double* htilde, double* out, double* ws_d,
                        double* ws_phi, hipStream_t st) {
  hipLaunchKernelGGL(moments_kernel, dim3(p.nfrag, (p.max_naux + 4 * kMomQ - 1) / (4 * kMomQ)),
                     dim3(256), 0, st, p.d_frag, B, D, ws_d);
  stage_mark(p, 2, st);
  const int etot = p.naux_cls_off.back();
  hipLaunchKernelGGL(field_kernel, dim3(p.nfrag), dim3(256), 4 * etot * sizeof(double), st, p.d_frag,
                     p.d_nbr_ptr, p.d_nbr_idx, p.d_nbr_s, G, p.d_off_G, p.P0, p.nclass,
                     p.d_naux_cls_off, ws_d, ws_phi);
  const int nnmax = p.max_nbf * p.max_nbf;
  hipLaunchKernelGGL(jbuild_kernel, dim3(p.nfrag, (nnmax + 511) / 512), dim3(256), 0, st,
                     p.d_frag, B, ws_phi, F0, htilde, out);
  return hipGetLastError();
}

}  // namespace fef
