// Half transform of the factored integrals (x-side half of the AO -> MO
// transform) and packing of the pair-kernel operands.
//
//   B_ov^x[P][ia] = sum_{mu nu} C^x_{mu i} B^x[P][mu][nu] C^x_{nu a}
//   W^x[Q][ia]    = sum_P G_{c(x),0}[P][Q] B_ov^x[P][ia]
//
// The contraction is done occupied side first (X = C_occ^T B_P, then
// X C_vir), the cheaper order for nocc < nvir.  Both steps read every element
// of B once; the kernel is bound by HBM bandwidth.
#include <algorithm>

#include "fef_internal.h"
#include "fef_device.h"
#include "fef_split.h"

namespace fef {

// Half transform of small fragments (nbf <= 32, one 96-wide tile, P_c <= 80)
// in two kernels.
//  ht_mo_small_kernel: one workgroup per (fragment, kSliceGroup factor
//    slices), fragment-major (the nsg slice groups of a fragment are
//    adjacent in the 1-D grid, so B is streamed in order and the
//    fragment's C is reused from cache): the slices of B^x are copied into
//    LDS (global_load_lds, 16 bytes per lane), then X = C_occ^T B_P and
//    B_ov = X C_vir are formed from LDS and B_ov is written densely.  Small groups keep the LDS of a
//    workgroup at 27 KB (nbf = 24), so five share a CU and the copies of
//    some overlap the contractions of others.
//  ht_pack_small_kernel: one workgroup (eight waves) per fragment: B_ov^x in LDS, W^x =
//    G^T B_ov^x on FP64 MFMA (accumulators stay in registers), and both
//    pair-kernel operands of mode PREC written directly (FP16 scales from
//    block-wide maxima).
constexpr int kSmallP = 80, kSliceGroup = 4;

__global__ __launch_bounds__(256) void ht_mo_small_kernel(const FragInfo* __restrict__ frag,
                                                          const int32_t* __restrict__ list,
                                                          const double* __restrict__ B,
                                                          const double* __restrict__ C,
                                                          double* __restrict__ bov, int max_nn,
                                                          int nsg) {
  extern __shared__ double sm[];
  const int cs_ld = (max_nn + 1) & ~1;              // keeps Bst 16-byte aligned
  double* Cs = sm;                                  // [nbf][nbf]
  double* Bst = sm + cs_ld;                         // [kSliceGroup][nbf][nbf]
  double* Xs = sm + cs_ld + kSliceGroup * max_nn;   // [kSliceGroup][nocc][nbf]
  const int fx = blockIdx.x / nsg, sg = blockIdx.x - fx * nsg;
  const FragInfo fi = frag[list[fx]];
  const int p0 = sg * kSliceGroup;
  if (p0 >= fi.naux) return;
  const int np = min(kSliceGroup, fi.naux - p0);
  const int n = fi.nbf, o = fi.nocc, v = fi.nvir, ov = fi.ov, nn = n * n;
  const double* src = B + fi.off_B + (int64_t)p0 * nn;
  const int tot = np * nn;
  if ((tot & 1) == 0 && ((fi.off_B + (int64_t)p0 * nn) & 1) == 0) {
    // the slices go straight into LDS, 16 bytes per lane, every piece of
    // the block in flight at once (wave w moves the 1 KB pieces w, w + 4, ...)
    const int nch = tot / 2, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int g = wave; g * 64 < nch; g += 4) {
      const int c = g * 64 + lane;
      if (c < nch)
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(src + 2 * (int64_t)c),
                                         (lds_void_t*)(Bst + 128 * g), 16, 0, 0);
    }
  } else {
    for (int e = threadIdx.x; e < tot; e += 256) Bst[e] = src[e];
  }
  {  // C (nn <= 1024): four loads per thread in flight, clamped addresses
    double cv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) cv[u] = C[fi.off_C + min((int)threadIdx.x + 256 * u, nn - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if ((int)threadIdx.x + 256 * u < nn) Cs[threadIdx.x + 256 * u] = cv[u];
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int e = threadIdx.x; e < np * o * n; e += 256) {  // X = C_occ^T B_P
    const int pp = e / (o * n), r = e - pp * (o * n);
    const int i = r / n, nu = r - (r / n) * n;
    const double* b = Bst + pp * nn + nu;
    double acc = 0.0;
#pragma unroll 8
    for (int mu = 0; mu < n; ++mu) acc = fma(Cs[mu * n + i], b[mu * n], acc);
    Xs[e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < np * ov; e += 256) {  // B_ov = X C_vir
    const int pp = e / ov, r = e - pp * ov;
    const int i = r / v, a = r - (r / v) * v;
    const double* xr = Xs + (pp * o + i) * n;
    double acc = 0.0;
#pragma unroll 8
    for (int nu = 0; nu < n; ++nu) acc = fma(xr[nu], Cs[nu * n + o + a], acc);
    bov[fi.off_bov + (int64_t)(p0 + pp) * ov + r] = acc;
  }
}

// Eight waves per workgroup: with the 62 KB LDS buffer two workgroups share
// a CU, and the extra waves hide the latency of the staging loads and of the
// operand stores.
constexpr int kPackThreads = 512;
template <int PREC>
__global__ __launch_bounds__(kPackThreads) void ht_pack_small_kernel(
    const FragInfo* __restrict__ frag, const int32_t* __restrict__ list,
    const double* __restrict__ bov, const double* __restrict__ G,
    const int64_t* __restrict__ off_G, int P0, int kpad, int pw, double* __restrict__ w_out,
    char* __restrict__ ops) {
  // Bs [P][kBld]: B_ov, zero past ov and past P (to a multiple of 4); the
  // split modes later reuse it as W^T [ia][P0 + 1] for coalesced packing
  constexpr int kBld = kTile + 1;
  __shared__ double Bs[(kSmallP * kBld > kTile * (kSmallP + 1)) ? kSmallP * kBld
                                                                 : kTile * (kSmallP + 1)];
  __shared__ double red[kPackThreads / 64];
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  const int ov = fi.ov, P = fi.naux;
  const int P4 = (P + 3) & ~3;
  // sixteen loads per thread in flight: positions outside B_ov load its first
  // element and store zero
  for (int eb = threadIdx.x; eb < P4 * kTile; eb += kPackThreads * 16) {
    double v16[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = eb + kPackThreads * u;
      const int pp = e / kTile, ia = e - (e / kTile) * kTile;
      const bool in = e < P4 * kTile && pp < P && ia < ov;
      const double x = bov[fi.off_bov + (in ? (int64_t)pp * ov + ia : 0)];
      v16[u] = in ? x : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = eb + kPackThreads * u;
      if (e < P4 * kTile) Bs[(e / kTile) * kBld + (e - (e / kTile) * kTile)] = v16[u];
    }
  }
  __syncthreads();
  // W = G_{c,0}^T B_ov on FP64 MFMA (16x16x4): output tiles (q tile, ia
  // tile) in q-major order, four consecutive tiles per wave (eight waves),
  // so that a wave meets at most two q tiles.  The A operands (G^T, from
  // the L2-resident coupling) of those two q tiles are loaded one k step
  // ahead; B comes from LDS.
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const double* g = G + off_G[fi.cls];  // [P][P0]
  constexpr int kIT = kTile / 16;
  const int QT = (P0 + 15) >> 4, NT = QT * kIT;
  constexpr int kTilesPerWave = (5 * kIT + kPackThreads / 64 - 1) / (kPackThreads / 64);
  constexpr int kSteps = kSmallP / 4;               // 20
  const int t0 = wave * kTilesPerWave;
  const int qa = t0 / kIT;  // first q tile of this wave; the other is qa + 1
  // A operands streamed one k step ahead (two L2 loads per step)
  auto ga_load = [&](int ks, int h) {
    const int pp = 4 * ks + lk, q = 16 * (qa + h) + li;
    const bool in = pp < P && q < P0;
    const double x = g[in ? (int64_t)pp * P0 + q : 0];
    return in ? x : 0.0;
  };
  d4 acc[kTilesPerWave];
#pragma unroll
  for (int k = 0; k < kTilesPerWave; ++k) acc[k] = d4{0, 0, 0, 0};
  // every tile of the wave is contracted, also tiles past NT (their B
  // columns are in range and their A values finite; they are never
  // stored), so that a k step's eight LDS reads are issued before its MFMAs
  double gc0 = ga_load(0, 0), gc1 = ga_load(0, 1);
#pragma unroll
  for (int ks = 0; ks < kSteps; ++ks) {
    if (4 * ks >= P4) break;  // rows past P4 are not staged
    const int pp = 4 * ks + lk;
    const double gn0 = ks + 1 < kSteps ? ga_load(ks + 1, 0) : 0.0;
    const double gn1 = ks + 1 < kSteps ? ga_load(ks + 1, 1) : 0.0;
    double bv[kTilesPerWave];
#pragma unroll
    for (int k = 0; k < kTilesPerWave; ++k) {
      const int tt = t0 + k, qt = tt / kIT, it = tt - qt * kIT;
      bv[k] = Bs[pp * kBld + 16 * it + li];
    }
#pragma unroll
    for (int k = 0; k < kTilesPerWave; ++k) {
      const int qt = (t0 + k) / kIT;
      const double av = qt == qa ? gc0 : gc1;
      acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[k], acc[k], 0, 0, 0);
    }
    gc0 = gn0;
    gc1 = gn1;
  }
  // element (r) of tile k: q = 16 qt + lk + 4 r, ia = 16 it + li
  double wmax = 0.0, bmax = 0.0;
#pragma unroll
  for (int k = 0; k < kTilesPerWave; ++k) {
    const int t = t0 + k;
    if (t < NT) {
      const int qt = t / (kTile / 16), it = t - qt * (kTile / 16);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = 16 * qt + lk + 4 * r, ia = 16 * it + li;
        if (q < P0 && ia < ov) {
          wmax = fmax(wmax, fabs(acc[k][r]));
          if (w_out) w_out[fi.off_w + (int64_t)q * ov + ia] = acc[k][r];
        }
      }
    }
  }
  for (int e = threadIdx.x; e < P * kTile; e += kPackThreads)
    bmax = fmax(bmax, fabs(Bs[(e / kTile) * kBld + (e - (e / kTile) * kTile)]));
  const bool right = fi.off_R[PREC] >= 0;
  if (PREC == FEF_F64 || PREC == FEF_F32) {
    typedef typename std::conditional<PREC == FEF_F64, double, float>::type T;
    T* L = reinterpret_cast<T*>(ops + fi.off_L[PREC]);
    T* R = right ? reinterpret_cast<T*>(ops + fi.off_R[PREC]) : nullptr;
    // [kpad][ld]: values, then zeros in the padding
#pragma unroll
    for (int k = 0; k < kTilesPerWave; ++k) {
      const int t = t0 + k;
      if (t < NT) {
        const int qt = t / (kTile / 16), it = t - qt * (kTile / 16);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = 16 * qt + lk + 4 * r, ia = 16 * it + li;
          if (q < P0 && ia < ov) L[(int64_t)q * fi.ld + ia] = (T)acc[k][r];
        }
      }
    }
    for (int e = threadIdx.x; e < kpad * kTile; e += kPackThreads) {
      const int k = e / kTile, m = e - (e / kTile) * kTile;
      if (k >= P0 || m >= ov) {
        L[(int64_t)k * fi.ld + m] = (T)0;
        if (R) R[(int64_t)k * fi.ld + m] = (T)0;
      } else if (R) {
        R[(int64_t)k * fi.ld + m] = (T)Bs[k * kBld + m];
      }
    }
  } else {
    constexpr bool kF16 = PREC == FEF_FP16X2;
    wmax = block_max(wmax, red);
    bmax = block_max(bmax, red);
    const double sL = kF16 ? split_scale(wmax) : 1.0;
    const double sR = kF16 ? split_scale(bmax) : 1.0;
    double* hdr = reinterpret_cast<double*>(ops);
    if (threadIdx.x == 0) {
      hdr[2 * f] = 1.0 / sL;
      hdr[2 * f + 1] = 1.0 / sR;
    }
    constexpr int NTERM = split_nterm(PREC);
    const int xs = NTERM * pw + 8;
    uint16_t* L = reinterpret_cast<uint16_t*>(ops + fi.off_L[PREC]);
    uint16_t* R = right ? reinterpret_cast<uint16_t*>(ops + fi.off_R[PREC]) : nullptr;
    // rows [ia][plane 0 | plane 1 | ... | 8 zeros], written in 16-byte
    // pieces: a thread splits eight consecutive q of one row and stores their
    // terms; rows >= ov and q >= P0 are zeros, so no separate zero fill
    const int nqc = pw / 8;
    const u16x8 z8 = {0, 0, 0, 0, 0, 0, 0, 0};
    if (R)
      for (int e = threadIdx.x; e < kTile * (nqc + 1); e += kPackThreads) {
        const int ia = e / (nqc + 1), c = e - (e / (nqc + 1)) * (nqc + 1);
        if (c == nqc) {
          *reinterpret_cast<u16x8*>(R + ia * xs + NTERM * pw) = z8;
          continue;
        }
        u16x8 h[NTERM];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int q = 8 * c + u;
          uint16_t tv[NTERM] = {};
          if (ia < ov && q < P0) split_terms<PREC, NTERM>(Bs[q * kBld + ia] * sR, tv);
#pragma unroll
          for (int k = 0; k < NTERM; ++k) h[k][u] = tv[k];
        }
#pragma unroll
        for (int k = 0; k < NTERM; ++k)
          *reinterpret_cast<u16x8*>(R + ia * xs + k * pw + 8 * c) = h[k];
      }
    __syncthreads();  // Bs is rewritten with W^T below
    const int wld = P0 + 1;
#pragma unroll
    for (int k = 0; k < kTilesPerWave; ++k) {
      const int t = t0 + k;
      if (t < NT) {
        const int qt = t / (kTile / 16), it = t - qt * (kTile / 16);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = 16 * qt + lk + 4 * r, ia = 16 * it + li;
          if (q < P0 && ia < ov) Bs[ia * wld + q] = acc[k][r];
        }
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kTile * (nqc + 1); e += kPackThreads) {
      const int ia = e / (nqc + 1), c = e - (e / (nqc + 1)) * (nqc + 1);
      if (c == nqc) {
        *reinterpret_cast<u16x8*>(L + ia * xs + NTERM * pw) = z8;
        continue;
      }
      u16x8 h[NTERM];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = 8 * c + u;
        uint16_t tv[NTERM] = {};
        if (ia < ov && q < P0) split_terms<PREC, NTERM>(Bs[ia * wld + q] * sL, tv);
#pragma unroll
        for (int k = 0; k < NTERM; ++k) h[k][u] = tv[k];
      }
#pragma unroll
      for (int k = 0; k < NTERM; ++k)
        *reinterpret_cast<u16x8*>(L + ia * xs + k * pw + 8 * c) = h[k];
    }
  }
}

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

// W = G_{c,0}^T B_ov for the generic fragments: block (fragment, 8 q, 256
// ia); each thread keeps the 8 q sums of its ia, so every B_ov load feeds 8
// FMAs and the G values are broadcast.
__global__ __launch_bounds__(256) void ht_w_kernel(const FragInfo* __restrict__ frag,
                                                   const int32_t* __restrict__ list,
                                                   const double* __restrict__ G,
                                                   const int64_t* __restrict__ off_G, int P0,
                                                   const double* __restrict__ bov,
                                                   double* __restrict__ w) {
  const FragInfo fi = frag[list[blockIdx.x]];
  const int ia = blockIdx.z * 256 + threadIdx.x;
  if (fi.ov == 0 || ia >= fi.ov) return;
  const double* g = G + off_G[fi.cls];  // [P_c][P0]
  const double* b = bov + fi.off_bov;   // [P_c][ov]
  const int q0 = blockIdx.y * 8;
  const int nq = min(8, P0 - q0);
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int P = 0; P < fi.naux; ++P) {
    const double bv = b[(int64_t)P * fi.ov + ia];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < nq) acc[k] = fma(g[(int64_t)P * P0 + q0 + k], bv, acc[k]);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k < nq) w[fi.off_w + (int64_t)(q0 + k) * fi.ov + ia] = acc[k];
}

// Operand pool, FP64 / FP32 modes: L^x = W^x and R^y = B_ov^y stored
// [kpad][ld] (row k, column ia), zero padded in both directions.
template <typename T>
__global__ __launch_bounds__(256) void pack_plain_kernel(const FragInfo* __restrict__ frag,
                                                         const int32_t* __restrict__ list,
                                                         int P0, int kpad, int prec,
                                                         const double* __restrict__ bov,
                                                         const double* __restrict__ w,
                                                         char* __restrict__ ops) {
  const FragInfo fi = frag[list[blockIdx.x]];
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
                                 fef_prec prec, hipStream_t st, bool dense_out) {
  char* o = static_cast<char*>(ops);
  const int kpad = p.geom[prec].kpad, pw = p.geom[prec].pw;
  if (!p.ht_fused.empty()) {
    double* wo = dense_out ? w : nullptr;
    const dim3 grid((unsigned)p.ht_fused.size());
    const size_t lds = (size_t)(((p.fuse_lds[0] + 1) & ~1) + kSliceGroup * p.fuse_lds[0] +
                                kSliceGroup * p.fuse_lds[1]) *
                       sizeof(double);
    const int nsg = (p.max_naux_small + kSliceGroup - 1) / kSliceGroup;
    hipLaunchKernelGGL(ht_mo_small_kernel, dim3((unsigned)((int64_t)grid.x * nsg)),
                       dim3(256), lds, st, p.d_frag, p.d_ht_fused, B, C, bov, p.fuse_lds[0], nsg);
#define FEF_FUSED(M)                                                                              \
  hipLaunchKernelGGL(ht_pack_small_kernel<M>, grid, dim3(kPackThreads), 0, st, p.d_frag, p.d_ht_fused,     \
                     bov, G, p.d_off_G, p.P0, kpad, pw, wo, o)
    switch (prec) {
      case FEF_F64: FEF_FUSED(FEF_F64); break;
      case FEF_F32: FEF_FUSED(FEF_F32); break;
      case FEF_BF16X2: FEF_FUSED(FEF_BF16X2); break;
      case FEF_BF16X3: FEF_FUSED(FEF_BF16X3); break;
      default: FEF_FUSED(FEF_FP16X2); break;
    }
#undef FEF_FUSED
  }
  if (!p.ht_generic.empty()) {
    const unsigned ng = (unsigned)p.ht_generic.size();
    if (p.ht_ntasks > 0) {
      const size_t lds = (size_t)std::max<int64_t>(p.max_on, 1) * sizeof(double);
      hipLaunchKernelGGL(ht_bov_kernel, dim3((unsigned)p.ht_ntasks), dim3(256), lds, st,
                         p.d_frag, p.d_ht, B, C, bov);
      hipLaunchKernelGGL(ht_w_kernel, dim3(ng, (p.P0 + 7) / 8, (p.max_ov + 255) / 256), dim3(256),
                         0, st, p.d_frag,
                         p.d_ht_generic, G, p.d_off_G, p.P0, bov, w);
    }
    switch (prec) {
      case FEF_F64:
        hipLaunchKernelGGL(pack_plain_kernel<double>, dim3(ng, kpad), dim3(256), 0, st, p.d_frag,
                           p.d_ht_generic, p.P0, kpad, (int)prec, bov, w, o);
        break;
      case FEF_F32:
        hipLaunchKernelGGL(pack_plain_kernel<float>, dim3(ng, kpad), dim3(256), 0, st, p.d_frag,
                           p.d_ht_generic, p.P0, kpad, (int)prec, bov, w, o);
        break;
      default: {
        hipError_t e = launch_pack_split(p, bov, w, ops, prec, st);
        if (e != hipSuccess) return e;
      }
    }
  }
  return hipGetLastError();
}


}  // namespace fef
