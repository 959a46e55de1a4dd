// Split-precision pair contraction (BF16 or FP16 terms, FP32 MFMA
// accumulation, FP64 weighting and sums).
//
// Each operand value x is stored as nterm 16-bit terms: two (BF16X2,
// FP16X2: x ~ t0 + t1) or three (BF16X3: x ~ t0 + t1 + t2), each term the
// nearest 16-bit value to what the earlier terms leave.  A stored row (one
// per ia) holds the term planes t0 | t1 [| t2], each pw = round_up(P0, 8)
// wide, then 8 zeros.  The product keeps the terms of order up to nterm - 1
// (order = the sum of the two terms' plane indices): order 0 is t0 t0',
// order 1 is t0 t1' + t1 t0', order 2 is t0 t2' + t1 t1' + t2 t0'.
// Two terms: the three products run as one MFMA chain over a concatenated
// contraction axis of 3 pw indices (x planes t0, t0, t1 against y planes
// t0, t1, t0), padded to chunks of 32 with the row's zero tail.  Three
// terms: the products of one order form one chain (x reads the planes
// 0..L concatenated, y the same planes in reverse order, over (L + 1) pw
// indices), and the chains run from the highest order to the lowest into
// one FP32 accumulator, so that x needs only the 3 pw indices of its row in
// registers.  In both forms pw is a multiple of 8, so the
// 8 contraction indices a lane feeds one MFMA never straddle two planes.
// FP16 operands carry a per-fragment power-of-two scale that places each
// operand's largest value in [2^13, 2^14), keeping the low terms out of the
// subnormal range; the scales are undone exactly in FP64.
#include <algorithm>
#include <type_traits>

#include "fef_internal.h"
#include "fef_device.h"
#include "fef_epilogue.h"
#include "fef_split.h"

namespace fef {

// Per-fragment scales: hdr[2 f] = 1 / scale_left, hdr[2 f + 1] = 1 / scale_right.
template <bool kFp16>
__global__ __launch_bounds__(256) void split_scale_kernel(const FragInfo* __restrict__ frag,
                                                          const int32_t* __restrict__ list,
                                                          int P0, const double* __restrict__ bov,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ hdr) {
  __shared__ double red[4];
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  double mL = 0.0, mR = 0.0;
  const int64_t nL = (int64_t)P0 * fi.ov;
  for (int64_t e = threadIdx.x; e < nL; e += blockDim.x) {
    mL = fmax(mL, fabs(w[fi.off_w + e]));
    if (fi.cls == 0) mR = fmax(mR, fabs(bov[fi.off_bov + e]));
  }
  mL = block_max(mL, red);
  mR = block_max(mR, red);
  if (threadIdx.x == 0) {
    const double sL = kFp16 ? split_scale(mL) : 1.0;
    const double sR = kFp16 ? split_scale(mR) : 1.0;
    hdr[2 * f] = 1.0 / sL;
    hdr[2 * f + 1] = 1.0 / sR;
  }
}

// Writes both operands of a fragment, layout [ld][nterm pw + 8]: row m holds
// term plane 0 (k = 0..P0-1, zeros up to pw), plane 1, [plane 2,] then 8
// zeros; rows m >= ov are zero.
template <int PREC>
__global__ __launch_bounds__(256) void split_pack_kernel(const FragInfo* __restrict__ frag,
                                                         const int32_t* __restrict__ list,
                                                         int P0, int pw,
                                                         const double* __restrict__ bov,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ hdr,
                                                         char* __restrict__ ops) {
  constexpr int NTERM = split_nterm(PREC);
  const int f = list[blockIdx.x];
  const FragInfo fi = frag[f];
  const int tile = blockIdx.y;
  if (tile >= fi.ntile) return;
  const double sL = 1.0 / hdr[2 * f];
  const double sR = 1.0 / hdr[2 * f + 1];
  uint16_t* L = reinterpret_cast<uint16_t*>(ops + fi.off_L[PREC]);
  uint16_t* R = fi.off_R[PREC] >= 0 ? reinterpret_cast<uint16_t*>(ops + fi.off_R[PREC]) : nullptr;
  const int nchunk = pw / 8;
  const int row = NTERM * pw + 8;
  const u16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int m = tile * kTile + threadIdx.x; m < (tile + 1) * kTile; m += blockDim.x) {
    *reinterpret_cast<u16x8*>(L + (int64_t)m * row + NTERM * pw) = z;
    if (R) *reinterpret_cast<u16x8*>(R + (int64_t)m * row + NTERM * pw) = z;
  }
  for (int e = threadIdx.x; e < kTile * nchunk; e += blockDim.x) {
    const int m = tile * kTile + e / nchunk;
    const int k0 = (e % nchunk) * 8;
    u16x8 lt[NTERM], rt[NTERM];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u;
      uint16_t a[NTERM] = {}, c[NTERM] = {};
      if (m < fi.ov && k < P0) {
        split_terms<PREC, NTERM>(w[fi.off_w + (int64_t)k * fi.ov + m] * sL, a);
        if (R) split_terms<PREC, NTERM>(bov[fi.off_bov + (int64_t)k * fi.ov + m] * sR, c);
      }
#pragma unroll
      for (int t = 0; t < NTERM; ++t) {
        lt[t][u] = a[t];
        rt[t][u] = c[t];
      }
    }
#pragma unroll
    for (int t = 0; t < NTERM; ++t) {
      *reinterpret_cast<u16x8*>(L + (int64_t)m * row + t * pw + k0) = lt[t];
      if (R) *reinterpret_cast<u16x8*>(R + (int64_t)m * row + t * pw + k0) = rt[t];
    }
  }
}

hipError_t launch_pack_split(const fef_plan_s& p, const double* bov, const double* w, void* ops,
                             fef_prec prec, hipStream_t st) {
  char* o = static_cast<char*>(ops);
  double* hdr = reinterpret_cast<double*>(o);
  const int pw = p.geom[prec].pw;
  int maxtile = 0;
  for (int32_t f : p.ht_generic) maxtile = std::max(maxtile, p.frag[f].ntile);
  if (maxtile == 0) return hipSuccess;
  const unsigned ng = (unsigned)p.ht_generic.size();
  if (prec == FEF_FP16X2) {
    hipLaunchKernelGGL(split_scale_kernel<true>, dim3(ng), dim3(256), 0, st, p.d_frag,
                       p.d_ht_generic, p.P0, bov, w, hdr);
    hipLaunchKernelGGL(split_pack_kernel<FEF_FP16X2>, dim3(ng, maxtile), dim3(256), 0, st,
                       p.d_frag, p.d_ht_generic, p.P0, pw, bov, w, hdr, o);
  } else if (prec == FEF_BF16X2 || prec == FEF_BF16X3) {
    hipLaunchKernelGGL(split_scale_kernel<false>, dim3(ng), dim3(256), 0, st, p.d_frag,
                       p.d_ht_generic, p.P0, bov, w, hdr);
    if (prec == FEF_BF16X2)
      hipLaunchKernelGGL(split_pack_kernel<FEF_BF16X2>, dim3(ng, maxtile), dim3(256), 0, st,
                         p.d_frag, p.d_ht_generic, p.P0, pw, bov, w, hdr, o);
    else
      hipLaunchKernelGGL(split_pack_kernel<FEF_BF16X3>, dim3(ng, maxtile), dim3(256), 0, st,
                         p.d_frag, p.d_ht_generic, p.P0, pw, bov, w, hdr, o);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Waits until at most n (0..15, uniform across the wave) of this wave's
// vector memory operations are outstanding; the other counters are not
// waited for.  gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8.
__device__ inline void wait_vm_upto(int n) {
#define FEF_VM(N) case N: __builtin_amdgcn_s_waitcnt((N) | (7 << 4) | (15 << 8)); break;
  switch (n) {
    FEF_VM(0) FEF_VM(1) FEF_VM(2) FEF_VM(3) FEF_VM(4) FEF_VM(5) FEF_VM(6) FEF_VM(7)
    FEF_VM(8) FEF_VM(9) FEF_VM(10) FEF_VM(11) FEF_VM(12) FEF_VM(13) FEF_VM(14) FEF_VM(15)
    default: __builtin_amdgcn_s_waitcnt(0);
  }
#undef FEF_VM
}

template <bool kFp16>
__device__ inline f4 mma16(u16x8 a, u16x8 b, f4 c) {
  if (kFp16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// The two-term contraction as one chain for a lane with k-group lk: chunk
// m covers kk = 32 m + 8 lk; segment s = kk / pw of the concatenated axis
// pairs x plane (0, 0, 1)[s] with y plane (0, 1, 0)[s] at offset kk - s pw
// within the plane, and kk >= 3 pw reads the row's zero tail.
template <bool kFp16, int NC>
struct SplitChain2 {
  static constexpr int kNterm = 2;
  static constexpr int NX = NC;
  int xoff[NC], yoff[NC];
  __device__ __forceinline__ SplitChain2(int pw, int lk) {
    const int tail = 2 * pw;
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      const int kk = 32 * m + 8 * lk;
      const int sg = kk / pw, in = kk - sg * pw;
      xoff[m] = kk < 3 * pw ? (sg == 2 ? pw : 0) + in : tail;
      yoff[m] = kk < 3 * pw ? (sg == 1 ? pw : 0) + in : tail;
    }
  }
  template <int TI>
  __device__ __forceinline__ void load_x(u16x8 (&xa)[TI][NX], const uint16_t* L, int xs) const {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int c = 0; c < NX; ++c) xa[i][c] = *reinterpret_cast<const u16x8*>(L + 16 * i * xs + xoff[c]);
  }
  template <int TI, int TJ>
  __device__ __forceinline__ void contract(f4 (&acc)[TI][TJ], const u16x8 (&xa)[TI][NX],
                                           const uint16_t* Yb, int xs) const {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      u16x8 b[TJ];
#pragma unroll
      for (int j = 0; j < TJ; ++j) b[j] = *reinterpret_cast<const u16x8*>(Yb + 16 * j * xs + yoff[c]);
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = mma16<kFp16>(xa[i][c], b[j], acc[i][j]);
    }
  }
};

// The chains of one split contraction for a lane with k-group lk: x chunk m
// reads the stored row at kk = 32 m + 8 lk (the planes concatenated); the
// chain of order L pairs it with y plane L - i, i = kk / pw, at the same
// offset within the plane, while kk < (L + 1) pw, and with the row's zero
// tail beyond.  N0, N1, N2: the chunks of orders 0, 1, 2 (N2 = 0 for two
// terms); NX = the chunks of the highest order, which cover every x chunk.
template <bool kFp16, int NTERM, int N0, int N1, int N2>
struct SplitChains {
  static constexpr int kNterm = NTERM;
  static constexpr int NX = NTERM == 3 ? N2 : N1;
  int xoff[NX], y0[N0], y1[N1], y2[N2 > 0 ? N2 : 1];
  __device__ __forceinline__ SplitChains(int pw, int lk) {
    const int tail = NTERM * pw;
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      const int kk = 32 * m + 8 * lk;
      xoff[m] = kk < tail ? kk : tail;
      const int i = kk / pw, in = kk - (kk / pw) * pw;
      if (m < N0) y0[m] = kk < pw ? kk : tail;
      if (m < N1) y1[m] = kk < 2 * pw ? (1 - i) * pw + in : tail;
      if (N2 > 0 && m < N2) y2[m] = kk < 3 * pw ? (2 - i) * pw + in : tail;
    }
  }
  // x rows r (at L + 16 i xs) of TI tiles, every chunk
  template <int TI>
  __device__ __forceinline__ void load_x(u16x8 (&xa)[TI][NX], const uint16_t* L, int xs) const {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int c = 0; c < NX; ++c) xa[i][c] = *reinterpret_cast<const u16x8*>(L + 16 * i * xs + xoff[c]);
  }
  template <int TI, int TJ, int NC>
  __device__ __forceinline__ static void chain(f4 (&acc)[TI][TJ], const u16x8 (&xa)[TI][NX],
                                               const uint16_t* Yb, int xs, const int (&yo)[NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      u16x8 b[TJ];
#pragma unroll
      for (int j = 0; j < TJ; ++j) b[j] = *reinterpret_cast<const u16x8*>(Yb + 16 * j * xs + yo[c]);
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = mma16<kFp16>(xa[i][c], b[j], acc[i][j]);
    }
  }
  // acc += the whole contraction against the y rows at Yb + 16 j xs, highest
  // order first
  template <int TI, int TJ>
  __device__ __forceinline__ void contract(f4 (&acc)[TI][TJ], const u16x8 (&xa)[TI][NX],
                                           const uint16_t* Yb, int xs) const {
    if constexpr (N2 > 0) chain<TI, TJ, N2>(acc, xa, Yb, xs, y2);
    chain<TI, TJ, N1>(acc, xa, Yb, xs, y1);
    chain<TI, TJ, N0>(acc, xa, Yb, xs, y0);
  }
};

// row stride bound (16-bit words) of a stored row, pw <= 80
template <int NTERM>
constexpr int split_row_max() { return NTERM * 80 + 8; }

// Persistent split-precision pair kernel.  Work items as in the plain
// kernel.  A workgroup serves XB x units with two waves each (128 XB
// threads; XB = 2 runs two workgroups per CU, whose barriers are
// independent, so one workgroup's FP32 epilogue overlaps the other's MFMA
// chains on the same SIMD).  Every wave owns 48 x rows x 96 y columns: its
// MFMA A fragments (rows of W^x, all contraction chunks) stay in registers
// for the whole item; the streamed y tiles (rows of B^y), their gaps and
// the y operand's scale are copied from global memory straight into a ring
// of NBUF LDS buffers (global_load_lds, 16 bytes per lane) while an earlier
// buffer is contracted: the copy of entry e + NBUF - 1 is issued at the
// start of entry e into the buffer entry e - 1 left, and at the end of
// entry e only entry e + 1's copy is waited for.  Buffer indices are
// compile-time constants (the entry loop is unrolled over the ring), so the
// compiler sees that reads of the current buffer never wait for a copy into
// another.  Nothing in the entry loop is loaded through the vector memory
// path except the copies, so no wait on a loaded value drains the copies
// in flight.  MFMA operand lane layout (16x16x32): row (or column) =
// lane % 16, contraction indices 8 (lane / 16) .. +7.
template <bool kFp16, int XB, class Ch>
__global__ __launch_bounds__(128 * XB, XB == 2 ? 2 : 1) void pair_split_kernel(
    const FragInfo* __restrict__ frag, const PairInfo* __restrict__ pairs,
    const int32_t* __restrict__ slot_pair, const XBlock* __restrict__ xblocks,
    const Entry* __restrict__ entries, const WorkItem* __restrict__ items, int32_t nitems,
    int32_t* __restrict__ head, const int32_t* __restrict__ grp_off, const char* __restrict__ ops,
    int prec, int pw, const double* __restrict__ gap, double* __restrict__ partial) {
  constexpr int NT = 128 * XB, NW = 2 * XB;
  constexpr int TI = 3, TJ = 6, TJP = 3;
  constexpr int NTERM = Ch::kNterm;
  constexpr int NX = Ch::NX;
  // ring depth: two buffers for two workgroups per CU, else as many as fit
  constexpr int NBUF = XB == 2 ? 2 : (NTERM == 3 ? 3 : 4);
  constexpr int GL = kTile + 2;  // gaps, then the y operand's two scales
  __shared__ __align__(16) uint16_t Ys[NBUF][kTile * split_row_max<NTERM>()];
  __shared__ __align__(16) double Gy[NBUF][GL];
  __shared__ float Gx[XB * kTile];
  __shared__ double red[2][NW];
  __shared__ int32_t s_item;
  // the wave index is uniform across a wave: readfirstlane lets the
  // per-entry metadata come through scalar loads
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int unit = wave >> 1, sub = wave & 1;
  const int r0 = sub * 48;
  const double* hdr = reinterpret_cast<const double*>(ops);
  const int xs = NTERM * pw + 8;       // row stride (16-bit elements) in HBM and LDS
  const int tile_ch = kTile * xs / 8;  // 16-byte chunks per tile
  const u16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
  const Ch ch(pw, lk);
  // global_load_lds operations one copy puts in flight in this wave
  int nload = wave == NW - 1 ? 1 : 0;
  for (int g = wave; g * 64 < tile_ch; g += NW) ++nload;
  // copy of entry E's y tile, gaps and scales into the LDS buffer (Y, G):
  // wave w moves the 1 KB pieces w, w + NW, ...; lanes 0-47 of the last wave
  // move the gaps and its lane 48 the scale pair hdr[2 y], hdr[2 y + 1]
  auto issue = [&](int E, uint16_t* Y, double* G) {
    const char* src = ops + entries[E].off_R;
    for (int g = wave; g * 64 < tile_ch; g += NW) {
      const int c = g * 64 + lane;
      if (c < tile_ch)
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(src + 16 * (int64_t)c),
                                         (lds_void_t*)(Y + g * 512), 16, 0, 0);
    }
    if (wave == NW - 1 && lane <= kTile / 2) {
      const double* gsrc = lane < kTile / 2 ? gap + entries[E].off_gap + 2 * lane
                                            : hdr + 2 * entries[E].y;
      __builtin_amdgcn_global_load_lds(static_cast<const void*>(gsrc), (lds_void_t*)(G), 16, 0, 0);
    }
  };
  for (;;) {
    if (threadIdx.x == 0) s_item = pull_item(head, grp_off, blockIdx.x & 7);
    __syncthreads();
    const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it < 0 || it >= nitems) break;
    const int32_t xbid = items[it].xblock, e0 = items[it].e0, ne = items[it].ne;
    if (ne == 0) continue;  // an item emptied by a pair mask
#pragma unroll
    for (int b = 0; b + 1 < NBUF; ++b)
      if (b < ne) issue(e0 + b, Ys[b], Gy[b]);
    const int fxi = xblocks[xbid].f[unit];
    const int mt = xblocks[xbid].mt[unit];
    const double sx = fxi >= 0 ? hdr[2 * fxi] : 0.0;
    u16x8 xa[TI][NX];
    if (fxi >= 0) {
      ch.template load_x<TI>(xa, reinterpret_cast<const uint16_t*>(ops + frag[fxi].off_L[prec]) +
                            (int64_t)(mt * kTile + r0 + li) * xs, xs);
    } else {
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int c = 0; c < NX; ++c) xa[i][c] = zero;
    }
    for (int t = threadIdx.x; t < XB * kTile; t += NT) {
      const int u = t / kTile, m = t - (t / kTile) * kTile;
      const int f = xblocks[xbid].f[u];
      Gx[t] = f >= 0 ? (float)gap[frag[f].off_gap + xblocks[xbid].mt[u] * kTile + m] : -1.0f;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // entry el (local index) on ring buffer B; issues entry el + NBUF - 1's
    // copy into the buffer entry el - 1 left
    auto entry = [&](auto Bc, int el) {
      constexpr int B = decltype(Bc)::value, BN = (B + NBUF - 1) % NBUF;
      const int e = e0 + el;
      const int slot = entries[e].slot[unit];
      if (el + NBUF - 1 < ne) issue(e + NBUF - 1, Ys[BN], Gy[BN]);
      const double* Gc = Gy[B];
      const double sy = Gc[kTile + 1];
      double mine = 0.0;
      if (slot >= 0) {
        const uint16_t* Yb = Ys[B] + li * xs;
        // the wave's TJ column tiles in passes of TJP, so that TI x TJP
        // independent accumulators stay live over the whole contraction
        double part = 0.0;
#pragma unroll
        for (int jh = 0; jh < TJ / TJP; ++jh) {
          f4 acc[TI][TJP];
#pragma unroll
          for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJP; ++j) acc[i][j] = f4{0, 0, 0, 0};
          ch.template contract<TI, TJP>(acc, xa, Yb + 16 * jh * TJP * xs, xs);
          part += weighted_tiles_f32<TI, TJP>(acc, Gx + unit * kTile + r0, Gc + 16 * jh * TJP,
                                             lane);
        }
        mine = wave_sum_dpp(part);
      }
      if (lane == 0) red[el & 1][wave] = mine;
      // entry el + 1's copy has landed (this wave's part; after the
      // barrier, every wave's part); later copies may stay in flight
      const int later = min(NBUF - 2, ne - el - 2);
      if (later > 0)
        wait_vm_upto(later * nload);
      else
        __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (sub == 0 && lane == 0 && slot >= 0) {
        const double s = entries[e].s[unit];
        const double sc = sx * sy;
        partial[slot] = 4.0 * s * s * sc * sc * (red[el & 1][wave] + red[el & 1][wave + 1]);
      }
    };
    for (int el = 0; el < ne; el += NBUF) {
      entry(std::integral_constant<int, 0>{}, el);
      if (el + 1 < ne) entry(std::integral_constant<int, 1 % NBUF>{}, el + 1);
      if (NBUF > 2 && el + 2 < ne) entry(std::integral_constant<int, 2 % NBUF>{}, el + 2);
      if (NBUF > 3 && el + 3 < ne) entry(std::integral_constant<int, 3 % NBUF>{}, el + 3);
    }
  }
}


// Pipelined two-term split kernel for the common plane width (pw fixed at
// compile time): two x units per workgroup, two waves each, two workgroups
// per CU, as the two-unit kernel.  Each wave splits the 96 y columns of an
// entry into two halves of 48 and issues the MFMA chain of one half while
// it weights the accumulators of the half before on the VALU, so that the
// matrix core and the VALU of one wave work side by side:
//   stage A(e): contract half 0 of entry e   | weight half 1 of entry e - 1
//   stage B(e): contract half 1 of entry e   | weight half 0 of entry e
// A stage runs chunk by chunk (the chunk's three B fragments and nine
// MFMAs, then one or two of the nine tiles to weight), each chunk fenced
// from the next so that the scheduler keeps the interleave and only one
// chunk's temporaries are live.  One workgroup barrier per entry (after
// stage B), y tiles in two LDS buffers with the next entry's copy issued at
// the start of an entry; a wave whose unit has no pair with an entry skips
// that entry's chains and weighting.  The sums are those of the two-unit
// kernel in the same order (tiles (i, j) of a half in FP32, the two halves
// in FP64, the unit's two waves), and the entry's partial slot is written
// after the next barrier.
template <bool kFp16, int NC, int PW>
__global__ __launch_bounds__(256, 2) void pair_split_pipe_kernel(
    const FragInfo* __restrict__ frag, const XBlock* __restrict__ xblocks,
    const Entry* __restrict__ entries, const WorkItem* __restrict__ items, int32_t nitems,
    int32_t* __restrict__ head, const int32_t* __restrict__ grp_off, const char* __restrict__ ops,
    int prec, const double* __restrict__ gap, double* __restrict__ partial) {
  constexpr int XB = 2, NT = 256, NW = 4;
  constexpr int TI = 3, TJ = 3;
  constexpr int XS = 2 * PW + 8;             // row stride (16-bit elements)
  constexpr int TILE_CH = kTile * XS / 8;     // 16-byte chunks per tile
  constexpr int GL = kTile + 2;               // gaps, then the y operand's scales
  __shared__ __align__(16) uint16_t Ys0[kTile * XS];
  __shared__ __align__(16) uint16_t Ys1[kTile * XS];
  __shared__ __align__(16) double Gy0[GL];
  __shared__ __align__(16) double Gy1[GL];
  __shared__ float Gx[XB * kTile];
  __shared__ double red[2][NW];
  __shared__ int32_t s_item;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int unit = wave >> 1, sub = wave & 1;
  const int r0 = sub * 48;
  const double* hdr = reinterpret_cast<const double*>(ops);
  const u16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
  const SplitChain2<kFp16, NC> ch(PW, lk);
  auto issue = [&](int E, uint16_t* Y, double* G) __attribute__((always_inline)) {
    const char* src = ops + entries[E].off_R;
    for (int g = wave; g * 64 < TILE_CH; g += NW) {
      const int c = g * 64 + lane;
      if (c < TILE_CH)
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(src + 16 * (int64_t)c),
                                         (lds_void_t*)(Y + g * 512), 16, 0, 0);
    }
    if (wave == NW - 1 && lane <= kTile / 2) {
      const double* gsrc = lane < kTile / 2 ? gap + entries[E].off_gap + 2 * lane
                                            : hdr + 2 * entries[E].y;
      __builtin_amdgcn_global_load_lds(static_cast<const void*>(gsrc), (lds_void_t*)(G), 16, 0, 0);
    }
  };
  using yes = std::true_type;
  using no = std::false_type;
  for (;;) {
    if (threadIdx.x == 0) s_item = pull_item(head, grp_off, blockIdx.x & 7);
    __syncthreads();
    const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it < 0 || it >= nitems) break;
    const int32_t xbid = items[it].xblock, e0 = items[it].e0, ne = items[it].ne;
    if (ne == 0) continue;  // an item emptied by a pair mask
    issue(e0, Ys0, Gy0);
    const int fxi = xblocks[xbid].f[unit];
    const int mt = xblocks[xbid].mt[unit];
    const double sx = fxi >= 0 ? hdr[2 * fxi] : 0.0;
    u16x8 xa[TI][NC];
    if (fxi >= 0) {
      ch.template load_x<TI>(xa, reinterpret_cast<const uint16_t*>(ops + frag[fxi].off_L[prec]) +
                            (int64_t)(mt * kTile + r0 + li) * XS, XS);
    } else {
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int c = 0; c < NC; ++c) xa[i][c] = zero;
    }
    for (int t = threadIdx.x; t < XB * kTile; t += NT) {
      const int u = t / kTile, m = t - (t / kTile) * kTile;
      const int f = xblocks[xbid].f[u];
      Gx[t] = f >= 0 ? (float)gap[frag[f].off_gap + xblocks[xbid].mt[u] * kTile + m] : -1.0f;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    float dx[TI][4];
    {
      const float* gx = Gx + unit * kTile + r0 + 4 * lk;
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) dx[i][r] = gx[16 * i + r];
    }
    f4 acc0[TI][TJ], acc1[TI][TJ];
    float dy0[TJ], dy1[TJ];
    // one stage on LDS buffer (Y, G): the chain of half h into acc (and its
    // column gaps into dy) if C, the weighting of accw with gaps dyw if Wt
    auto stage = [&](auto C, auto Wt, const uint16_t* Y, const double* G, int h,
                     f4(&acc)[TI][TJ], float(&dy)[TJ], const f4(&accw)[TI][TJ],
                     const float(&dyw)[TJ]) __attribute__((always_inline)) -> double {
      constexpr bool kC = decltype(C)::value, kW = decltype(Wt)::value;
      constexpr int NG = kC ? NC : 1;
      const uint16_t* Yb = Y + (48 * h + li) * XS;
      if constexpr (kC) {
#pragma unroll
        for (int j = 0; j < TJ; ++j) dy[j] = (float)G[48 * h + li + 16 * j];
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) acc[i][j] = f4{0, 0, 0, 0};
      }
      float w = 0.0f;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        if constexpr (kC) {
          u16x8 b[TJ];
#pragma unroll
          for (int j = 0; j < TJ; ++j)
            b[j] = *reinterpret_cast<const u16x8*>(Yb + 16 * j * XS + ch.yoff[g]);
#pragma unroll
          for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) acc[i][j] = mma16<kFp16>(xa[i][g], b[j], acc[i][j]);
        }
        if constexpr (kW) {
          // the nine tiles over NG groups, the first 9 % NG groups one more
          constexpr int q = 9 / NG, rm = 9 % NG;
          const int t0 = g * q + (g < rm ? g : rm), nt = q + (g < rm ? 1 : 0);
#pragma unroll
          for (int tt = 0; tt < q + (rm ? 1 : 0); ++tt)
            if (tt < nt) {
              const int t = t0 + tt, ti = t / TJ, tj = t - TJ * (t / TJ);
              w += weighted_tile_f32(accw[ti][tj], dx[ti], dyw[tj]);
            }
          // the group's weighting happens here, not sunk past later chunks
          if constexpr (kC) asm volatile("" : "+v"(w));
        }
        if constexpr (kC && kW) __builtin_amdgcn_sched_barrier(0);
      }
      return (double)w;
    };
    auto run = [&](bool c, bool w, const uint16_t* Y, const double* G, int h, f4(&acc)[TI][TJ],
                   float(&dy)[TJ], const f4(&accw)[TI][TJ], const float(&dyw)[TJ])
                   __attribute__((always_inline)) -> double {
      if (c && w) return stage(yes{}, yes{}, Y, G, h, acc, dy, accw, dyw);
      if (c) return stage(yes{}, no{}, Y, G, h, acc, dy, accw, dyw);
      if (w) return stage(no{}, yes{}, Y, G, h, acc, dy, accw, dyw);
      return 0.0;
    };
    // entry el on buffer (Y, G), the next entry's buffer (Yn, Gn)
    bool vprev = false;   // the previous entry had a pair for this wave's unit
    int slot_prev = -1;
    double sc_prev = 0.0, s_prev = 0.0;
    bool v0 = entries[e0].slot[unit] >= 0;
    (void)run(v0, false, Ys0, Gy0, 0, acc0, dy0, acc1, dy1);
    auto entry = [&](int el, const uint16_t* Y, const double* G, uint16_t* Yn, double* Gn)
                     __attribute__((always_inline)) {
      const int e = e0 + el;
      const int slot = entries[e].slot[unit];
      const bool v = slot >= 0;
      if (el + 1 < ne) issue(e + 1, Yn, Gn);
      const double sy = G[kTile + 1];
      // B(el): half 1 of el | weight half 0 of el
      double part = run(v, v, Y, G, 1, acc1, dy1, acc0, dy0);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      // entry el - 1's partial slot: its wave sums are in red[(el - 1) & 1]
      if (el >= 1 && sub == 0 && lane == 0 && slot_prev >= 0)
        partial[slot_prev] = 4.0 * s_prev * s_prev * sc_prev * sc_prev *
                             (red[(el - 1) & 1][wave] + red[(el - 1) & 1][wave + 1]);
      // A(el + 1): half 0 of el + 1 | weight half 1 of el
      const bool vn = el + 1 < ne && entries[e + 1].slot[unit] >= 0;
      part += run(vn, v, Yn, Gn, 0, acc0, dy0, acc1, dy1);
      const double mine = v ? wave_sum_dpp(part) : 0.0;
      if (lane == 0) red[el & 1][wave] = mine;
      slot_prev = slot;
      s_prev = v ? entries[e].s[unit] : 0.0;
      sc_prev = sx * sy;
    };
    for (int el = 0; el < ne; el += 2) {
      entry(el, Ys0, Gy0, Ys1, Gy1);
      if (el + 1 < ne) entry(el + 1, Ys1, Gy1, Ys0, Gy0);
    }
    __syncthreads();
    if (sub == 0 && lane == 0 && slot_prev >= 0)
      partial[slot_prev] = 4.0 * s_prev * s_prev * sc_prev * sc_prev *
                           (red[(ne - 1) & 1][wave] + red[(ne - 1) & 1][wave + 1]);
    (void)vprev;
  }
}


// Ping-pong split pair kernel: two x units per workgroup, eight waves, one
// workgroup per CU.  Waves w and w + 4 share a SIMD and hold the same 48 x
// rows of one unit (wave w: columns 0-47 of the streamed y tile, wave w + 4:
// columns 48-95), 3 x 3 MFMA tiles each.  The two groups of four waves run
// half a step apart: in every phase one group contracts an entry on MFMA
// while the other weights the previous entry's accumulators on the VALU, so
// on each SIMD the matrix chain of one wave overlaps the FP32 epilogue of
// the other by construction.  A phase ends at a workgroup barrier:
//   phase 2e    : group A contracts entry e,  group B weights entry e - 1
//   phase 2e + 1: group A weights entry e,    group B contracts entry e
// The y tiles rotate through three LDS buffers: the copy of entry e + 2 is
// issued at phase 2e into the buffer entry e - 1 left, and entry e + 1's
// copy (issued two phases earlier) is waited for at the end of phase 2e + 1
// while the newest copy stays in flight, so a copy has three phases to land.
// Each wave takes its column gaps into registers while it contracts, so an
// epilogue never reads a buffer being refilled.  Each wave leaves its weighted sum in LDS; once
// both groups have weighted entry e, one lane per unit adds the four wave
// sums in a fixed order into the entry's partial slot.
template <bool kFp16, class Ch>
__global__ __launch_bounds__(512, 1) void pair_split_pp_kernel(
    const FragInfo* __restrict__ frag, const XBlock* __restrict__ xblocks,
    const Entry* __restrict__ entries, const WorkItem* __restrict__ items, int32_t nitems,
    int32_t* __restrict__ head, const int32_t* __restrict__ grp_off, const char* __restrict__ ops,
    int prec, int pw, const double* __restrict__ gap, double* __restrict__ partial) {
  constexpr int XB = 2, NW = 8, NT = 512, NBUF = 3;
  constexpr int NTERM = Ch::kNterm;
  constexpr int NX = Ch::NX;
  __shared__ __align__(16) uint16_t Ys[NBUF][kTile * split_row_max<NTERM>()];
  __shared__ __align__(16) double Gy[NBUF][kTile + 2];  // gaps, then the y scales
  __shared__ double ysc[2];  // y scale of the entries being finished
  __shared__ float Gx[XB * kTile];
  __shared__ double red[2][NW];
  __shared__ int32_t s_item;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int grp = wave >> 2, unit = (wave >> 1) & 1;
  const int r0 = 48 * (wave & 1), c0 = 48 * grp;
  const double* hdr = reinterpret_cast<const double*>(ops);
  const int xs = NTERM * pw + 8;
  const int tile_ch = kTile * xs / 8;
  const u16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
  const Ch ch(pw, lk);
  // global_load_lds operations one copy puts in flight in this wave
  int nload = wave == NW - 1 ? 1 : 0;
  for (int g = wave; g * 64 < tile_ch; g += NW) ++nload;
  auto issue = [&](int E, uint16_t* Y, double* G) {
    const char* src = ops + entries[E].off_R;
    for (int g = wave; g * 64 < tile_ch; g += NW) {
      const int c = g * 64 + lane;
      if (c < tile_ch)
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(src + 16 * (int64_t)c),
                                         (lds_void_t*)(Y + g * 512), 16, 0, 0);
    }
    if (wave == NW - 1 && lane <= kTile / 2) {
      const double* gsrc = lane < kTile / 2 ? gap + entries[E].off_gap + 2 * lane
                                            : hdr + 2 * entries[E].y;
      __builtin_amdgcn_global_load_lds(static_cast<const void*>(gsrc), (lds_void_t*)(G), 16, 0, 0);
    }
  };
  for (;;) {
    if (threadIdx.x == 0) s_item = pull_item(head, grp_off, blockIdx.x & 7);
    __syncthreads();
    const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it < 0 || it >= nitems) break;
    const int32_t xbid = items[it].xblock, e0 = items[it].e0, ne = items[it].ne;
    if (ne == 0) continue;  // an item emptied by a pair mask
    issue(e0, Ys[0], Gy[0]);
    if (ne > 1) issue(e0 + 1, Ys[1], Gy[1]);
    const int fxi = xblocks[xbid].f[unit];
    const int mt = xblocks[xbid].mt[unit];
    u16x8 xa[3][NX];
    if (fxi >= 0) {
      ch.template load_x<3>(xa, reinterpret_cast<const uint16_t*>(ops + frag[fxi].off_L[prec]) +
                           (int64_t)(mt * kTile + r0 + li) * xs, xs);
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < NX; ++c) xa[i][c] = zero;
    }
    for (int t = threadIdx.x; t < XB * kTile; t += NT) {
      const int u = t / kTile, m = t - (t / kTile) * kTile;
      const int f = xblocks[xbid].f[u];
      Gx[t] = f >= 0 ? (float)gap[frag[f].off_gap + xblocks[xbid].mt[u] * kTile + m] : -1.0f;
    }
    // x scale of thread u's unit (u < XB finishes unit u's slots)
    const int fu = threadIdx.x < XB ? xblocks[xbid].f[threadIdx.x] : -1;
    const double sxu = fu >= 0 ? hdr[2 * fu] : 0.0;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // partial slot of entry E for unit u, from the four wave sums of
    // the unit in a fixed order; the scales come from registers and LDS, so
    // no vector load waits on the copies in flight
    auto finish = [&](int el, int u) {
      const int E = e0 + el;
      // both units' metadata through uniform (scalar) loads
      const int sl0 = entries[E].slot[0], sl1 = entries[E].slot[1];
      const double s0 = entries[E].s[0], s1 = entries[E].s[1];
      const int slot = u == 0 ? sl0 : sl1;
      if (slot < 0) return;
      const double s = u == 0 ? s0 : s1;
      const double sc = sxu * ysc[el & 1];
      const double* r = red[el & 1];
      partial[slot] = 4.0 * s * s * sc * sc *
                      ((r[2 * u] + r[2 * u + 1]) + (r[4 + 2 * u] + r[4 + 2 * u + 1]));
    };
    f4 acc[3][3];
    float dy[3];
    for (int t = 0; t <= 2 * ne; ++t) {
      if (t >= 3 && (t & 1) && threadIdx.x < XB) finish((t - 3) >> 1, threadIdx.x);
      const int en = (t >> 1) + 2;  // the copy issued at this even phase
      if (!(t & 1) && en < ne) issue(e0 + en, Ys[en % NBUF], Gy[en % NBUF]);
      if ((grp == 0) == !(t & 1)) {
        // contraction phase
        const int el = grp == 0 ? (t >> 1) : ((t - 1) >> 1);
        if (wave == 0 && lane == 0 && el < ne) ysc[el & 1] = Gy[el % NBUF][kTile + 1];
        if (el < ne && entries[e0 + el].slot[unit] >= 0) {
          const uint16_t* Yb = Ys[el % NBUF] + (c0 + li) * xs;
          const double* Gc = Gy[el % NBUF] + c0 + li;
#pragma unroll
          for (int j = 0; j < 3; ++j) dy[j] = (float)Gc[16 * j];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) acc[i][j] = f4{0, 0, 0, 0};
          ch.template contract<3, 3>(acc, xa, Yb, xs);
        }
      } else {
        // weighting phase
        const int el = grp == 0 ? ((t - 1) >> 1) : ((t >> 1) - 1);
        if (el >= 0) {
          double mine = 0.0;
          if (entries[e0 + el].slot[unit] >= 0) {
            float dx[3][4];
            const float* gx = Gx + unit * kTile + r0 + 4 * lk;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int r = 0; r < 4; ++r) dx[i][r] = gx[16 * i + r];
            mine = wave_sum_dpp(weighted_tiles_f32_regs<3, 3>(acc, dx, dy));
          }
          if (lane == 0) red[el & 1][wave] = mine;
        }
      }
      // at the end of an odd phase 2e + 1 the copy of entry e + 1 has landed
      // (this wave's part; after the barrier, every wave's part); the copy of
      // entry e + 2, issued last, may stay in flight
      if (t & 1) {
        if ((t >> 1) + 2 < ne)
          wait_vm_upto(nload);
        else
          __builtin_amdgcn_s_waitcnt(0);
      }
      __syncthreads();
    }
    if (threadIdx.x < XB) finish(ne - 1, threadIdx.x);
  }
}

// Persistent grid: xb = 4 runs the four-unit kernel, one workgroup per CU;
// xb = 2 runs, for two terms, the two-unit kernel with two workgroups per CU
// (their barriers independent), for three terms (whose x fragments leave no
// room for two workgroups) the ping-pong kernel, one workgroup per CU.
template <bool F16, class Ch>
static void launch_split_kernel(const fef_plan_s& p, int xb, int ncu, hipStream_t st,
                                const char* o, int prec, int pw, const double* gap,
                                const Entry* entries, const WorkItem* items, double* partial,
                                int32_t* head) {
  const TileSet& t = p.tiles[prec];
  const bool two_wg = xb == 2 && Ch::kNterm == 2;
  const int64_t want = (int64_t)ncu * (two_wg ? 2 : 1);
  const dim3 grid((unsigned)std::min<int64_t>(want, std::max<int64_t>(t.nitems, 1)));
  if (xb == 4) {
    hipLaunchKernelGGL((pair_split_kernel<F16, 4, Ch>), grid, dim3(512), 0, st, p.d_frag,
                       p.d_pair, p.d_slot_pair, t.d_xblocks, entries, items, (int32_t)t.nitems,
                       head, t.d_grp_off, o, prec, pw, gap, partial);
  } else if constexpr (Ch::kNterm == 2) {
    if constexpr (Ch::NX == 7) {
      if (pw == 72) {
        hipLaunchKernelGGL((pair_split_pipe_kernel<F16, 7, 72>), grid, dim3(256), 0, st,
                           p.d_frag, t.d_xblocks, entries, items, (int32_t)t.nitems, head,
                           t.d_grp_off, o, prec, gap, partial);
        return;
      }
    }
    hipLaunchKernelGGL((pair_split_kernel<F16, 2, Ch>), grid, dim3(256), 0, st, p.d_frag,
                       p.d_pair, p.d_slot_pair, t.d_xblocks, entries, items, (int32_t)t.nitems,
                       head, t.d_grp_off, o, prec, pw, gap, partial);
  } else {
    hipLaunchKernelGGL((pair_split_pp_kernel<F16, Ch>), grid, dim3(512), 0, st, p.d_frag,
                       t.d_xblocks, entries, items, (int32_t)t.nitems, head, t.d_grp_off, o,
                       prec, pw, gap, partial);
  }
}

// Kernel instance for the chain lengths of (nterm, pw).
template <bool F16, int NTERM>
static bool launch_split_terms(const fef_plan_s& p, int xb, int pw, int ncu, hipStream_t st,
                               const char* o, int prec, const double* gap, const Entry* entries,
                               const WorkItem* items, double* partial, int32_t* head) {
  if constexpr (NTERM == 2) {
    const int nc = (3 * pw + 31) / 32;
#define FEF_CHAIN(NC)                                                                          \
  if (nc == NC) {                                                                              \
    launch_split_kernel<F16, SplitChain2<F16, NC>>(p, xb, ncu, st, o, prec, pw, gap, entries,  \
                                                   items, partial, head);                      \
    return true;                                                                               \
  }
    FEF_CHAIN(1) FEF_CHAIN(2) FEF_CHAIN(3) FEF_CHAIN(4) FEF_CHAIN(5) FEF_CHAIN(6) FEF_CHAIN(7)
    FEF_CHAIN(8)
#undef FEF_CHAIN
  } else {
    const int n0 = split_chain(0, pw), n1 = split_chain(1, pw), n2 = split_chain(2, pw);
#define FEF_CHAINS(A, B, C)                                                                    \
  if (n0 == A && n1 == B && n2 == C) {                                                         \
    launch_split_kernel<F16, SplitChains<F16, 3, A, B, C>>(p, xb, ncu, st, o, prec, pw, gap,   \
                                                           entries, items, partial, head);     \
    return true;                                                                               \
  }
    FEF_CHAINS(1, 1, 1) FEF_CHAINS(1, 1, 2) FEF_CHAINS(1, 2, 3) FEF_CHAINS(2, 3, 4)
    FEF_CHAINS(2, 3, 5) FEF_CHAINS(2, 4, 6) FEF_CHAINS(3, 5, 7) FEF_CHAINS(3, 5, 8)
#undef FEF_CHAINS
  }
  return false;
}

hipError_t launch_split_pairs(const fef_plan_s& p, const void* ops, const double* gap,
                              fef_prec prec, const Entry* entries, const WorkItem* items,
                              double* partial, int32_t* head, int ncu, hipStream_t st) {
  const char* o = static_cast<const char*>(ops);
  const int pw = p.geom[prec].pw;
  const int xb = p.tiles[prec].xb;
  if (pw > 80 || pw < 8 || pw % 8 != 0) return hipErrorInvalidValue;
  if ((p.ops_header & 15) != 0) return hipErrorInvalidValue;  // 16-byte copies
  bool ok = false;
  if (prec == FEF_FP16X2)
    ok = launch_split_terms<true, 2>(p, xb, pw, ncu, st, o, (int)prec, gap, entries, items,
                                     partial, head);
  else if (prec == FEF_BF16X2)
    ok = launch_split_terms<false, 2>(p, xb, pw, ncu, st, o, (int)prec, gap, entries, items,
                                      partial, head);
  else if (prec == FEF_BF16X3)
    ok = launch_split_terms<false, 3>(p, xb, pw, ncu, st, o, (int)prec, gap, entries, items,
                                      partial, head);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace fef
