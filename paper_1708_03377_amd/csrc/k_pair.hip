// Pair contraction on MFMA and the denominator-weighted squared sum.
//
// For a pair (x, y) (y in class 0):
//   V[ia][jb] = s_xy sum_Q W^x[Q][ia] B_ov^y[Q][jb]        ( = (ia|jb) )
//   E2_xy     = 4 sum_{ia,jb} V^2 / (Delta^x_ia + Delta^y_jb),
//   Delta_ia  = eps_i - eps_a
// (dimer second-order energy with first-order dimer doubles, canonical
// orbitals).  V is produced tile by tile in MFMA accumulators and reduced in
// registers; it is never written to memory.
#include <algorithm>

#include "fef_internal.h"
#include "fef_device.h"
#include "fef_epilogue.h"

namespace fef {

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4 acc_t;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef f4 acc_t;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Persistent FP64 / FP32 pair kernel.  A workgroup pulls work items from the
// queue groups (LPT order inside each).  An item is XB x units (fragment x,
// row tile mt) and a run of y tiles.  Four waves serve a unit, each a 48x48
// quadrant of V (3x3 MFMA tiles); a wave keeps its x rows (the MFMA A
// operand of every k step) in registers for the whole item.  Each y tile
// ([kpad][96], k-major) and its gaps are copied from global memory straight
// into one of two LDS buffers (global_load_lds, 16 bytes per lane) while the
// other buffer is contracted; the buffers are separate LDS arrays, so reads
// of the current one never wait for the copy into the next.  With two units
// a workgroup has eight waves, two per SIMD.
constexpr int kPadMax = 80;
typedef __attribute__((address_space(3))) void plain_lds_t;

template <typename T, int KS, int XB>
__global__ __launch_bounds__(256 * XB) void pair_plain_kernel(
    const FragInfo* __restrict__ frag, const PairInfo* __restrict__ pairs,
    const int32_t* __restrict__ slot_pair, const XBlock* __restrict__ xblocks,
    const Entry* __restrict__ entries, const WorkItem* __restrict__ items, int32_t nitems,
    int32_t* __restrict__ head, const int32_t* __restrict__ grp_off, const char* __restrict__ ops, int prec, int kpad,
    const double* __restrict__ gap, double* __restrict__ partial) {
  typedef typename Mfma<T>::acc_t acc_t;
  static_assert(4 * KS <= kPadMax, "k steps");
  constexpr int NT = 256 * XB, NW = 4 * XB;
  constexpr int kRowCh = kTile * (int)sizeof(T) / 16;  // 16-byte chunks per k row of a tile
  __shared__ __align__(16) T YsA[kPadMax * kTile];
  __shared__ __align__(16) T YsB[kPadMax * kTile];
  __shared__ __align__(16) double GyA[kTile];
  __shared__ __align__(16) double GyB[kTile];
  __shared__ double Gx[XB * kTile];
  __shared__ double red[2][NW];
  __shared__ int32_t s_item;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int unit = wave >> 2, sub = wave & 3;
  const int r0 = (sub >> 1) * 48, c0 = (sub & 1) * 48;
  const int tile_ch = kpad * kRowCh;
  // The MFMA loop reads k rows up to 4 KS - 1 of both buffers, the copies
  // fill rows below kpad only: rows kpad .. 4 KS - 1 are zeroed once here
  // (the barrier after the first queue pull orders this before any read),
  // so a stale non-finite value can never meet the zero x operand there.
  for (int e = kpad * kTile + (int)threadIdx.x; e < 4 * KS * kTile; e += NT) {
    YsA[e] = (T)0;
    YsB[e] = (T)0;
  }
  // copy of entry E's y tile ([kpad][96] of a [kpad][ld_y] operand) and gaps
  auto issue = [&](int E, T* Y, double* G) {
    const int64_t yld = entries[E].ld_y;
    const char* src = ops + entries[E].off_R;
    for (int g = wave; g * 64 < tile_ch; g += NW) {
      const int c = g * 64 + lane;
      if (c < tile_ch) {
        const int k = c / kRowCh, q = c - (c / kRowCh) * kRowCh;
        __builtin_amdgcn_global_load_lds(
            static_cast<const void*>(src + ((int64_t)k * yld * sizeof(T) + 16 * q)),
            (plain_lds_t*)(Y + g * 64 * (16 / (int)sizeof(T))), 16, 0, 0);
      }
    }
    if (wave == NW - 1 && lane < kTile / 2)
      __builtin_amdgcn_global_load_lds(static_cast<const void*>(gap + entries[E].off_gap + 2 * lane),
                                       (plain_lds_t*)(G), 16, 0, 0);
  };
  for (;;) {
    if (threadIdx.x == 0) s_item = pull_item(head, grp_off, blockIdx.x & 7);
    __syncthreads();
    const int32_t it = s_item;
    __syncthreads();
    if (it < 0 || it >= nitems) break;
    const int32_t xbid = items[it].xblock, e0 = items[it].e0, ne = items[it].ne;
    if (ne == 0) continue;  // an item emptied by a pair mask
    issue(e0, YsA, GyA);
    const int fxi = xblocks[xbid].f[unit];
    const int mt = xblocks[xbid].mt[unit];
    // x rows r0 + 16 i + li at k = 4 s + lk, all k steps
    T xa[3][KS];
    if (fxi >= 0) {
      const int64_t xld = frag[fxi].ld;
      const T* L = reinterpret_cast<const T*>(ops + frag[fxi].off_L[prec]) + mt * kTile + r0 + li;
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i)
          xa[i][s] = 4 * s + lk < kpad ? L[(int64_t)(4 * s + lk) * xld + 16 * i] : (T)0;
    } else {
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int i = 0; i < 3; ++i) xa[i][s] = (T)0;
    }
    for (int t = threadIdx.x; t < XB * kTile; t += NT) {
      const int u = t / kTile, m = t - (t / kTile) * kTile;
      const int f = xblocks[xbid].f[u];
      Gx[t] = f >= 0 ? gap[frag[f].off_gap + xblocks[xbid].mt[u] * kTile + m] : -1.0;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int end = e0 + ne;
    auto entry = [&](int e, int cur, const T* Yc, const double* Gc, T* Yn, double* Gn) {
      const int slot = entries[e].slot[unit];
      const double s = entries[e].s[unit];
      if (e + 1 < end) issue(e + 1, Yn, Gn);
      double mine = 0.0;
      if (slot >= 0) {
        acc_t acc[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
        const T* yr = Yc + lk * kTile + c0 + li;
#pragma unroll
        for (int st = 0; st < KS; ++st) {
          T b[3];
#pragma unroll
          for (int j = 0; j < 3; ++j) b[j] = yr[4 * st * kTile + 16 * j];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) acc[i][j] = Mfma<T>::mma(xa[i][st], b[j], acc[i][j]);
        }
        mine = wave_sum_dpp(weighted_tiles<sizeof(T) == 8, 3, 3>(acc, Gx + unit * kTile + r0,
                                                              Gc + c0, lane, 1.0));
      }
      if (lane == 0) red[cur][wave] = mine;
      // this wave's part of the next copy has landed; after the barrier,
      // every wave's part has
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (sub == 0 && lane == 0 && slot >= 0)
        partial[slot] = 4.0 * s * s *
                        ((red[cur][wave] + red[cur][wave + 1]) +
                         (red[cur][wave + 2] + red[cur][wave + 3]));
    };
    for (int e = e0; e < end; e += 2) {
      entry(e, 0, YsA, GyA, YsB, GyB);
      if (e + 1 < end) entry(e + 1, 1, YsB, GyB, YsA, GyA);
    }
  }
}

__global__ void reset_head_kernel(int32_t* head) {
  for (int g = 0; g < kQueues; ++g) head[g] = 0;
}

// Pair mask: copies every work item's entries, in order, into the same
// positions of a second table, keeping only the units whose pair is selected
// and dropping entries left with none; the item keeps its x-block and start
// and gets the new length (possibly 0).
__global__ void mask_items_kernel(const WorkItem* __restrict__ items, int32_t nitems,
                                  const Entry* __restrict__ entries,
                                  const int32_t* __restrict__ slot_pair,
                                  const int32_t* __restrict__ select,
                                  Entry* __restrict__ out_entries,
                                  WorkItem* __restrict__ out_items) {
  const int32_t it = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (it >= nitems) return;
  const WorkItem w = items[it];
  int32_t k = 0;
  for (int32_t e = w.e0; e < w.e0 + w.ne; ++e) {
    Entry en = entries[e];
    bool any = false;
#pragma unroll
    for (int u = 0; u < kMaxXB; ++u) {
      if (en.slot[u] >= 0 && !select[slot_pair[en.slot[u]]]) en.slot[u] = -1;
      any |= en.slot[u] >= 0;
    }
    if (any) out_entries[w.e0 + k++] = en;
  }
  out_items[it] = WorkItem{w.xblock, w.e0, k, 0};
}

// Delta_ia = eps_i - eps_a for every fragment, -1 on the padding up to ld;
// raises the gap flag for a non-negative Delta.
__global__ __launch_bounds__(256) void gaps_kernel(const FragInfo* __restrict__ frag,
                                                   const double* __restrict__ eps,
                                                   double* __restrict__ gap,
                                                   int32_t* __restrict__ flags) {
  const FragInfo fi = frag[blockIdx.x];
  const double* e = eps + fi.off_eps;
  bool bad = false;
  for (int m = threadIdx.x; m < fi.ld; m += blockDim.x) {
    double g = -1.0;
    if (m < fi.ov) {
      const int i = m / fi.nvir, a = m - (m / fi.nvir) * fi.nvir;
      g = e[i] - e[fi.nocc + a];
      bad |= !(g < 0.0);
    }
    gap[fi.off_gap + m] = g;
  }
  if (bad) atomicOr(flags, FEF_FLAG_GAP);
}

// E2_pair[p] = sum of the pair's tile partials, in slot order; with a mask,
// only the selected pairs are written.
__global__ void pair_reduce_kernel(const PairInfo* __restrict__ pairs, int64_t npair,
                                   const double* __restrict__ partial,
                                   const int32_t* __restrict__ select,
                                   double* __restrict__ E2_pair, int32_t* __restrict__ flags) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npair) return;
  if (select && !select[p]) return;
  const PairInfo pr = pairs[p];
  double s = 0.0;
  for (int k = 0; k < pr.ntx * pr.nty; ++k) s += partial[pr.slot_first + k];
  E2_pair[p] = s;
  if (!isfinite(s)) atomicOr(flags, FEF_FLAG_NONFINITE);
}

// E2_total in two fixed-order stages: block b sums the strided elements
// b + 256 k (k = 0, 1, ...) of each thread's lane in order, reduces its
// block in lane/wave order; one block then adds the 256 block sums.
constexpr int kTotalBlocks = 256;
__global__ __launch_bounds__(256) void total_stage1_kernel(const double* __restrict__ E2_pair,
                                                           int64_t npair,
                                                           double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < npair;
       k += (int64_t)kTotalBlocks * 256)
    s += E2_pair[k];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}
__global__ __launch_bounds__(256) void total_stage2_kernel(const double* __restrict__ part,
                                                           double* __restrict__ out) {
  __shared__ double red[4];
  const double t = block_sum(part[threadIdx.x], red);
  if (threadIdx.x == 0) *out = t;
}

hipError_t launch_split_pairs(const fef_plan_s& p, const void* ops, const double* gap,
                              fef_prec prec, const Entry* entries, const WorkItem* items,
                              double* partial, int32_t* head, int grid, hipStream_t st);

int compute_units() {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      ncu = n;
    else
      ncu = 256;
  }
  return ncu;
}

static int persistent_grid(int64_t nitems, int per_cu) {
  const int64_t g = (int64_t)compute_units() * per_cu;
  return (int)(nitems < g ? nitems : g);
}

hipError_t launch_pair_energies(const fef_plan_s& p, const void* ops, const double* eps,
                                fef_prec prec, const int32_t* select, double* E2_pair,
                                double* E2_total, int32_t* flags, void* ws, hipStream_t st) {
  double* partial = static_cast<double*>(ws);
  char* wsb = static_cast<char*>(ws) + round_up(std::max<int64_t>(p.nslot, 1) * (int64_t)sizeof(double), 256);
  int32_t* head = reinterpret_cast<int32_t*>(wsb);
  double* gap = reinterpret_cast<double*>(wsb + 256);
  const char* o = static_cast<const char*>(ops);
  const TileSet& t = p.tiles[prec];
  const Entry* entries = t.d_entries;
  const WorkItem* items = t.d_items;
  if (select && t.nitems > 0) {
    char* mb = static_cast<char*>(ws) + pair_ws_bytes(p, prec);
    Entry* me = reinterpret_cast<Entry*>(mb);
    WorkItem* mi = reinterpret_cast<WorkItem*>(
        mb + round_up(std::max<int64_t>(t.nentries, 1) * (int64_t)sizeof(Entry), 256));
    hipLaunchKernelGGL(mask_items_kernel, dim3((unsigned)((t.nitems + 255) / 256)), dim3(256), 0,
                       st, t.d_items, (int32_t)t.nitems, t.d_entries, p.d_slot_pair, select, me,
                       mi);
    entries = me;
    items = mi;
  }
  if (t.nitems > 0) {
    hipLaunchKernelGGL(reset_head_kernel, dim3(1), dim3(1), 0, st, head);
    hipLaunchKernelGGL(gaps_kernel, dim3(p.nfrag), dim3(256), 0, st, p.d_frag, eps, gap, flags);
    const int kpad = p.geom[prec].kpad;
    switch (prec) {
      case FEF_F64:
      case FEF_F32: {
        const bool f64 = prec == FEF_F64;
        const int xbp = t.xb == 2 ? 2 : 1;
        const dim3 grid(persistent_grid(t.nitems, f64 || xbp == 2 ? 1 : 2));
#define FEF_PLAIN(T, KS, XB)                                                                    \
  hipLaunchKernelGGL((pair_plain_kernel<T, KS, XB>), grid, dim3(256 * XB), 0, st, p.d_frag,    \
                     p.d_pair, p.d_slot_pair, t.d_xblocks, entries, items, (int32_t)t.nitems,   \
                     head, t.d_grp_off, o, (int)prec, kpad, gap, partial)
#define FEF_PLAIN_K(T, XB)                                                                      \
  if (kpad == 72) FEF_PLAIN(T, 18, XB); else if (kpad == 8) FEF_PLAIN(T, 2, XB);                \
  else FEF_PLAIN(T, kPadMax / 4, XB)
        if (f64) {
          if (xbp == 2) { FEF_PLAIN_K(double, 2); } else { FEF_PLAIN_K(double, 1); }
        } else {
          if (xbp == 2) { FEF_PLAIN_K(float, 2); } else { FEF_PLAIN_K(float, 1); }
        }
#undef FEF_PLAIN_K
#undef FEF_PLAIN
        break;
      }
      default: {
        hipError_t e = launch_split_pairs(p, ops, gap, prec, entries, items, partial, head,
                                          compute_units(), st);
        if (e != hipSuccess) return e;
      }
    }
  }
  if (p.npair > 0)
    hipLaunchKernelGGL(pair_reduce_kernel, dim3((unsigned)((p.npair + 255) / 256)), dim3(256), 0,
                       st, p.d_pair, p.npair, partial, select, E2_pair, flags);
  double* tpart = gap + round_up(std::max<int64_t>(p.nGap, 1), 32);
  hipLaunchKernelGGL(total_stage1_kernel, dim3(kTotalBlocks), dim3(256), 0, st, E2_pair, p.npair,
                     tpart);
  hipLaunchKernelGGL(total_stage2_kernel, dim3(1), dim3(256), 0, st, tpart, E2_total);
  return hipGetLastError();
}

}  // namespace fef
