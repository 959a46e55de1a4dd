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

// Persistent FP64 / FP32 pair kernel.  A workgroup pulls work items from a
// global queue (LPT order).  An item is one x unit (fragment x, row tile mt)
// and a run of y tiles: the x tile (kpad x 96, k-major) sits in LDS for the
// whole item; each y tile is staged in LDS too, the next one being fetched
// into registers while the current one is contracted by four waves, each a
// 48x48 quadrant of V (3x3 MFMA tiles).  Orbital-energy gaps of both sides
// are staged with their tiles.
template <typename T, int KS>
__global__ __launch_bounds__(256) void pair_plain_kernel(
    const FragInfo* __restrict__ frag, const PairInfo* __restrict__ pairs,
    const int32_t* __restrict__ slot_pair, const XBlock* __restrict__ xblocks,
    const Entry* __restrict__ entries, const WorkItem* __restrict__ items, int32_t nitems,
    int32_t* __restrict__ head, const int32_t* __restrict__ grp_off, const char* __restrict__ ops, int prec, int kpad,
    const double* __restrict__ gap, double* __restrict__ partial) {
  typedef typename Mfma<T>::acc_t acc_t;
  typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
  constexpr int kVec = 16 / sizeof(T);        // elements per 16-byte chunk
  constexpr int kRowCh = kTile / kVec;        // chunks per k-row of a tile
  constexpr int NPF = (80 * kRowCh + 255) / 256;  // staging chunks per thread (kpad <= 80)
  extern __shared__ char smem[];
  T* Xs = reinterpret_cast<T*>(smem);          // [kpad][kTile]
  T* Ys = Xs + kpad * kTile;                   // [kpad][kTile]
  __shared__ double Gx[kTile], Gy[kTile];
  __shared__ double red[4];
  __shared__ int32_t s_item;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = (wave >> 1) * 48, c0 = (wave & 1) * 48;
  const int tot = kpad * kRowCh;
  for (;;) {
    if (threadIdx.x == 0) s_item = pull_item(head, grp_off, blockIdx.x & 7);
    __syncthreads();
    const int32_t it = s_item;
    __syncthreads();
    if (it < 0 || it >= nitems) break;
    const int32_t xbid = items[it].xblock, e0 = items[it].e0, ne = items[it].ne;
    if (ne == 0) continue;  // an item emptied by a pair mask
    const int fxi = xblocks[xbid].f[0];
    const int mt = xblocks[xbid].mt[0];
    {
      const int64_t xld = frag[fxi].ld;
      const T* L = reinterpret_cast<const T*>(ops + frag[fxi].off_L[prec]) + mt * kTile;
      for (int c = threadIdx.x; c < tot; c += 256) {
        const int k = c / kRowCh, q = c - (c / kRowCh) * kRowCh;
        *reinterpret_cast<i32x4*>(Xs + k * kTile + q * kVec) =
            *reinterpret_cast<const i32x4*>(L + (int64_t)k * xld + q * kVec);
      }
      if (threadIdx.x < kTile) Gx[threadIdx.x] = gap[frag[fxi].off_gap + mt * kTile + threadIdx.x];
    }
    i32x4 pf[NPF];
    double pg = 0.0;
    auto issue = [&](int e) {
      const int64_t yld = entries[e].ld_y;
      const T* R = reinterpret_cast<const T*>(ops + entries[e].off_R);
#pragma unroll
      for (int k = 0; k < NPF; ++k) {
        const int c = threadIdx.x + 256 * k;
        if (c < tot) {
          const int kk = c / kRowCh, q = c - (c / kRowCh) * kRowCh;
          pf[k] = *reinterpret_cast<const i32x4*>(R + (int64_t)kk * yld + q * kVec);
        }
      }
      if (threadIdx.x < kTile) pg = gap[entries[e].off_gap + threadIdx.x];
    };
    issue(e0);
    for (int e = e0; e < e0 + ne; ++e) {
      __syncthreads();  // x tile stored / previous y tile consumed
#pragma unroll
      for (int k = 0; k < NPF; ++k) {
        const int c = threadIdx.x + 256 * k;
        if (c < tot) *reinterpret_cast<i32x4*>(Ys + c * kVec) = pf[k];
      }
      if (threadIdx.x < kTile) Gy[threadIdx.x] = pg;
      __syncthreads();
      if (e + 1 < e0 + ne) issue(e + 1);
      const int slot = entries[e].slot[0];
      acc_t acc[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
      // KS > 0: the contraction loop is fully unrolled so the accumulators
      // stay in the MFMA registers across steps
#define FEF_KSTEP(K0)                                                              \
  {                                                                                \
    const T* xr = Xs + ((K0) + lk) * kTile + r0 + li;                              \
    const T* yr = Ys + ((K0) + lk) * kTile + c0 + li;                              \
    T a[3], b[3];                                                                  \
    _Pragma("unroll") for (int i = 0; i < 3; ++i) a[i] = xr[16 * i];                \
    _Pragma("unroll") for (int j = 0; j < 3; ++j) b[j] = yr[16 * j];                \
    _Pragma("unroll") for (int i = 0; i < 3; ++i)                                   \
      _Pragma("unroll") for (int j = 0; j < 3; ++j)                                 \
        acc[i][j] = Mfma<T>::mma(a[i], b[j], acc[i][j]);                            \
  }
      if constexpr (KS > 0) {
#pragma unroll
        for (int st = 0; st < KS; ++st) FEF_KSTEP(4 * st)
      } else {
        for (int k = 0; k < kpad; k += 4) FEF_KSTEP(k)
      }
#undef FEF_KSTEP
      const double sum = weighted_tiles<sizeof(T) == 8, 3, 3>(acc, Gx + r0, Gy + c0, lane, 1.0);
      const double total = block_sum(sum, red);
      if (threadIdx.x == 0) {
        const double s = entries[e].s[0];
        partial[slot] = 4.0 * s * s * total;
      }
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

void configure_plain_kernels(int kpad64, int kpad32) {
  const int need64 = 2 * kpad64 * kTile * (int)sizeof(double);
  const int need32 = 2 * kpad32 * kTile * (int)sizeof(float);
  if (need64 > 65536) {
    (void)hipFuncSetAttribute((const void*)pair_plain_kernel<double, 18>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, need64);
    (void)hipFuncSetAttribute((const void*)pair_plain_kernel<double, 0>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, need64);
  }
  if (need32 > 65536)
    (void)hipFuncSetAttribute((const void*)pair_plain_kernel<float, 0>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, need32);
  (void)hipGetLastError();
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
        const dim3 grid(persistent_grid(t.nitems, f64 ? 1 : 2));
        const size_t lds = 2 * (size_t)kpad * kTile * (f64 ? sizeof(double) : sizeof(float));
#define FEF_PLAIN(T, KS)                                                                        \
  hipLaunchKernelGGL((pair_plain_kernel<T, KS>), grid, dim3(256), lds, st, p.d_frag, p.d_pair,  \
                     p.d_slot_pair, t.d_xblocks, entries, items, (int32_t)t.nitems,             \
                     head, t.d_grp_off, o, (int)prec, kpad, gap, partial)
        if (f64) {
          if (kpad == 72) FEF_PLAIN(double, 18); else if (kpad == 8) FEF_PLAIN(double, 2);
          else FEF_PLAIN(double, 0);
        } else {
          if (kpad == 72) FEF_PLAIN(float, 18); else if (kpad == 8) FEF_PLAIN(float, 2);
          else FEF_PLAIN(float, 0);
        }
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
