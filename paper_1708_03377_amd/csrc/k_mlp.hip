// Distant-pair surrogate (a project addition; the paper has no learned
// component): rotation-invariant scalars of each fragment's Coulomb moments
// d^x = B^x : D^x (the moments of the effective field, Eqs. wc / dp2e), pair
// features, an ensemble of 17-128-128-1 SiLU networks that predicts
// E2_xy R_xy^2 (Eq. ED2 with its leading 1/R^2 removed), its training
// (forward, backward, Adam) and the selection of the pairs that the exact
// pair kernel must evaluate.
//
// Parameters of one member are packed as W0[128][17], b0[128], W1[128][128],
// b1[128], W2[128], b2 (FEF_MLP_NPARAM numbers, member stride
// FEF_MLP_STRIDE).  Inference runs the two wide layers on MFMA with BF16
// weights and activations and FP32 accumulation; training runs in FP32 on
// the BF16-rounded weights and keeps FP32 master weights for Adam.
#include "fef_internal.h"
#include "fef_device.h"
#include "fef_split.h"

namespace fef {

constexpr int kNin = FEF_MLP_NIN;
constexpr int kNh = FEF_MLP_NHID;
constexpr int kMStride = FEF_MLP_STRIDE;
constexpr int oW0 = 0;
constexpr int oB0 = oW0 + kNh * kNin;
constexpr int oW1 = oB0 + kNh;
constexpr int oB1 = oW1 + kNh * kNh;
constexpr int oW2 = oB1 + kNh;
constexpr int oB2 = oW2 + kNh;
static_assert(oB2 + 1 == FEF_MLP_NPARAM, "parameter packing");
static_assert(kMStride % 8 == 0 && kMStride >= FEF_MLP_NPARAM, "member stride");
static_assert(oW1 % 8 == 0, "W1 rows must be 16-byte aligned in BF16");

__device__ inline float bf16f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ inline float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ inline float silu_grad_f(float z) {
  const float sg = 1.0f / (1.0f + expf(-z));
  return sg * (1.0f + z * (1.0f - sg));
}

// ---------------------------------------------------------------------------
// Coupling modes: the eigenvectors of G_00 with the four largest eigenvalues,
// taken from the ascending eigensolver output (columns of V), largest first.
__global__ void top_modes_kernel(const double* __restrict__ V, int n, double* __restrict__ Q) {
  for (int t = threadIdx.x; t < 4 * n; t += blockDim.x) {
    const int k = t / n, p = t - (t / n) * n;
    Q[t] = k < n ? V[(int64_t)p * n + (n - 1 - k)] : 0.0;
  }
}

// u^x = [d.G^k.d (k = 0..3), (q_k.d)^2 (k = 0..3)] for class-0 fragments;
// NaN for the others (their pairs always go to the exact kernel).
__global__ __launch_bounds__(128) void invariants_kernel(const FragInfo* __restrict__ frag,
                                                         const double* __restrict__ dmom,
                                                         const double* __restrict__ G,
                                                         const double* __restrict__ Q, int P0,
                                                         double* __restrict__ U) {
  __shared__ double v[2][80];
  __shared__ double red[2];
  const int x = blockIdx.x;
  const int p = threadIdx.x;
  if (frag[x].cls != 0) {
    if (p < 8) U[(int64_t)x * 8 + p] = __builtin_nan("");
    return;
  }
  const double* d = dmom + frag[x].off_aux;
  const double dp = p < P0 ? d[p] : 0.0;
  if (p < P0) v[0][p] = dp;
  __syncthreads();
  double u[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int cur = k & 1;
    const double vp = p < P0 ? v[cur][p] : 0.0;
    u[k] = block_sum(dp * vp, red);
    if (k < 3) {
      if (p < P0) {
        double acc = 0.0;
        for (int q = 0; q < P0; ++q) acc = fma(G[(int64_t)p * P0 + q], v[cur][q], acc);
        v[cur ^ 1][p] = acc;
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double pr = block_sum(p < P0 ? Q[k * P0 + p] * dp : 0.0, red);
    u[4 + k] = pr * pr;
  }
  if (p == 0)
#pragma unroll
    for (int k = 0; k < 8; ++k) U[(int64_t)x * 8 + k] = u[k];
}

// X[q] = [R, u^x + u^y, u^x * u^y] (R in bohr) for pair idx[q] (or q), and
// optionally the training target T[q] = E2_pair * R^2.
__global__ void features_kernel(const PairInfo* __restrict__ pairs,
                                const int32_t* __restrict__ idx, int64_t n,
                                const double* __restrict__ U, const double* __restrict__ E2,
                                float* __restrict__ X, float* __restrict__ T) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int64_t k = idx ? idx[q] : q;
  const PairInfo pr = pairs[k];
  const double R = 1.0 / pr.s;
  float* xr = X + q * kNin;
  xr[0] = (float)R;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double a = U[(int64_t)pr.x * 8 + j], b = U[(int64_t)pr.y * 8 + j];
    xr[1 + j] = (float)(a + b);
    xr[9 + j] = (float)(a * b);
  }
  if (T) T[q] = (float)(E2[k] * R * R);
}

// Column mean and standard deviation, or its inverse (two passes, FP64,
// fixed order); a zero deviation reads as 1.
__global__ __launch_bounds__(256) void column_stats_kernel(const float* __restrict__ A, int64_t n,
                                                           int ncol, int inverse,
                                                           float* __restrict__ mean,
                                                           float* __restrict__ sdev) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) s += (double)A[r * ncol + c];
  const double m = n > 0 ? block_sum(s, red) / (double)n : 0.0;
  double s2 = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    const double dv = (double)A[r * ncol + c] - m;
    s2 += dv * dv;
  }
  const double var = n > 0 ? block_sum(s2, red) / (double)n : 0.0;
  if (threadIdx.x == 0) {
    mean[c] = (float)m;
    const double sd = var > 0.0 ? sqrt(var) : 1.0;
    sdev[c] = (float)(inverse ? 1.0 / sd : sd);
  }
}

__global__ void mlp_pack_kernel(const float* __restrict__ P, int64_t n, uint16_t* __restrict__ W) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) W[i] = bf16_rne(P[i]);
}

// ---------------------------------------------------------------------------
// Ensemble inference on MFMA (16x16x32 BF16, FP32 accumulation).
//
// A block of 4 waves takes chunks of 256 rows (each wave 4 row tiles of 16)
// and, member by member, stages that member's BF16 weights in LDS: W0 as
// [128][40] (k >= 17 zero), W1 as [128][136].  Per row tile: layer 0 gives a
// 16x128 tile, SiLU in FP32, rounded to BF16 into the wave's H tile; layer 1
// reads H as the A operand; the output layer is a FP32 dot product reduced
// over the 16 lanes that share a row.  Rows are either given features
// (X [n][17]) or pairs of the plan, whose features are formed on the fly.
// Outputs: per-member standardised predictions Y [nmember][n] (optional) and
// for pairs the ensemble mean as an energy, and the exact-fallback flag.
constexpr int kInfRows = 256;
constexpr int kW0Ld = 40, kW1Ld = 136, kHLd = 136;
constexpr size_t kInferLds = (size_t)kNh * kW0Ld * 2 + (size_t)kNh * kW1Ld * 2 +
                             (size_t)4 * 16 * kHLd * 2 + (3 * kNh + 4) * sizeof(float) +
                             3 * kInfRows * sizeof(float) + 40 * sizeof(float);

__device__ inline f4 mma_bf16(const u16x8& a, const u16x8& b, const f4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

template <bool kPairs>
__global__ __launch_bounds__(256) void mlp_infer_kernel(
    int64_t n, int nmember, const float* __restrict__ X, const PairInfo* __restrict__ pairs,
    const double* __restrict__ U, const float* __restrict__ stats,
    const uint16_t* __restrict__ W, float* __restrict__ Y, double r_exact, double thr,
    double* __restrict__ E2_pair, int32_t* __restrict__ select) {
  extern __shared__ __align__(16) char smem[];
  uint16_t* W0s = reinterpret_cast<uint16_t*>(smem);
  uint16_t* W1s = W0s + kNh * kW0Ld;
  uint16_t* Hs = W1s + kNh * kW1Ld;
  float* b0s = reinterpret_cast<float*>(Hs + 4 * 16 * kHLd);
  float* b1s = b0s + kNh;
  float* w2s = b1s + kNh;
  float* b2s = w2s + kNh;  // [4]
  float* ysum = b2s + 4;
  float* ymin = ysum + kInfRows;
  float* ymax = ymin + kInfRows;
  float* st = ymax + kInfRows;  // [36]: mean[17], inv[17], tmean, tstd
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  if (tid < 36) st[tid] = stats[tid];
  __syncthreads();
  uint16_t* H = Hs + wave * 16 * kHLd;
  for (int64_t base = (int64_t)blockIdx.x * kInfRows; base < n;
       base += (int64_t)gridDim.x * kInfRows) {
    // layer-0 A operands: row li of each of this wave's row tiles, features
    // 8 lk .. 8 lk + 7 (standardised, zero beyond 17)
    u16x8 a0[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int64_t row = base + wave * 64 + rt * 16 + li;
      float f[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) f[j] = 0.0f;
      if (row < n) {
        if (kPairs) {
          const PairInfo pr = pairs[row];
          const double R = 1.0 / pr.s;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int k = 8 * lk + j;
            float v = 0.0f;
            if (k == 0) {
              v = (float)R;
            } else if (k < 9) {
              v = (float)(U[(int64_t)pr.x * 8 + k - 1] + U[(int64_t)pr.y * 8 + k - 1]);
            } else if (k < 17) {
              v = (float)(U[(int64_t)pr.x * 8 + k - 9] * U[(int64_t)pr.y * 8 + k - 9]);
            }
            f[j] = k < 17 ? (v - st[k]) * st[17 + k] : 0.0f;
          }
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int k = 8 * lk + j;
            f[j] = k < 17 ? (X[row * kNin + k] - st[k]) * st[17 + k] : 0.0f;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) a0[rt][j] = bf16_rne(f[j]);
    }
    for (int m = 0; m < nmember; ++m) {
      __syncthreads();  // the previous member's weights are no longer read
      const uint16_t* Wm = W + (int64_t)m * kMStride;
      for (int t = tid; t < kNh * kW0Ld; t += 256) {
        const int r = t / kW0Ld, k = t - (t / kW0Ld) * kW0Ld;
        W0s[t] = k < kNin ? Wm[oW0 + r * kNin + k] : (uint16_t)0;
      }
      for (int t = tid; t < kNh * kNh / 8; t += 256) {
        const int r = t / (kNh / 8), c8 = t - (t / (kNh / 8)) * (kNh / 8);
        *reinterpret_cast<u16x8*>(W1s + r * kW1Ld + 8 * c8) =
            *reinterpret_cast<const u16x8*>(Wm + oW1 + r * kNh + 8 * c8);
      }
      if (tid < kNh) {
        b0s[tid] = bf16f(Wm[oB0 + tid]);
        b1s[tid] = bf16f(Wm[oB1 + tid]);
        w2s[tid] = bf16f(Wm[oW2 + tid]);
      }
      if (tid == 0) b2s[0] = bf16f(Wm[oB2]);
      __syncthreads();
#pragma unroll 1
      for (int rt = 0; rt < 4; ++rt) {
        f4 acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const u16x8 b = *reinterpret_cast<const u16x8*>(W0s + (16 * j + li) * kW0Ld + 8 * lk);
          acc[j] = mma_bf16(a0[rt], b, f4{0, 0, 0, 0});
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int col = 16 * j + li;
            H[(4 * lk + r) * kHLd + col] = bf16_rne(silu_f(acc[j][r] + b0s[col]));
          }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = f4{0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < kNh / 32; ++c) {
          const u16x8 a = *reinterpret_cast<const u16x8*>(H + li * kHLd + 32 * c + 8 * lk);
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const u16x8 b =
                *reinterpret_cast<const u16x8*>(W1s + (16 * j + li) * kW1Ld + 32 * c + 8 * lk);
            acc[j] = mma_bf16(a, b, acc[j]);
          }
        }
        float pr[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int col = 16 * j + li;
          const float w = w2s[col], bb = b1s[col];
#pragma unroll
          for (int r = 0; r < 4; ++r) pr[r] = fmaf(w, silu_f(acc[j][r] + bb), pr[r]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int off = 8; off > 0; off >>= 1) pr[r] += __shfl_xor(pr[r], off, 16);
        if (li == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rc = wave * 64 + rt * 16 + 4 * lk + r;
            const float y = pr[r] + b2s[0];
            if (Y && base + rc < n) Y[(int64_t)m * n + base + rc] = y;
            if (m == 0) {
              ysum[rc] = y; ymin[rc] = y; ymax[rc] = y;
            } else {
              ysum[rc] += y; ymin[rc] = fminf(ymin[rc], y); ymax[rc] = fmaxf(ymax[rc], y);
            }
          }
        }
        __syncthreads();  // H is rewritten by the next row tile
      }
    }
    if (kPairs) {
      const int64_t q = base + tid;
      if (q < n) {
        const PairInfo pr = pairs[q];
        const double R = 1.0 / pr.s;
        const double r2 = R * R;
        // fragments outside class 0 carry NaN invariants: always exact
        const bool inval = !(U[(int64_t)pr.x * 8] == U[(int64_t)pr.x * 8]) ||
                           !(U[(int64_t)pr.y * 8] == U[(int64_t)pr.y * 8]);
        const double tmean = st[34], tstd = st[35];
        const double mean = (double)ysum[tid] / (double)nmember;
        const double e = (mean * tstd + tmean) / r2;
        const double spread = ((double)ymax[tid] - (double)ymin[tid]) * tstd / r2;
        const bool exact = inval || R < r_exact || !(spread <= thr) || !isfinite(e);
        select[q] = exact ? 1 : 0;
        E2_pair[q] = exact ? 0.0 : e;
      }
    }
    __syncthreads();  // ysum / ymin / ymax are rewritten by the next chunk
  }
}

// ---------------------------------------------------------------------------
// Training: one block of 128 threads (thread j = hidden unit j) takes 32 rows
// of member m's mini-batch, runs forward and backward in FP32 on the member's
// BF16 weights and writes its partial gradients (and partial squared error);
// a second kernel sums the block partials in block order and applies Adam to
// the FP32 master weights, refreshing the BF16 copy.
constexpr int kTrRows = 32;
constexpr size_t kTrainLds =
    ((size_t)kNh * (kNh + 1) + 4 * (size_t)kTrRows * kNh + (size_t)kTrRows * kNin + 2 * kTrRows +
     kNh + 40) * sizeof(float);

__global__ __launch_bounds__(128) void mlp_train_kernel(
    const float* __restrict__ X, const float* __restrict__ T, const int32_t* __restrict__ idx,
    int32_t nb, const float* __restrict__ stats, const uint16_t* __restrict__ W,
    float* __restrict__ gpart, float* __restrict__ lpart, int nblk) {
  extern __shared__ __align__(16) char smem[];
  float* W1f = reinterpret_cast<float*>(smem);   // [128][129]
  float* h0 = W1f + kNh * (kNh + 1);             // [R][128]
  float* z0 = h0 + kTrRows * kNh;
  float* z1 = z0 + kTrRows * kNh;
  float* gz = z1 + kTrRows * kNh;
  float* xs = gz + kTrRows * kNh;                // [R][17]
  float* gy = xs + kTrRows * kNin;               // [R]
  float* l2 = gy + kTrRows;                      // [R]
  float* w2s = l2 + kTrRows;                     // [128]
  float* st = w2s + kNh;                         // [36]
  const int m = blockIdx.y, b = blockIdx.x, j = threadIdx.x;
  const uint16_t* Wm = W + (int64_t)m * kMStride;
  if (j < 36) st[j] = stats[j];
  for (int e = j; e < kNh * kNh; e += kNh) W1f[(e >> 7) * (kNh + 1) + (e & (kNh - 1))] = bf16f(Wm[oW1 + e]);
  w2s[j] = bf16f(Wm[oW2 + j]);
  float w0[kNin];
#pragma unroll
  for (int i = 0; i < kNin; ++i) w0[i] = bf16f(Wm[oW0 + j * kNin + i]);
  const float b0 = bf16f(Wm[oB0 + j]), b1 = bf16f(Wm[oB1 + j]), w2 = bf16f(Wm[oW2 + j]);
  const float b2 = bf16f(Wm[oB2]);
  __syncthreads();
  for (int e = j; e < kTrRows * kNin; e += kNh) {
    const int r = e / kNin, i = e - (e / kNin) * kNin;
    const int g = b * kTrRows + r;
    float v = 0.0f;
    if (g < nb) {
      const int64_t s = idx[(int64_t)m * nb + g];
      v = (X[s * kNin + i] - st[i]) * st[17 + i];
    }
    xs[e] = v;
  }
  __syncthreads();
  for (int r = 0; r < kTrRows; ++r) {
    float z = b0;
#pragma unroll
    for (int i = 0; i < kNin; ++i) z = fmaf(w0[i], xs[r * kNin + i], z);
    z0[r * kNh + j] = z;
    h0[r * kNh + j] = silu_f(z);
  }
  __syncthreads();
  for (int r = 0; r < kTrRows; ++r) {
    float z = b1;
    for (int k = 0; k < kNh; ++k) z = fmaf(W1f[j * (kNh + 1) + k], h0[r * kNh + k], z);
    z1[r * kNh + j] = z;
  }
  __syncthreads();
  if (j < kTrRows) {
    const int g = b * kTrRows + j;
    float y = b2;
    for (int k = 0; k < kNh; ++k) y = fmaf(w2s[k], silu_f(z1[j * kNh + k]), y);
    float d = 0.0f;
    if (g < nb) {
      const int64_t s = idx[(int64_t)m * nb + g];
      d = y - (T[s] - st[34]) / st[35];
    }
    gy[j] = g < nb ? 2.0f * d / (float)nb : 0.0f;
    l2[j] = d * d;
  }
  __syncthreads();
  // backward, hidden unit j
  float gW2 = 0.0f, gb1 = 0.0f;
  float gzr[kTrRows];
#pragma unroll
  for (int r = 0; r < kTrRows; ++r) {
    const float z = z1[r * kNh + j];
    gW2 = fmaf(gy[r], silu_f(z), gW2);
    const float g = gy[r] * w2 * silu_grad_f(z);
    gzr[r] = g;
    gz[r * kNh + j] = g;
    gb1 += g;
  }
  float* gp = gpart + ((int64_t)m * nblk + b) * kMStride;
  for (int k = 0; k < kNh; ++k) {
    float acc = 0.0f;
#pragma unroll
    for (int r = 0; r < kTrRows; ++r) acc = fmaf(gzr[r], h0[r * kNh + k], acc);
    gp[oW1 + j * kNh + k] = acc;
  }
  __syncthreads();
  float g0[kTrRows];
  float gb0 = 0.0f;
#pragma unroll
  for (int r = 0; r < kTrRows; ++r) {
    float s = 0.0f;
    for (int jj = 0; jj < kNh; ++jj) s = fmaf(gz[r * kNh + jj], W1f[jj * (kNh + 1) + j], s);
    g0[r] = s * silu_grad_f(z0[r * kNh + j]);
    gb0 += g0[r];
  }
#pragma unroll
  for (int i = 0; i < kNin; ++i) {
    float acc = 0.0f;
#pragma unroll
    for (int r = 0; r < kTrRows; ++r) acc = fmaf(g0[r], xs[r * kNin + i], acc);
    gp[oW0 + j * kNin + i] = acc;
  }
  gp[oB0 + j] = gb0;
  gp[oB1 + j] = gb1;
  gp[oW2 + j] = gW2;
  if (j == 0) {
    float s = 0.0f, l = 0.0f;
    for (int r = 0; r < kTrRows; ++r) { s += gy[r]; l += l2[r]; }
    gp[oB2] = s;
    lpart[(int64_t)m * nblk + b] = l;
  }
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(
    int nblk, int32_t nb, const float* __restrict__ gpart, const float* __restrict__ lpart,
    float* __restrict__ P, float* __restrict__ M, float* __restrict__ V,
    uint16_t* __restrict__ W, int32_t step, float lr, float* __restrict__ grad_out,
    float* __restrict__ loss_out) {
  const int m = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  constexpr float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  if (p < FEF_MLP_NPARAM) {
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += gpart[((int64_t)m * nblk + b) * kMStride + p];
    const int64_t o = (int64_t)m * kMStride + p;
    if (grad_out) grad_out[o] = g;
    if (step > 0) {
      const float mm = beta1 * M[o] + (1.0f - beta1) * g;
      const float vv = beta2 * V[o] + (1.0f - beta2) * g * g;
      M[o] = mm;
      V[o] = vv;
      const float bc1 = (float)(1.0 - pow((double)beta1, (double)step));
      const float bc2 = (float)(1.0 - pow((double)beta2, (double)step));
      const float upd = (mm / bc1) / (sqrtf(vv / bc2) + eps);
      const float np = P[o] - lr * upd;
      P[o] = np;
      W[o] = bf16_rne(np);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss_out) {
    float l = 0.0f;
    for (int b = 0; b < nblk; ++b) l += lpart[(int64_t)m * nblk + b];
    loss_out[m] = nb > 0 ? l / (float)nb : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// launchers
hipError_t launch_invariants(const fef_plan_s& p, const double* dmom, const double* G,
                             const double* Q, double* U, hipStream_t st) {
  hipLaunchKernelGGL(invariants_kernel, dim3(p.nfrag), dim3(128), 0, st, p.d_frag, dmom, G, Q,
                     p.P0, U);
  return hipGetLastError();
}

hipError_t launch_top_modes(const double* V, int n, double* Q, hipStream_t st) {
  hipLaunchKernelGGL(top_modes_kernel, dim3(1), dim3(256), 0, st, V, n, Q);
  return hipGetLastError();
}

hipError_t launch_features(const fef_plan_s& p, const double* U, const double* E2,
                           const int32_t* idx, int64_t n, float* X, float* T, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     p.d_pair, idx, n, U, E2, X, T);
  return hipGetLastError();
}

hipError_t launch_column_stats(int64_t n, int ncol, int inverse, const float* A, float* mean,
                               float* sdev, hipStream_t st) {
  hipLaunchKernelGGL(column_stats_kernel, dim3(ncol), dim3(256), 0, st, A, n, ncol, inverse, mean,
                     sdev);
  return hipGetLastError();
}

hipError_t launch_mlp_pack(int nmember, const float* P, uint16_t* W, hipStream_t st) {
  const int64_t n = (int64_t)nmember * kMStride;
  hipLaunchKernelGGL(mlp_pack_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, n, W);
  return hipGetLastError();
}

static bool g_mlp_configured = false;
static void configure_mlp_kernels() {
  if (g_mlp_configured) return;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&mlp_infer_kernel<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kInferLds);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&mlp_infer_kernel<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kInferLds);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&mlp_train_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTrainLds);
  (void)hipGetLastError();
  g_mlp_configured = true;
}

static unsigned infer_grid(int64_t n) {
  const int64_t chunks = (n + kInfRows - 1) / kInfRows;
  const int64_t cap = (int64_t)compute_units() * 2;
  return (unsigned)(chunks < cap ? chunks : cap);
}

hipError_t launch_mlp_forward(int nmember, int64_t n, const float* X, const float* stats,
                              const uint16_t* W, float* Y, hipStream_t st) {
  if (n == 0) return hipSuccess;
  configure_mlp_kernels();
  hipLaunchKernelGGL(mlp_infer_kernel<false>, dim3(infer_grid(n)), dim3(256), kInferLds, st, n,
                     nmember, X, nullptr, nullptr, stats, W, Y, 0.0, 0.0, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_surrogate_select(const fef_plan_s& p, const double* U, int nmember,
                                   const float* stats, const uint16_t* W, double r_exact,
                                   double thr, double* E2_pair, int32_t* select, float* Y,
                                   hipStream_t st) {
  if (p.npair == 0) return hipSuccess;
  configure_mlp_kernels();
  hipLaunchKernelGGL(mlp_infer_kernel<true>, dim3(infer_grid(p.npair)), dim3(256), kInferLds, st,
                     p.npair, nmember, nullptr, p.d_pair, U, stats, W, Y, r_exact, thr, E2_pair,
                     select);
  return hipGetLastError();
}

int64_t mlp_train_ws_bytes(int nmember, int32_t nb) {
  const int64_t nblk = (nb + kTrRows - 1) / kTrRows;
  return round_up((int64_t)nmember * nblk * kMStride * (int64_t)sizeof(float), 256) +
         round_up((int64_t)nmember * nblk * (int64_t)sizeof(float), 256);
}

hipError_t launch_mlp_train_step(int nmember, const float* X, const float* T, const int32_t* idx,
                                 int32_t nb, const float* stats, float* P, float* M, float* V,
                                 uint16_t* W, int32_t step, float lr, float* loss, float* grad,
                                 void* ws, hipStream_t st) {
  configure_mlp_kernels();
  const int nblk = (nb + kTrRows - 1) / kTrRows;
  float* gpart = static_cast<float*>(ws);
  float* lpart = reinterpret_cast<float*>(
      static_cast<char*>(ws) +
      round_up((int64_t)nmember * nblk * kMStride * (int64_t)sizeof(float), 256));
  if (nblk > 0)
    hipLaunchKernelGGL(mlp_train_kernel, dim3(nblk, nmember), dim3(kNh), kTrainLds, st, X, T, idx,
                       nb, stats, W, gpart, lpart, nblk);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((FEF_MLP_NPARAM + 255) / 256, nmember), dim3(256), 0,
                     st, nblk, nb, gpart, lpart, P, M, V, W, step, lr, grad, loss);
  return hipGetLastError();
}

}  // namespace fef
