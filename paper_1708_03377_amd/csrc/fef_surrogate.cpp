// Host side of the surrogate entry points and the masked pair energies:
// argument checks and dispatch (the arithmetic is in k_mlp.hip, k_pair.hip,
// k_split.hip, k_field.hip and k_eigh.hip).
#include <algorithm>

#include "fef_internal.h"

using namespace fef;

namespace {

fef_status hip_status(hipError_t e) { return e == hipSuccess ? FEF_OK : FEF_E_HIP; }
bool valid_prec(int prec) { return prec >= 0 && prec < FEF_NPREC; }
constexpr int kMaxMembers = 64;

}  // namespace

extern "C" {

fef_status fef_pair_energies_masked(fef_plan p, const void* ops, const double* eps,
                                    fef_prec prec, const int32_t* select, double* E2_pair,
                                    double* E2_total, int32_t* flags, void* ws,
                                    size_t ws_bytes, void* stream) {
  if (!p) return FEF_E_ARG;
  if (!valid_prec(prec)) return FEF_E_PREC;
  if (!E2_total || !flags) return FEF_E_ARG;
  if (p->npair > 0 && (!ops || !eps || !E2_pair || !select)) return FEF_E_ARG;
  if ((int64_t)ws_bytes < masked_ws_bytes(*p, prec) || !ws) return FEF_E_WORKSPACE;
  return hip_status(launch_pair_energies(*p, ops, eps, prec, p->npair > 0 ? select : nullptr,
                                         E2_pair, E2_total, flags, ws,
                                         static_cast<hipStream_t>(stream)));
}

fef_status fef_coupling_modes(fef_plan p, const double* G, double* Q, void* ws, size_t ws_bytes,
                              void* stream) {
  if (!p || !G || !Q) return FEF_E_ARG;
  if ((int64_t)ws_bytes < surr_ws_bytes(*p) || !ws) return FEF_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = p->P0;
  char* b = static_cast<char*>(ws);
  double* V = reinterpret_cast<double*>(b);
  double* Dnew = V + n * n;
  double* Dold = Dnew + n * n;
  double* ev = Dold + n * n;
  double* dmax = ev + n;
  int32_t* flags = reinterpret_cast<int32_t*>(dmax + 1);
  double* slots = reinterpret_cast<double*>(
      b + round_up((3 * n * n + n + 2) * (int64_t)sizeof(double), 256));
  // G_{0,0} is the first block of the G pool
  hipError_t e = launch_eigh_one(p->d_gfrag, p->d_glist, (int)n, G, Dold, V, ev, Dnew, dmax,
                                 flags, slots, st);
  if (e == hipSuccess) e = launch_top_modes(V, (int)n, Q, st);
  return hip_status(e);
}

fef_status fef_fragment_invariants(fef_plan p, const double* B, const double* G, const double* D,
                                   const double* Q, double* U, void* ws, size_t ws_bytes,
                                   void* stream) {
  if (!p) return FEF_E_ARG;
  if (p->nfrag > 0 && (!B || !G || !D || !Q || !U)) return FEF_E_ARG;
  if ((int64_t)ws_bytes < surr_ws_bytes(*p) || !ws) return FEF_E_WORKSPACE;
  if (p->nfrag == 0) return FEF_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* dmom = static_cast<double*>(ws);
  hipError_t e = launch_moments(*p, B, D, dmom, st);
  if (e == hipSuccess) e = launch_invariants(*p, dmom, G, Q, U, st);
  return hip_status(e);
}

fef_status fef_pair_features(fef_plan p, const double* U, const double* E2_pair,
                             const int32_t* idx, int64_t n, float* X, float* T, void* stream) {
  if (!p || n < 0) return FEF_E_ARG;
  if (n == 0) return FEF_OK;
  if (!U || !X) return FEF_E_ARG;
  if ((T == nullptr) != (E2_pair == nullptr)) return FEF_E_ARG;
  if (!idx && n > p->npair) return FEF_E_SHAPE;
  return hip_status(launch_features(*p, U, E2_pair, idx, n, X, T,
                                    static_cast<hipStream_t>(stream)));
}

fef_status fef_column_stats(int64_t n, int32_t ncol, int32_t inverse, const float* A,
                            float* mean, float* sdev, void* stream) {
  if (n < 0 || ncol < 1 || ncol > 65535 || !mean || !sdev) return FEF_E_ARG;
  if (n > 0 && !A) return FEF_E_ARG;
  return hip_status(launch_column_stats(n, ncol, inverse, A, mean, sdev,
                                        static_cast<hipStream_t>(stream)));
}

fef_status fef_mlp_pack(int32_t nmember, const float* P, uint16_t* W, void* stream) {
  if (nmember < 1 || nmember > kMaxMembers || !P || !W) return FEF_E_ARG;
  return hip_status(launch_mlp_pack(nmember, P, W, static_cast<hipStream_t>(stream)));
}

fef_status fef_mlp_forward(int32_t nmember, int64_t n, const float* X, const float* stats,
                           const uint16_t* W, float* Y, void* stream) {
  if (nmember < 1 || nmember > kMaxMembers || n < 0) return FEF_E_ARG;
  if (n > 0 && (!X || !stats || !W || !Y)) return FEF_E_ARG;
  return hip_status(launch_mlp_forward(nmember, n, X, stats, W, Y,
                                       static_cast<hipStream_t>(stream)));
}

fef_status fef_mlp_train_ws_bytes(int32_t nmember, int32_t nb, int64_t* out) {
  if (nmember < 1 || nmember > kMaxMembers || nb < 0 || !out) return FEF_E_ARG;
  *out = mlp_train_ws_bytes(nmember, nb);
  return FEF_OK;
}

fef_status fef_mlp_train_step(int32_t nmember, const float* X, const float* T,
                              const int32_t* idx, int32_t nb, const float* stats, float* P,
                              float* M, float* V, uint16_t* W, int32_t step, float lr,
                              float* loss, float* grad, void* ws, size_t ws_bytes,
                              void* stream) {
  if (nmember < 1 || nmember > kMaxMembers || nb < 0 || step < 0) return FEF_E_ARG;
  if (!P || !M || !V || !W || !stats) return FEF_E_ARG;
  if (nb > 0 && (!X || !T || !idx)) return FEF_E_ARG;
  if ((int64_t)ws_bytes < mlp_train_ws_bytes(nmember, nb) || !ws) return FEF_E_WORKSPACE;
  return hip_status(launch_mlp_train_step(nmember, X, T, idx, nb, stats, P, M, V, W, step, lr,
                                          loss, grad, ws, static_cast<hipStream_t>(stream)));
}

fef_status fef_surrogate_select(fef_plan p, const double* U, int32_t nmember, const float* stats,
                                const uint16_t* W, double r_exact, double threshold,
                                double* E2_pair, int32_t* select, void* stream) {
  if (!p || nmember < 1 || nmember > kMaxMembers) return FEF_E_ARG;
  if (p->npair > 0 && (!U || !stats || !W || !E2_pair || !select)) return FEF_E_ARG;
  return hip_status(launch_surrogate_select(*p, U, nmember, stats, W, r_exact, threshold, E2_pair,
                                            select, nullptr, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
