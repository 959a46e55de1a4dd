// Internal definitions shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/fef.h"

namespace fef {

// Pair-kernel output tile (rows = ia of x, columns = jb of y).  96 = 6 x 16
// MFMA tiles, so a water-like fragment (ov = 95) needs one tile per side.
constexpr int kTile = 96;

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Per-fragment table (device and host copies are identical).
struct FragInfo {
  int32_t nbf, nocc, nvir, ov;
  int32_t cls, naux;     // class and its factor rank P_c
  int32_t ntile;         // ceil(ov / kTile)
  int32_t pad0;
  int64_t off_B, off_C, off_eps;
  int64_t off_bov, off_w;            // dense FP64 Bov / W pools
  int64_t off_aux;                   // offset into per-fragment [P_c] vectors
  int64_t ld;                        // ntile * kTile
  int64_t off_L[FEF_NPREC];          // byte offsets of the left operand
  int64_t off_R[FEF_NPREC];          // byte offsets of the right operand (-1: none)
};

// Oriented pair: y is always a class-0 fragment.
struct PairInfo {
  int32_t x, y;
  double s;
  int32_t item_first, item_count;
};

struct Item {
  int32_t pair, mt, nt, pad;
};

struct HtTask {
  int32_t f, p0, np, pad;
};

// Operand geometry of a precision mode.
struct OpsGeom {
  int elem_bytes;   // bytes per stored element (per plane for split modes)
  int kpad;         // padded contraction length
};

}  // namespace fef

struct fef_plan_s {
  int device = 0;
  int32_t nfrag = 0, nclass = 0, P0 = 0;
  int64_t npair = 0, nitems = 0;
  int32_t max_nbf = 0, max_naux = 0, max_ov = 0;
  int64_t max_on = 0;   // max nocc * nbf (half-transform LDS)
  int64_t ops_header = 0;  // bytes of per-fragment scale factors at the start of ops
  std::vector<fef::FragInfo> frag;
  std::vector<int32_t> naux_cls;
  std::vector<int64_t> off_G;
  std::vector<int32_t> naux_cls_off;  // prefix sums of P_c over classes
  int64_t nB = 0, nC = 0, nEps = 0, nBov = 0, nW = 0, nG = 0;
  int64_t ops_bytes[FEF_NPREC] = {0, 0, 0, 0};
  fef::OpsGeom geom[FEF_NPREC];
  // eigen-solver groups: fragments by size class
  std::vector<int32_t> eig_small, eig_mid, eig_large;
  int32_t eig_large_max_nbf = 0;
  int64_t ht_ntasks = 0;
  // device tables
  fef::FragInfo* d_frag = nullptr;
  fef::PairInfo* d_pair = nullptr;
  fef::Item* d_item = nullptr;
  fef::HtTask* d_ht = nullptr;
  int64_t* d_off_G = nullptr;
  int32_t* d_naux_cls_off = nullptr;
  int32_t* d_nbr_ptr = nullptr;
  int32_t* d_nbr_idx = nullptr;
  double* d_nbr_s = nullptr;
  int32_t* d_eig_small = nullptr;
  int32_t* d_eig_mid = nullptr;
  int32_t* d_eig_large = nullptr;
  int64_t nbr_total = 0;
};

namespace fef {

// Kernel launchers (defined next to their kernels).
hipError_t launch_half_transform(const fef_plan_s& p, const double* B, const double* C,
                                 const double* G, double* bov, double* w, void* ops,
                                 fef_prec prec, hipStream_t st);
hipError_t launch_pack_split(const fef_plan_s& p, const double* bov, const double* w,
                             void* ops, fef_prec prec, hipStream_t st);
hipError_t launch_pair_energies(const fef_plan_s& p, const void* ops, const double* eps,
                                fef_prec prec, double* E2_pair, double* E2_total,
                                int32_t* flags, void* ws, hipStream_t st);
hipError_t launch_density(const fef_plan_s& p, const double* C, double* D,
                          double* dD_max, hipStream_t st);
hipError_t launch_field(const fef_plan_s& p, const double* B, const double* G,
                        const double* D, const double* F0, const double* htilde,
                        double* out, double* ws_d, double* ws_phi, hipStream_t st);
hipError_t launch_eigh(const fef_plan_s& p, const double* F, const double* Dold,
                       double* C, double* eps, double* Dnew, double* dD_max,
                       int32_t* flags, double* ws_eig, hipStream_t st);

// Workspace sizes (bytes).
int64_t half_ws_bytes(const fef_plan_s& p, fef_prec prec);
int64_t pair_ws_bytes(const fef_plan_s& p, fef_prec prec);
int64_t field_ws_bytes(const fef_plan_s& p);
int64_t scf_ws_bytes(const fef_plan_s& p);

}  // namespace fef
