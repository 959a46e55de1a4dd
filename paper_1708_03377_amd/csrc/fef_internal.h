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
// Largest number of x-side row tiles ("x units") one pair-kernel block holds.
constexpr int kMaxXB = 4;

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Per-fragment table (device and host copies are identical).
struct FragInfo {
  int32_t nbf, nocc, nvir, ov;
  int32_t cls, naux;     // class and its factor rank P_c
  int32_t ntile;         // ceil(ov / kTile)
  int32_t rank;          // position in the locality (RCM) order
  int64_t off_B, off_C, off_eps;
  int64_t off_bov, off_w;            // dense FP64 Bov / W pools
  int64_t off_aux;                   // offset into per-fragment [P_c] vectors
  int64_t off_gap;                   // offset into the gap pool [ld] (Delta_ia, -1 padded)
  int64_t ld;                        // ntile * kTile
  int64_t off_L[FEF_NPREC];          // byte offsets of the left operand
  int64_t off_R[FEF_NPREC];          // byte offsets of the right operand (-1: none)
};

// Oriented pair: y is always a class-0 fragment.  Its (mt, nt) output tiles
// own the partial-sum slots slot_first + mt * nty + nt.
struct PairInfo {
  int32_t x, y;
  double s;
  int32_t slot_first, ntx, nty, pad;
};

// Pair-kernel work decomposition: an x-block holds up to kMaxXB x units
// (fragment, row tile); its entries list every streamed y tile (fragment,
// column tile) that pairs with at least one unit, with the unit's partial
// slot (-1: no pair) and, resolved on the host so that a kernel reads them in
// one round of scalar loads, the tile's operand and gap offsets and each
// unit's coupling s_xy.  A work item is a contiguous range of one block's
// entries.
struct XBlock {
  int32_t f[kMaxXB];
  int32_t mt[kMaxXB];
};
struct Entry {
  int32_t y, nt;
  int32_t slot[kMaxXB];
  int32_t ld_y, pad;    // leading dimension of y's operand
  int64_t off_R;        // byte offset of the y tile in this mode's operand pool
  int64_t off_gap;      // offset of the y tile's gaps in the gap pool
  double s[kMaxXB];     // s_xy of each unit's pair (0 without a pair)
};
struct WorkItem {
  int32_t xblock, e0, ne, pad;
};

struct HtTask {
  int32_t f, p0, np, pad;
};

// Operand geometry of a precision mode.
//   FP64 / FP32: operand stored [kpad][ld], k-major, kpad = round_up(P0, 4).
//   split modes: operand stored [ld][nterm * pw + 8] (row = ia; the term
//   planes, pw = round_up(P0, 8) each, then 8 zeros so that rows staged in
//   LDS sit apart in the banks).  Two terms: the three products run as one
//   chain over round_up(3 pw, 32) contraction indices.  Three terms: the
//   products of order L (the sum of the two terms' plane indices) form
//   chain L over (L + 1) pw indices, ceil((L + 1) pw / 32) MFMA chunks of
//   32.  kpad is the total contraction length issued.
__host__ __device__ constexpr int split_chain(int level, int pw) {
  return ((level + 1) * pw + 31) / 32;
}
__host__ __device__ constexpr int split_nterm(int prec) { return prec == FEF_BF16X3 ? 3 : 2; }

// Eigensolver workspace (doubles) per fragment with nbf > 48, for the
// largest such nbf: the Jacobi path keeps V^T and a product matrix
// (2 (n + 1)^2), the tridiagonal path T (three vectors), the packed
// reflectors, the eigenvectors of T (rows padded to n + 64 columns) and the
// reflectors expanded in blocks of four for the back-transformation (rows
// of kTriVbStride, then 16 Gram entries per block).
constexpr int kTriVbStride = 152;
__host__ __device__ inline int64_t eig_large_slot(int nmax) {
  const int64_t jac = 2 * (int64_t)(nmax + 1) * (nmax + 1);
  const int64_t nb = nmax > 2 ? (nmax - 2 + 3) / 4 : 0;
  const int64_t tri = 3 * (int64_t)nmax + (int64_t)nmax * (nmax + 1) / 2 +
                      (int64_t)nmax * (nmax + 64) + nb * (4 * kTriVbStride + 16);
  return jac > tri ? jac : tri;
}
// Largest nbf of the tridiagonal (Householder) eigensolver.
constexpr int kTriMax = 152;

struct OpsGeom {
  int elem_bytes;   // bytes per stored element
  int kpad;         // padded contraction length
  int pw;           // plane width (split modes)
  int nterm;        // stored terms per value (split modes)
};

// Work items come in kQueues groups of contiguous x-blocks (locality order,
// about equal work each); group g's items are items[grp_off[g] ..
// grp_off[g + 1]), longest first.  A workgroup serves the group of its XCD
// first (workgroups are dealt to the XCDs round robin) and then helps the
// others, so neighbouring x-blocks, which stream mostly the same y tiles,
// run on one XCD and share its L2.
constexpr int kQueues = 8;
struct TileSet {
  int32_t xb = 0, yc = 0;
  int64_t nitems = 0, nentries = 0, nxblocks = 0;
  WorkItem* d_items = nullptr;
  Entry* d_entries = nullptr;
  XBlock* d_xblocks = nullptr;
  int32_t* d_grp_off = nullptr;  // [kQueues + 1]
};

}  // namespace fef

// [begin, end) of a flat pool, all inside fragment `frag`; the density pool
// is cut into chunks of at most kDensityChunk elements, the packed
// coefficient pool into chunks of at most kPackChunk.
constexpr int kDensityChunk = 1024;
constexpr int kPackChunk = 4096;
struct Chunk {
  int64_t begin, end;
  int32_t frag, pad;
};

namespace fef {
// Coupled dimer doubles: offsets (doubles) inside one pair slot of a group.
struct CgSlot {
  int64_t v, d, t, r, p, ap, q, ph, hp, hh, size;
  int64_t nmax;  // largest amplitude count ov_x ov_y of the group
  int64_t npb;   // doubles of p's storage (at least one per thread: partial sums)
};
// Pairs of one class of x (a list range), solved by nslots workgroups; lds:
// the search direction and its product live in LDS.
struct CoupledGroup {
  int32_t first = 0, count = 0, nslots = 0;
  bool lds = false;
  size_t lds_bytes = 0;
  CgSlot L{};
};
}  // namespace fef

// Stage markers of an SCF step: start, after the density, after the
// moments, after the field and Coulomb build, after the eigensolver.
constexpr int kStageMarks = 5;

struct fef_plan_s {
  int device = 0;
  // SCF stage timing (fef_plan_stage_timing): events recorded at the stage
  // markers of every SCF step while enabled
  hipEvent_t stage_ev[kStageMarks] = {};
  bool stage_timing = false;
  int32_t nfrag = 0, nclass = 0, P0 = 0;
  int64_t npair = 0, nslot = 0;
  int32_t max_nbf = 0, max_naux = 0, max_ov = 0;
  int64_t max_on = 0;   // max nocc * nbf (half-transform LDS)
  int64_t ops_header = 0;  // bytes of per-fragment scale factors at the start of ops
  std::vector<fef::FragInfo> frag;
  std::vector<int32_t> naux_cls;
  std::vector<int64_t> off_G;
  std::vector<int32_t> naux_cls_off;  // prefix sums of P_c over classes
  int64_t nB = 0, nC = 0, nEps = 0, nBov = 0, nW = 0, nG = 0, nGap = 0;
  int64_t ops_bytes[FEF_NPREC] = {};
  fef::OpsGeom geom[FEF_NPREC];
  // eigen-solver groups: fragments by size class
  std::vector<int32_t> eig_small, eig_mid, eig_large;
  int32_t eig_w_off[5] = {0, 0, 0, 0, 0};  // eig_small ranges with n <= 8, 16, 24, 32
  int32_t eig_large_max_nbf = 0;
  int64_t ht_ntasks = 0;
  std::vector<int32_t> ht_fused, ht_generic;  // half-transform paths per fragment
  int32_t fuse_lds[3] = {0, 0, 0};             // small-fragment maxima: nbf^2, nocc nbf, P ov
  int32_t max_naux_small = 0;                  // largest P_c among the small fragments
  int32_t* d_ht_fused = nullptr;
  int32_t* d_ht_generic = nullptr;
  // device tables
  fef::FragInfo* d_frag = nullptr;
  fef::PairInfo* d_pair = nullptr;
  int32_t* d_slot_pair = nullptr;     // slot -> pair index
  std::vector<fef::PairInfo> pairs;   // host copy (oriented)
  std::vector<int32_t> rank;          // locality order position per fragment
  fef::TileSet tiles[FEF_NPREC];
  // captured passes alive per mode: while any holds a mode's tile tables,
  // a retune keeps the superseded tables (freed with the plan)
  int32_t graphs_live[FEF_NPREC] = {};
  std::vector<fef::TileSet> retired_tiles;
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
  // packed (upper-triangle) coefficient pool: per-fragment offsets
  int64_t nBp = 0;
  int64_t* d_off_Bp = nullptr;
  int64_t nTri = 0;                 // sum of nbf (nbf + 1) / 2
  int64_t* d_off_tri = nullptr;     // per-fragment offsets of packed nbf x nbf triangles
  // element chunks of the flat density pool and of the packed coefficient
  // pool, each inside one fragment (one block per chunk)
  int64_t n_chunk_C = 0, n_chunk_Bp = 0;
  Chunk* d_chunk_C = nullptr;
  Chunk* d_chunk_Bp = nullptr;
  // G_{0,0} posed as one "fragment" for the eigensolver (coupling modes)
  fef::FragInfo* d_gfrag = nullptr;
  int32_t* d_glist = nullptr;
  // coupled dimer doubles: pair groups and their pair lists
  std::vector<fef::CoupledGroup> cp_groups;
  std::vector<int32_t> cp_list;
  int32_t* d_cp_list = nullptr;
  // dimer dressings: per-pair record offsets, per-fragment output offsets,
  // and each fragment's record parts in pair order
  int64_t n_rec = 0, n_oo = 0, n_vv = 0;
  int64_t* d_rec_off = nullptr;
  int64_t* d_off_oo = nullptr;
  int64_t* d_off_vv = nullptr;
  int32_t* d_inc_ptr = nullptr;
  int64_t* d_inc_base = nullptr;
};

namespace fef {

// Kernel launchers (defined next to their kernels).
hipError_t launch_half_transform(const fef_plan_s& p, const double* B, const double* C,
                                 const double* G, double* bov, double* w, void* ops,
                                 fef_prec prec, hipStream_t st, bool dense_out);
hipError_t launch_pack_split(const fef_plan_s& p, const double* bov, const double* w,
                             void* ops, fef_prec prec, hipStream_t st);
hipError_t launch_pair_energies(const fef_plan_s& p, const void* ops, const double* eps,
                                fef_prec prec, const int32_t* select, double* E2_pair,
                                double* E2_total, int32_t* flags, void* ws, hipStream_t st);
hipError_t launch_density(const fef_plan_s& p, const double* C, double* D, double* Dw,
                          double* dD_max, hipStream_t st);
hipError_t launch_field(const fef_plan_s& p, const double* B, const double* G,
                        const double* D, const double* F0, const double* htilde,
                        double* out, double* ws_d, double* ws_phi, hipStream_t st);
// Dw non-null (only when every fragment has nbf <= 32): the register-
// resident solvers also write the weighted packed density of the new
// orbitals, bitwise as launch_density forms it, for the next step
// Bp and dmom non-null (moments_carry_ok only, with Dw): the register-resident
// solvers also leave the Coulomb moments of the new densities in dmom,
// bitwise as the packed moments kernel forms them, for the next step
hipError_t launch_eigh(const fef_plan_s& p, const double* F, const double* Dold,
                       double* C, double* eps, double* Dnew, double* dD_max,
                       int32_t* flags, double* ws_eig, hipStream_t st, double* Dw = nullptr,
                       const double* Bp = nullptr, double* dmom = nullptr);
hipError_t launch_eigh_tri(const fef_plan_s& p, const double* F, const double* Dold, double* C,
                           double* eps, double* Dnew, double* dD_max, int32_t* flags,
                           double* ws_eig, hipStream_t st);
hipError_t launch_eigh_one(const FragInfo* d_fi, const int32_t* d_list, int n, const double* F,
                           const double* Dold, double* C, double* eps, double* Dnew,
                           double* dmax, int32_t* flags, double* ws_eig, hipStream_t st);
hipError_t launch_pack_coefficients(const fef_plan_s& p, const double* B, double* Bp,
                                    hipStream_t st);
// every fragment has nbf <= 32 and P <= 80 (the fused field + J kernel applies)
bool small_fragments(const fef_plan_s& p);
hipError_t launch_zero_scalar(double* x, hipStream_t st);  // *x = 0 (a kernel, not a memset)
// B_pack non-null: the moments kernel reads the slices from B and writes
// their packed copy to Bp_out (= Bp) on the way (the first step of a pass).
// zero_out non-null: the moments kernel also sets *zero_out = 0.
hipError_t launch_field_packed(const fef_plan_s& p, const double* Bp, const double* G,
                               const double* Dw, const double* F0, const double* htilde,
                               double* out, double* ws_d, double* ws_phi, hipStream_t st,
                               const double* B_pack = nullptr, double* Bp_out = nullptr,
                               double* zero_out = nullptr, bool moments_given = false);
hipError_t launch_moments(const fef_plan_s& p, const double* B, const double* D, double* dmom,
                          hipStream_t st);
// One packed SCF step that also writes the packed copy Bp of B (its moments
// kernel reads the slices from B): the first step of a captured pass, in
// place of packing followed by a packed step, with the same results.
fef_status scf_step_packing(fef_plan p, const double* B, double* Bp, const double* G,
                            const double* F0, const double* htilde, double* C, double* eps,
                            double* D, double* dD_max, int32_t* flags, void* ws, size_t ws_bytes,
                            void* stream);
// Packed SCF steps of a captured pass when every fragment has nbf <= 32
// (step = 0 .. nsteps - 1; B_pack non-null only for step 0, which packs B
// into Bp on the way): each step's eigensolver also leaves the weighted
// packed density of its orbitals in the workspace, so the next step runs
// no density kernel.  The densities alternate between a spare workspace
// pool and D, the last step's landing in D.  Same results as packed steps.
bool density_carry_ok(const fef_plan_s& p);
// the carried steps also carry the Coulomb moments (the eigensolver of one
// step forms those of the next): every fragment small enough for the
// register-resident eigensolver and the fused field kernel, with an even
// packed triangle of at most 384 numbers
bool moments_carry_ok(const fef_plan_s& p);
fef_status scf_step_carry(fef_plan p, const double* B_pack, double* Bp, const double* G,
                          const double* F0, const double* htilde, double* C, double* eps,
                          double* D, double* dD_max, int32_t* flags, void* ws, size_t ws_bytes,
                          void* stream, int step, int nsteps);

// Surrogate (k_mlp.hip).
hipError_t launch_top_modes(const double* V, int n, double* Q, hipStream_t st);
hipError_t launch_invariants(const fef_plan_s& p, const double* dmom, const double* G,
                             const double* Q, double* U, hipStream_t st);
hipError_t launch_features(const fef_plan_s& p, const double* U, const double* E2,
                           const int32_t* idx, int64_t n, float* X, float* T, hipStream_t st);
hipError_t launch_column_stats(int64_t n, int ncol, int inverse, const float* A, float* mean,
                               float* sdev, hipStream_t st);
hipError_t launch_mlp_pack(int nmember, const float* P, uint16_t* W, hipStream_t st);
hipError_t launch_mlp_forward(int nmember, int64_t n, const float* X, const float* stats,
                              const uint16_t* W, float* Y, hipStream_t st);
hipError_t launch_surrogate_select(const fef_plan_s& p, const double* U, int nmember,
                                   const float* stats, const uint16_t* W, double r_exact,
                                   double thr, double* E2_pair, int32_t* select, float* Y,
                                   hipStream_t st);
int64_t mlp_train_ws_bytes(int nmember, int32_t nb);
hipError_t launch_mlp_train_step(int nmember, const float* X, const float* T, const int32_t* idx,
                                 int32_t nb, const float* stats, float* P, float* M, float* V,
                                 uint16_t* W, int32_t step, float lr, float* loss, float* grad,
                                 void* ws, hipStream_t st);

// Pair-kernel tiling (fef_tiles.cpp).
void order_and_orient(fef_plan_s& p);
hipError_t build_tiles(fef_plan_s& p, int prec, int xb, int yc);
void free_tiles(fef::TileSet& t);

// Address of this library's fixed pair-kernel scratch array on `device`
// (looked up once per device, with that device current).
hipError_t noalloc_setup(int device);

// Records stage marker i of an SCF step on st when stage timing is on.
inline void stage_mark(const fef_plan_s& p, int i, hipStream_t st) {
  if (p.stage_timing) (void)hipEventRecord(p.stage_ev[i], st);
}

// Compute units of the current device (queried once, cached).
int compute_units();
// coupled dimer doubles and dressings: pair groups and tables (plan
// creation; allocates), workspace bytes
hipError_t coupled_setup(fef_plan_s& p);
int64_t coupled_ws_bytes(const fef_plan_s& p);
int64_t dressing_ws_bytes(const fef_plan_s& p);

// One-time kernel attributes (dynamic LDS above 64 KB).

// Workspace sizes (bytes).
int64_t half_ws_bytes(const fef_plan_s& p, fef_prec prec);
int64_t pair_ws_bytes(const fef_plan_s& p, fef_prec prec);
int64_t field_ws_bytes(const fef_plan_s& p);
int64_t scf_ws_bytes(const fef_plan_s& p);
int64_t masked_ws_bytes(const fef_plan_s& p, fef_prec prec);
int64_t surr_ws_bytes(const fef_plan_s& p);
int64_t naux_total(const fef_plan_s& p);

}  // namespace fef
