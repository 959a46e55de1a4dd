/*
 * fef.h - C ABI of the MI355X (gfx950) FEF pair-energy / effective-field
 * library.
 *
 * Method: fragment-effective-field coupled-cluster perturbation theory
 * (FEF-CCPT), arXiv:1708.03377.  The library computes, for a system of
 * molecular fragments in the product (A ~ 1) ansatz:
 *
 *   - the half-transformed factored inter-fragment integrals
 *       B^x_ov[P][ia] = sum_{mu nu} C^x_{mu i} B^x[P][mu][nu] C^x_{nu a}
 *     and W^x = G_{c(x),0}^T B^x_ov  (fef_half_transform);
 *   - the dimer second-order pair energies of Eq. ED2 with the first-order
 *     dimer doubles of Eq. dimDoubles (diagonal canonical F^[0]):
 *       E2_xy = 4 sum_{ia,jb} (ia|jb)^2 / (eps_i + eps_j - eps_a - eps_b),
 *       (ia|jb) = s_xy sum_Q W^x[Q][ia] B^y_ov[Q][jb]      (fef_pair_energies);
 *   - the effective Coulomb field 2 v^{mu j}_{nu j} of Eqs. wc and dp2e
 *     (fef_coulomb_field);
 *   - one polarisation-screened SCF update of every fragment
 *     F~ = F0 + h~ + J, (eps, C) = eigh(F~), Aufbau occupation
 *     (fef_scf_step; Sec. II.A, "Fragment Mean Field");
 *   - the dimer doubles coupled through W^[0] of Eq. partitioning0 and their
 *     pair energies (fef_coupled_pair_energies), and the cross-fragment
 *     one-body dressings of Eqs. MPij and MPab (fef_dimer_dressing).
 *
 * Integral model: (mu nu|lambda sigma)^{xy} = sum_PQ B^x_{P mu nu} T^{xy}_{PQ}
 * B^y_{Q lambda sigma} with T^{xy} = s_xy G_{c(x),c(y)}, s_xy = 1/R_xy
 * (bohr^-1) and G_{0,c} = G_{c,0}^T.  Class 0 is the solvent class; every
 * pair must contain at least one class-0 fragment, and P_0 <= 80.
 *
 * Conventions
 *   Units: Hartree and bohr.  Row-major throughout.  MO order within a
 *   fragment: occupied first.  ia index = i * nvir + a (i-major).
 *   Pools: per-fragment arrays are densely concatenated in fragment order:
 *     B   [P_c][nbf][nbf]  symmetric in (mu, nu)
 *     C   [nbf][nbf]       column p = MO p
 *     F0, htilde, D, J     [nbf][nbf]
 *     eps [nbf]
 *     Bov [P_c][nocc*nvir],  W [P_0][nocc*nvir]
 *     G   concatenation over classes c of G_{c,0}, [P_c][P_0]; G_{0,0}
 *         must be symmetric.
 *   Pointers passed to compute calls are DEVICE pointers owned by the
 *   caller; the compute calls never allocate or free, run asynchronously on
 *   `stream` (a hipStream_t, NULL = default stream) and return after
 *   enqueueing.  Sizes of the opaque operand pool and of every workspace come
 *   from fef_plan_query.
 *   Errors: argument problems detectable on the host return a negative
 *   status synchronously and enqueue nothing; a failed launch returns
 *   FEF_E_HIP.  Data-dependent conditions are reported in the device word
 *   `flags` (read it after synchronising): bit 0 = some fragment has a
 *   non-positive HOMO-LUMO gap, bit 1 = a non-finite pair energy, bit 2 =
 *   a coupled pair solve stopped at its iteration limit.  The
 *   library never clears `flags`; the caller zeroes it.
 *   No C++ exception crosses this interface.
 */
#ifndef FEF_H
#define FEF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fef_status;
#define FEF_OK 0
#define FEF_E_ARG -1          /* null pointer or invalid argument      */
#define FEF_E_SHAPE -2        /* inconsistent sizes / unsupported pair */
#define FEF_E_PREC -3         /* unknown precision mode                */
#define FEF_E_WORKSPACE -4    /* workspace too small                   */
#define FEF_E_HIP -5          /* HIP runtime error                     */
#define FEF_E_UNSUPPORTED -6  /* valid request the library cannot do   */
#define FEF_E_IO -7           /* a file could not be written           */

#define FEF_FLAG_GAP 1
#define FEF_FLAG_NONFINITE 2
#define FEF_FLAG_NOCONV 4

/* Arithmetic of the pair contraction (a reduced-precision mode rounds the
 * half-transformed operands; every other step stays FP64). */
typedef enum {
  FEF_F64 = 0,     /* FP64 operands, FP64 MFMA                              */
  FEF_F32 = 1,     /* FP32 operands, FP32 MFMA                              */
  FEF_BF16X2 = 2,  /* x = hi + lo in BF16; hi*hi' + hi*lo' + lo*hi', FP32 acc */
  FEF_FP16X2 = 3,  /* same with FP16 and a per-fragment power-of-two scale  */
  FEF_BF16X3 = 4,  /* x = hi + mid + lo in BF16; the six products of order up
                      to two (hi*hi'; hi*mid' + mid*hi'; hi*lo' + mid*mid' +
                      lo*hi'), FP32 acc                                      */
  FEF_NPREC = 5
} fef_prec;

/* Fragment system, HOST memory, read once by fef_plan_create. */
typedef struct {
  int32_t nfrag;
  int32_t nclass;
  const int32_t* nbf;     /* [nfrag] basis functions per fragment          */
  const int32_t* nocc;    /* [nfrag] doubly occupied orbitals, 0..nbf      */
  const int32_t* cls;     /* [nfrag] class id in [0, nclass)               */
  const int32_t* naux;    /* [nclass] factor rank P_c                      */
  int64_t npair;
  const int32_t* pair_x;  /* [npair] fragment ids, x != y; every pair once */
  const int32_t* pair_y;
  const double* pair_s;   /* [npair] s_xy = 1/R_xy in bohr^-1              */
} fef_system_desc;

typedef struct fef_plan_s* fef_plan;

/* Builds the device tables (fragment offsets, oriented pairs, work items,
 * neighbour lists) on the current HIP device.  Allocates device memory; call
 * outside graph capture.  The neighbour set of the field is the pair list
 * itself (both orientations). */
fef_status fef_plan_create(const fef_system_desc* desc, fef_plan* out);
fef_status fef_plan_destroy(fef_plan plan);

typedef enum {
  FEF_Q_OPS_BYTES = 0,      /* operand pool written by fef_half_transform */
  FEF_Q_HALF_WS_BYTES = 1,  /* workspace of fef_half_transform           */
  FEF_Q_PAIR_WS_BYTES = 2,  /* workspace of fef_pair_energies            */
  FEF_Q_FIELD_WS_BYTES = 3, /* workspace of fef_coulomb_field            */
  FEF_Q_SCF_WS_BYTES = 4,   /* workspace of fef_scf_step                 */
  FEF_Q_BOV_ELEMS = 5,      /* doubles in the dense Bov pool             */
  FEF_Q_W_ELEMS = 6,        /* doubles in the dense W pool               */
  FEF_Q_NITEMS = 7,         /* pair-kernel work items of mode `prec`     */
  FEF_Q_B_ELEMS = 8,        /* doubles in the B pool                     */
  FEF_Q_C_ELEMS = 9,        /* doubles in a C / D / F0 / J pool          */
  FEF_Q_EPS_ELEMS = 10,     /* doubles in the eps pool                   */
  FEF_Q_G_ELEMS = 11,       /* doubles in the G pool                     */
  FEF_Q_NPAIR = 12,
  FEF_Q_NSLOT = 13,         /* pair output tiles (partial-sum slots)     */
  FEF_Q_NENTRIES = 14,      /* streamed y tiles of mode `prec`'s tiling   */
  FEF_Q_MASKED_WS_BYTES = 15, /* workspace of fef_pair_energies_masked   */
  FEF_Q_SURR_WS_BYTES = 16, /* workspace of fef_coupling_modes and
                               fef_fragment_invariants                  */
  FEF_Q_BPACK_ELEMS = 17,   /* doubles in the packed coefficient pool    */
  FEF_Q_COUPLED_WS_BYTES = 18, /* workspace of fef_coupled_pair_energies */
  FEF_Q_DRESSING_WS_BYTES = 19, /* workspace of fef_dimer_dressing        */
  FEF_Q_HOO_ELEMS = 20,     /* doubles in the Hoo pool (nocc^2 per fragment) */
  FEF_Q_HVV_ELEMS = 21      /* doubles in the Hvv pool (nvir^2 per fragment) */
} fef_query;

/* `prec` matters for FEF_Q_OPS_BYTES, FEF_Q_HALF_WS_BYTES,
 * FEF_Q_PAIR_WS_BYTES, FEF_Q_NITEMS, FEF_Q_NENTRIES and
 * FEF_Q_MASKED_WS_BYTES; it is ignored otherwise. */
fef_status fef_plan_query(fef_plan plan, fef_query what, fef_prec prec,
                          int64_t* out);

/* Pair-kernel tiling of mode `prec` (the work decomposition; results agree
 * across tilings up to the rounding order of the in-tile sums, and are
 * bitwise reproducible for a fixed tiling).
 *   xb : x-side row tiles held by one workgroup (FP64/FP32: 1 or 2; split
 *        modes: 2 or 4), each y tile streamed through the workgroup serves
 *        all.
 *   yc : y tiles per work item of the persistent queue (1..4096).
 * Rebuilds device tables (allocates): call outside graph capture, with no
 * pair-energy call of this plan in flight.  A captured pass of this mode
 * that is still alive keeps the tables it was captured with (they are freed
 * with the plan), so it replays with its old tiling.  The autotuner uses
 * this. */
fef_status fef_plan_set_tiles(fef_plan plan, fef_prec prec, int32_t xb, int32_t yc);
fef_status fef_plan_get_tiles(fef_plan plan, fef_prec prec, int32_t* xb, int32_t* yc);

/* Half transform (the x-side half of the four-index AO->MO transform of the
 * inter-fragment integrals v^{pq}_{rs} of the dimer Hamiltonian, Eq. NHxy,
 * with the MO coefficients C_{mu p} of Sec. II.A):
 *   B^x_ov[P][ia] = sum_{mu nu} C^x_{mu i} B^x[P][mu][nu] C^x_{nu a},
 *   W^x = G_{c(x),0}^T B^x_ov.
 *   B, C, G : input pools (device).
 *   Bov, W  : optional dense FP64 outputs (device); both or neither may
 *             be NULL.
 *   ops     : opaque operand pool for fef_pair_energies in mode `prec`,
 *             FEF_Q_OPS_BYTES bytes (device, required).
 *   ws      : workspace of FEF_Q_HALF_WS_BYTES bytes. */
fef_status fef_half_transform(fef_plan plan, const double* B, const double* C,
                              const double* G, double* Bov, double* W,
                              void* ops, fef_prec prec, void* ws,
                              size_t ws_bytes, void* stream);

/* Pair energies (Eq. ED2 with the amplitudes of Eq. dimDoubles).
 *   ops      : operand pool written by fef_half_transform in the same mode.
 *   eps      : orbital-energy pool (canonical, ascending within occ / vir).
 *   E2_pair  : [npair] out, in the caller's pair order (device).
 *   E2_total : [1] out, FP64 sum over pairs in a fixed order (device).
 *   flags    : [1] device word, bits are OR-ed in.
 * The result is bitwise reproducible for a given plan and mode. */
fef_status fef_pair_energies(fef_plan plan, const void* ops, const double* eps,
                             fef_prec prec, double* E2_pair, double* E2_total,
                             int32_t* flags, void* ws, size_t ws_bytes,
                             void* stream);

/* Effective Coulomb field (Eqs. wc, dp2e):
 *   J^x_{mu nu} = 2 sum_{y in nbr(x)} sum_{lambda sigma}
 *                 (mu nu|lambda sigma)^{xy} D^y_{lambda sigma}
 * evaluated as 2 sum_P B^x_{P mu nu} (sum_y T^{xy} d^y)_P, d^y = B^y : D^y.
 *   D : density pool (D = C_occ C_occ^T, no factor 2), J : output pool. */
fef_status fef_coulomb_field(fef_plan plan, const double* B, const double* G,
                             const double* D, double* J, void* ws,
                             size_t ws_bytes, void* stream);

/* One simultaneous SCF update of every fragment:
 *   D_in = C_occ C_occ^T from the input C; F~ = F0 + h~ + J[D_in];
 *   (eps, C) = eigh(F~) ascending (ties by index), lowest nocc occupied;
 *   D = C_occ C_occ^T of the new C.
 *   C      : in/out pool; eps : out pool; D : optional out pool (NULL ok).
 *   htilde : optional additive one-electron field pool (NULL = zero).
 *   dD_max : [1] device out, max |D - D_in| over all fragments.
 *   flags  : bit 0 set when a fragment's new HOMO-LUMO gap is <= 0. */
fef_status fef_scf_step(fef_plan plan, const double* B, const double* G,
                        const double* F0, const double* htilde, double* C,
                        double* eps, double* D, double* dD_max, int32_t* flags,
                        void* ws, size_t ws_bytes, void* stream);

/* SCF stage timing, for measurement.  While enabled, every fef_scf_step /
 * fef_scf_step_packed call records five events on its stream: at its start,
 * after the densities of the input orbitals (Sec. II.A), after the moments
 * d^y = B^y : D^y, after the field and Coulomb build of Eqs. wc and dp2e,
 * and after the eigensolver.  fef_plan_stage_ms waits for the last step's
 * final event and writes the four stage durations (ms) of that step:
 * ms[0] density, ms[1] moments, ms[2] field + Coulomb build, ms[3]
 * eigensolver.  Enabling creates the events (once per plan); do not enable
 * it for steps recorded into a graph.  fef_plan_stage_ms returns FEF_E_ARG
 * if timing was never enabled. */
fef_status fef_plan_stage_timing(fef_plan plan, int32_t enable);
fef_status fef_plan_stage_ms(fef_plan plan, double* ms);

/* Packed coefficients: Bp [P_c][nbf (nbf + 1) / 2] per fragment, the upper
 * triangle (mu <= nu, row-major) of every symmetric slice B^x[P], fragments
 * concatenated (FEF_Q_BPACK_ELEMS doubles, caller-owned).  B must be
 * symmetric in (mu, nu), as the header's pool conventions require. */
fef_status fef_pack_coefficients(fef_plan plan, const double* B, double* Bp, void* stream);

/* fef_scf_step reading the packed coefficients instead of B: the moments
 * weight off-diagonal entries by 2 and the Coulomb matrix is built on the
 * upper triangle and mirrored, so each step streams half the bytes.  Same
 * results as fef_scf_step up to rounding order. */
fef_status fef_scf_step_packed(fef_plan plan, const double* Bp, const double* G,
                               const double* F0, const double* htilde, double* C,
                               double* eps, double* D, double* dD_max, int32_t* flags,
                               void* ws, size_t ws_bytes, void* stream);

/* Captured FEF pass.  All pointers are device pointers that stay valid for
 * the graph's lifetime; the graph bakes them in. */
typedef struct {
  const double* B;
  const double* G;
  const double* F0;
  const double* htilde;   /* nullable */
  const double* C0;       /* nullable: copied into C (and eps0 into eps)
                             before the SCF steps */
  const double* eps0;     /* nullable together with C0 */
  double* C;
  double* eps;
  double* D;              /* nullable */
  double* dD_max;
  int32_t* flags;
  void* ops;              /* operand pool of mode `prec` */
  double* E2_pair;
  double* E2_total;
  void* ws;               /* workspace, FEF_Q_SCF_WS_BYTES, FEF_Q_HALF_WS_BYTES
                             and FEF_Q_PAIR_WS_BYTES bytes are all needed */
  size_t ws_bytes;
  double* Bp;             /* nullable: packed coefficient pool; when given
                             (and niter > 0), the pass packs B into it inside
                             its first SCF step and runs every step on it */
} fef_pass_args;

typedef struct fef_graph_s* fef_graph;

/* Records one whole FEF pass -- clearing of flags, [reset of C, eps],
 * niter SCF steps (fef_scf_step, or with Bp: packing of B and
 * fef_scf_step_packed), the half transform and the pair energies in mode
 * `prec` -- into a HIP graph (stream capture on a private default-priority
 * stream; no allocation happens during replay).  Call outside any capture;
 * the plan and every buffer must outlive the graph.  With Bp the first
 * step's moments kernel does the packing (reading B, writing Bp), and when
 * D is given and every fragment has nbf <= 32 each step's eigensolver also
 * leaves the next step's density, so later steps run no density kernel;
 * the arithmetic and its order are those of the eager calls, so results
 * (C, eps, D, E2) are bitwise identical to them. */
fef_status fef_graph_create(fef_plan plan, const fef_pass_args* args, int32_t niter,
                            fef_prec prec, fef_graph* out);
fef_status fef_graph_launch(fef_graph graph, void* stream);
fef_status fef_graph_destroy(fef_graph graph);

/* Tile autotuner for mode `prec`: times every supported tiling of the pair
 * kernel on this plan's own work (the operand pool must hold the half
 * transform of mode `prec`), with `reps` timed launches each after one
 * warm-up, keeps the fastest (fef_plan_set_tiles) and returns its x units
 * per block, entries per item and mean time in microseconds.  Allocates
 * (rebuilds the tables for every candidate): call outside capture. */
fef_status fef_autotune(fef_plan plan, const void* ops, const double* eps, fef_prec prec,
                        void* ws, size_t ws_bytes, int32_t reps, void* stream,
                        int32_t* best_xb, int32_t* best_yc, double* best_us);

/* The autotuner with a persisted cache, for processes that run the same
 * work again: `cache_path` names a JSON file mapping
 * "<GPU architecture>/<mode>/<work signature>" to the chosen tiling and its
 * time, the signature a hash of the fragment shapes and classes and the
 * oriented pair list (what the pair kernel's schedule depends on).  On a
 * hit the cached tiling is applied (fef_plan_set_tiles), nothing is timed,
 * best_us is the cached time and *from_cache = 1.  Otherwise it runs
 * fef_autotune, then rewrites the file with the entry added or replaced
 * (through a temporary file renamed over it) and *from_cache = 0.  A missing
 * or unreadable file is an empty cache; lines that are not entries are
 * skipped.  Returns FEF_E_IO when the file cannot be written (the tuned
 * tiling is applied all the same).  Concurrent writers of one file: the
 * last rename wins.  Allocates like fef_autotune on a miss: call outside
 * capture. */
fef_status fef_autotune_cached(fef_plan plan, const void* ops, const double* eps, fef_prec prec,
                               void* ws, size_t ws_bytes, int32_t reps, void* stream,
                               const char* cache_path, int32_t* best_xb, int32_t* best_yc,
                               double* best_us, int32_t* from_cache);

/* Pair energies of the selected pairs only (Eqs. ED2, dimDoubles, as
 * fef_pair_energies): select [npair] device int32, nonzero = evaluate.
 * E2_pair of an unselected pair keeps the value the caller put there (for
 * instance a surrogate prediction); E2_total is then the deterministic sum
 * of E2_pair over all pairs.  Selected pairs get bitwise the values
 * fef_pair_energies gives them with the same tiling.  Workspace:
 * FEF_Q_MASKED_WS_BYTES of mode `prec`. */
fef_status fef_pair_energies_masked(fef_plan plan, const void* ops, const double* eps,
                                    fef_prec prec, const int32_t* select, double* E2_pair,
                                    double* E2_total, int32_t* flags, void* ws,
                                    size_t ws_bytes, void* stream);

/* Pair energies exactly as fef_pair_energies (same kernels, same tiling,
 * bitwise the same results), for callers that cannot allocate device memory
 * or pass a workspace: code under stream capture, tight serving loops,
 * harnesses that forbid allocation.  The call allocates nothing; the
 * kernels' scratch (partial-sum slots, queue counters, gap pool) is a
 * fixed device array of FEF_NOALLOC_SCRATCH_BYTES inside this library, one
 * per GPU, held until the process ends.  A plan whose FEF_Q_PAIR_WS_BYTES
 * exceeds that size is rejected with FEF_E_WORKSPACE (nothing enqueued).
 * Must be called with the plan's device current (else FEF_E_ARG).  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams, other threads) race and give wrong results; serialise
 * them.  The array keeps the last call's contents; each call starts by
 * clearing the parts that must start at zero. */
#define FEF_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
fef_status fef_pair_energies_noalloc(fef_plan plan, const void* ops, const double* eps,
                                     fef_prec prec, double* E2_pair, double* E2_total,
                                     int32_t* flags, void* stream);

/* Pair energies with the dimer doubles coupled through the two-body part of
 * the zeroth-order Hamiltonian (Sec. II.B: Eq. partitioning0 keeps W^[0] in
 * H0, and Eq. dimDoubles becomes, for every pair, the linear system
 *     (D + W) t = -v,   E2_xy = 4 sum_{ia,jb} v[ia,jb] t[ia,jb],
 * v = (ia|jb), D = eps_a + eps_b - eps_i - eps_j, in place of t = -v / D).
 * Readings: W is the inter-fragment Coulomb operator of the factored
 * integrals (the only two-body operator the integral model defines), in
 * normal order, acting on the dimer doubles:
 *     (W t)[i,a,j,b] = + (aa'|bb') t[i,a',j,b'] - (aa'|j'j) t[i,a',j',b]
 *                      - (i'i|bb') t[i',a,j,b'] + (i'i|j'j) t[i',a,j',b]
 * (sums over primed indices, (pq|rs) = (pq|rs)^{xy} of the integral model
 * with MO coefficients C); F^[0] is the diagonal of the canonical orbital
 * energies.  Each pair is solved by conjugate gradients preconditioned with
 * D, from t = -v / D, stopped when ||r|| <= tol ||v|| (FP64 throughout).
 *   B, C, eps, G : input pools (device), as for fef_half_transform and
 *                  fef_pair_energies.
 *   tol, maxit   : stopping rule (tol >= 0 finite, maxit >= 0; maxit = 0
 *                  gives the uncoupled energy of fef_pair_energies without
 *                  forming W, and sets flag bit 2).
 *   E2_pair      : [npair] out, in the caller's pair order (device).
 *   E2_total     : [1] out, FP64 sum over pairs in a fixed order (device).
 *   iters        : optional [npair] int32 out, CG iterations per pair.
 *   flags        : bit 1 for a non-finite energy, bit 2 when a pair stopped
 *                  at maxit without meeting tol.
 *   ws           : FEF_Q_COUPLED_WS_BYTES bytes (device).
 * One workgroup solves one pair; the search direction and its product live
 * in LDS when they fit and in the workspace otherwise.  Results are bitwise
 * reproducible for a given plan.  Plans with a fragment of 2048 or more
 * basis functions return FEF_E_UNSUPPORTED. */
fef_status fef_coupled_pair_energies(fef_plan plan, const double* B, const double* C,
                                     const double* eps, const double* G, double tol,
                                     int32_t maxit, double* E2_pair, double* E2_total,
                                     int32_t* iters, int32_t* flags, void* ws, size_t ws_bytes,
                                     void* stream);

/* Cross-fragment dressing of every fragment's one-body intermediates by the
 * dimer doubles (Sec. III, Eqs. MPij and MPab, their dimer-doubles terms;
 * the fragment singles vanish at this order, so Eq. MPia adds nothing):
 *     Hoo^x[i][i1] =  2 sum_y sum_{a, j, b} (ia|jb) t[i1 a, j b]
 *     Hvv^x[a][a1] = -2 sum_y sum_{i, j, b} (i a1|jb) t[i a, j b]
 * over every pair (x, y) of the list (the factor 2 sums the spin of the
 * other fragment's orbitals; no exchange between fragments), each pair
 * dressing both of its fragments.  t are the dimer doubles of
 * fef_coupled_pair_energies with the same tol and maxit: maxit = 0 gives
 * t = -(ia|jb) / D, the amplitudes of fef_pair_energies.
 *   B, C, eps, G : input pools (device).
 *   E2_pair, E2_total : as fef_coupled_pair_energies.
 *   Hoo : out pool, [nocc][nocc] per fragment (FEF_Q_HOO_ELEMS doubles).
 *   Hvv : out pool, [nvir][nvir] per fragment (FEF_Q_HVV_ELEMS doubles).
 *   ws  : FEF_Q_DRESSING_WS_BYTES bytes (device).
 * Each fragment's blocks are summed over its pairs in pair order, so the
 * result is bitwise reproducible for a given plan. */
fef_status fef_dimer_dressing(fef_plan plan, const double* B, const double* C, const double* eps,
                              const double* G, double tol, int32_t maxit, double* E2_pair,
                              double* E2_total, double* Hoo, double* Hvv, int32_t* flags,
                              void* ws, size_t ws_bytes, void* stream);

/* Monomer part of the second-order energy (Sec. II.B, Eq. EFEF2): for every
 * fragment the contraction of its two-body de-excitation operator with its
 * first-order doubles (Eq. EM2), the doubles solving Eq. monDoubles with the
 * two-body part of H0 dropped (as for the pair energies), summed over spin:
 *   E_M2^x = sum_{ijab} (ia|jb) [2 (ia|jb) - (ib|ja)]
 *                       / (eps_i + eps_j - eps_a - eps_b),
 * i, j occupied and a, b virtual orbitals of fragment x.  The integrals
 * inside a fragment are the factored tensor with the solvent class's own
 * coupling block at unit scale: (ia|jb) = sum_PQ B_ov[P][ia] G_{0,0}[P][Q]
 * B_ov[Q][jb] = sum_Q W[Q][ia] B_ov[Q][jb].
 *   Bov, W   : the dense FP64 outputs of fef_half_transform (device).
 *   eps      : orbital-energy pool (device).
 *   E_M2     : [nfrag] out, per fragment (device).
 *   E_M2_total : [1] out, FP64 sum over fragments in a fixed order (device).
 *   flags    : bit 1 is OR-ed in when a fragment energy is not finite.
 * Every fragment must be of class 0 (no other class has a coupling block
 * with itself): otherwise FEF_E_SHAPE.  nocc * nvir above 128 or P_0
 * above 80 returns FEF_E_UNSUPPORTED.  No workspace; bitwise
 * reproducible. */
fef_status fef_monomer_energies(fef_plan plan, const double* Bov, const double* W,
                                const double* eps, double* E_M2, double* E_M2_total,
                                int32_t* flags, void* stream);

/* ------------------------------------------------------------------------
 * Distant-pair surrogate.  A project addition: the paper has no learned
 * component.  It predicts E2_xy of Eq. ED2 for distant pairs from
 * rotation-invariant scalars of the Coulomb moments d^x = B^x : D^x (the
 * moments that carry the effective field of Eqs. wc and dp2e); the exact
 * pair kernel (fef_pair_energies_masked) evaluates every pair the surrogate
 * declines, so it is both the fallback and the reference for the error.
 *
 * Network: 17 -> 128 -> 128 -> 1 with SiLU after the two hidden layers.
 * Parameters of one member, packed in this order:
 *   W0[128][17], b0[128], W1[128][128], b1[128], W2[128], b2
 * (FEF_MLP_NPARAM numbers; members are FEF_MLP_STRIDE elements apart).
 * FP32 master copies (P, Adam moments M, V) and a BF16 copy W (uint16
 * bit patterns, round to nearest even) are kept; inference and training
 * both evaluate the network on W.
 * Statistics `stats` [FEF_MLP_NSTATS] floats: feature means [17], inverse
 * feature standard deviations [17], target mean, target standard deviation.
 * The network sees (x - mean) * inv and predicts (t - tmean) / tstd with
 * t = E2_xy R_xy^2 (R in bohr).
 * ------------------------------------------------------------------------ */
#define FEF_MLP_NIN 17
#define FEF_MLP_NHID 128
#define FEF_MLP_NPARAM 18945
#define FEF_MLP_STRIDE 18952
#define FEF_MLP_NSTATS 36

/* Q [4][P_0] (device out): eigenvectors of G_{0,0} for its four largest
 * eigenvalues, largest first (each column's sign is arbitrary).  FP64 Jacobi
 * on the device.  Workspace: FEF_Q_SURR_WS_BYTES. */
fef_status fef_coupling_modes(fef_plan plan, const double* G, double* Q, void* ws,
                              size_t ws_bytes, void* stream);

/* U [nfrag][8] (device out): for each class-0 fragment, with its moments
 * d_P = sum_{mu nu} B[P][mu][nu] D[mu][nu] (D as from fef_scf_step):
 * U = [d.G^k.d for k = 0..3, (Q_k.d)^2 for k = 0..3], G = G_{0,0}.  Other
 * classes get NaN (their pairs are always evaluated exactly).  Workspace:
 * FEF_Q_SURR_WS_BYTES. */
fef_status fef_fragment_invariants(fef_plan plan, const double* B, const double* G,
                                   const double* D, const double* Q, double* U, void* ws,
                                   size_t ws_bytes, void* stream);

/* X [n][17] floats (device out) for the pairs idx [n] (device int32; NULL =
 * pairs 0..n-1): [R_xy, U^x + U^y (8), U^x * U^y (8)] (symmetric in x, y).
 * With E2_pair and T non-NULL also the targets T[q] = E2_pair[idx[q]] R^2. */
fef_status fef_pair_features(fef_plan plan, const double* U, const double* E2_pair,
                             const int32_t* idx, int64_t n, float* X, float* T,
                             void* stream);

/* Per-column mean and standard deviation (inverse != 0: its inverse) of a
 * row-major [n][ncol] float matrix, FP64 two-pass, fixed summation order. */
fef_status fef_column_stats(int64_t n, int32_t ncol, int32_t inverse, const float* A,
                            float* mean, float* sdev, void* stream);

/* W = BF16(P) for nmember members (device pointers, FEF_MLP_STRIDE apart). */
fef_status fef_mlp_pack(int32_t nmember, const float* P, uint16_t* W, void* stream);

/* Y [nmember][n] (device out): standardised predictions of every member for
 * the rows of X [n][17] (raw features).  MFMA BF16, FP32 accumulation. */
fef_status fef_mlp_forward(int32_t nmember, int64_t n, const float* X, const float* stats,
                           const uint16_t* W, float* Y, void* stream);

/* One training step of every member on its own mini-batch: rows
 * idx [nmember][nb] (device int32) of X [*][17] with targets T [*] (raw).
 * Mean squared error of the standardised targets; gradients in FP32 on the
 * BF16 weights W, summed over the batch in a fixed order; Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected step `step` >= 1, rate lr) on the
 * FP32 masters P, M, V, then W = BF16(P).  step = 0 computes gradients and
 * loss only.  loss [nmember] and grad [nmember][FEF_MLP_STRIDE] (device,
 * nullable) receive the batch loss and the gradient.  Workspace bytes from
 * fef_mlp_train_ws_bytes. */
fef_status fef_mlp_train_step(int32_t nmember, const float* X, const float* T,
                              const int32_t* idx, int32_t nb, const float* stats, float* P,
                              float* M, float* V, uint16_t* W, int32_t step, float lr,
                              float* loss, float* grad, void* ws, size_t ws_bytes,
                              void* stream);
fef_status fef_mlp_train_ws_bytes(int32_t nmember, int32_t nb, int64_t* out);

/* Surrogate selection over every pair of the plan: the ensemble (nmember
 * members, features from U) predicts E2_xy = (mean * tstd + tmean) / R^2;
 * a pair is sent to the exact kernel (select = 1, E2_pair = 0) when
 * R < r_exact (bohr), when the members' spread (max - min) in Eh exceeds
 * `threshold`, when a fragment is outside class 0 or the prediction is not
 * finite; otherwise select = 0 and E2_pair holds the prediction.  Follow with
 * fef_pair_energies_masked to complete E2_pair and E2_total. */
fef_status fef_surrogate_select(fef_plan plan, const double* U, int32_t nmember,
                                const float* stats, const uint16_t* W, double r_exact,
                                double threshold, double* E2_pair, int32_t* select,
                                void* stream);

const char* fef_status_string(fef_status s);

#ifdef __cplusplus
}
#endif
#endif /* FEF_H */
