// Graph capture of a whole FEF pass and the pair-kernel tile autotuner.
#include <algorithm>
#include <cfloat>
#include <new>
#include <vector>

#include "fef_internal.h"

struct fef_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  fef_plan plan = nullptr;  // its tile tables of mode `prec` are baked in
  int prec = 0;
};

namespace fef {

// Start of a replay, one kernel: the flags cleared and, with C0 given, the
// generated orbitals and orbital energies copied back (one element per
// thread, C then eps).
__global__ void reset_kernel(int32_t* __restrict__ flags, const double* __restrict__ C0,
                             double* __restrict__ C, int64_t nC, const double* __restrict__ eps0,
                             double* __restrict__ eps, int64_t nEps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *flags = 0;
  if (!C0) return;
  if (i < nC)
    C[i] = C0[i];
  else if (i < nC + nEps)
    eps[i - nC] = eps0[i - nC];
}

}  // namespace fef

using namespace fef;

extern "C" {

fef_status fef_graph_create(fef_plan p, const fef_pass_args* a, int32_t niter, fef_prec prec,
                            fef_graph* out) {
  if (!p || !a || !out || niter < 0) return FEF_E_ARG;
  *out = nullptr;
  if (prec < 0 || prec >= FEF_NPREC) return FEF_E_PREC;
  if ((a->C0 == nullptr) != (a->eps0 == nullptr)) return FEF_E_ARG;
  if (!a->ws || !a->ops || !a->E2_total || !a->flags || !a->dD_max) return FEF_E_ARG;
  int64_t need = std::max(std::max(scf_ws_bytes(*p), half_ws_bytes(*p, prec)),
                          pair_ws_bytes(*p, prec));
  if ((int64_t)a->ws_bytes < need) return FEF_E_WORKSPACE;
  fef_graph_s* g = new (std::nothrow) fef_graph_s();
  if (!g) return FEF_E_UNSUPPORTED;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    delete g;
    return FEF_E_HIP;
  }
  fef_status status = FEF_OK;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) status = FEF_E_HIP;
  if (status == FEF_OK) {
    // each replay reports its own flags (a fill kernel, not a memset node)
    {
      const int64_t n = a->C0 ? p->nC + p->nEps : 0;
      const unsigned nb = (unsigned)std::max<int64_t>(1, (n + 255) / 256);
      hipLaunchKernelGGL(reset_kernel, dim3(nb), dim3(256), 0, st, a->flags, a->C0, a->C, p->nC,
                         a->eps0, a->eps, p->nEps);
    }
    // with a packed pool the first step packs B on the way (its moments
    // kernel reads B and writes Bp), the later steps read Bp; with small
    // fragments and a D pool each step also carries its density to the next
    const bool carry = a->Bp && a->D && density_carry_ok(*p);
    for (int it = 0; it < niter && status == FEF_OK; ++it)
      status = !a->Bp ? fef_scf_step(p, a->B, a->G, a->F0, a->htilde, a->C, a->eps, a->D,
                                     a->dD_max, a->flags, a->ws, a->ws_bytes, st)
               : carry ? scf_step_carry(p, it == 0 ? a->B : nullptr, a->Bp, a->G, a->F0,
                                        a->htilde, a->C, a->eps, a->D, a->dD_max, a->flags,
                                        a->ws, a->ws_bytes, st, it, niter)
               : it == 0 ? scf_step_packing(p, a->B, a->Bp, a->G, a->F0, a->htilde, a->C, a->eps,
                                            a->D, a->dD_max, a->flags, a->ws, a->ws_bytes, st)
                         : fef_scf_step_packed(p, a->Bp, a->G, a->F0, a->htilde, a->C, a->eps,
                                               a->D, a->dD_max, a->flags, a->ws, a->ws_bytes, st);
    if (status == FEF_OK)
      status = fef_half_transform(p, a->B, a->C, a->G, nullptr, nullptr, a->ops, prec, a->ws,
                                  a->ws_bytes, st);
    if (status == FEF_OK)
      status = fef_pair_energies(p, a->ops, a->eps, prec, a->E2_pair, a->E2_total, a->flags,
                                 a->ws, a->ws_bytes, st);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (status == FEF_OK && e != hipSuccess) status = FEF_E_HIP;
    g->graph = graph;
    if (status == FEF_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess)
      status = FEF_E_HIP;
  }
  (void)hipStreamDestroy(st);
  if (status != FEF_OK) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return status;
  }
  g->plan = p;
  g->prec = (int)prec;
  ++p->graphs_live[prec];
  *out = g;
  return FEF_OK;
}

fef_status fef_graph_launch(fef_graph g, void* stream) {
  if (!g || !g->exec) return FEF_E_ARG;
  return hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? FEF_OK
                                                                                 : FEF_E_HIP;
}

fef_status fef_graph_destroy(fef_graph g) {
  if (!g) return FEF_E_ARG;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->plan) --g->plan->graphs_live[g->prec];
  delete g;
  return FEF_OK;
}

fef_status fef_autotune(fef_plan p, const void* ops, const double* eps, fef_prec prec, void* ws,
                        size_t ws_bytes, int32_t reps, void* stream, int32_t* best_xb,
                        int32_t* best_yc, double* best_us) {
  if (!p || !ops || !eps || !best_xb || !best_yc || !best_us || reps < 1) return FEF_E_ARG;
  if (prec < 0 || prec >= FEF_NPREC) return FEF_E_PREC;
  if ((int64_t)ws_bytes < pair_ws_bytes(*p, prec) || !ws) return FEF_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool plain = prec == FEF_F64 || prec == FEF_F32;
  std::vector<std::pair<int, int>> cand;
  const int ycs[] = {8, 16, 32, 64};
  if (plain) {
    for (int xb : {1, 2})
      for (int yc : ycs) cand.push_back({xb, yc});
  } else {
    // three-term operands keep 84 registers of x resident: only the
    // ping-pong kernel (xb = 2) holds them without spilling
    for (int xb : {2, 4})
      if (xb == 2 || prec != FEF_BF16X3)
        for (int yc : ycs) cand.push_back({xb, yc});
  }
  // the candidates write their results into library-owned scratch, so the
  // caller's E2_pair / E2_total keep their contents
  double* e2 = nullptr;
  double* tot = nullptr;
  int32_t* flags = nullptr;
  if (hipMalloc(&e2, std::max<int64_t>(p->npair, 1) * sizeof(double)) != hipSuccess ||
      hipMalloc(&tot, sizeof(double)) != hipSuccess || hipMalloc(&flags, sizeof(int32_t)) != hipSuccess) {
    if (e2) (void)hipFree(e2);
    if (tot) (void)hipFree(tot);
    return FEF_E_HIP;
  }
  hipEvent_t t0, t1;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  double best = DBL_MAX;
  int bxb = p->tiles[prec].xb, byc = p->tiles[prec].yc;
  fef_status status = FEF_OK;
  for (const auto& c : cand) {
    if (build_tiles(*p, prec, c.first, c.second) != hipSuccess) { status = FEF_E_HIP; break; }
    if (launch_pair_energies(*p, ops, eps, prec, nullptr, e2, tot, flags, ws, st) != hipSuccess) {
      status = FEF_E_HIP;
      break;
    }
    (void)hipEventRecord(t0, st);
    for (int r = 0; r < reps; ++r) (void)launch_pair_energies(*p, ops, eps, prec, nullptr, e2, tot, flags, ws, st);
    (void)hipEventRecord(t1, st);
    (void)hipEventSynchronize(t1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    const double us = 1e3 * ms / reps;
    if (us < best) { best = us; bxb = c.first; byc = c.second; }
  }
  if (status == FEF_OK && build_tiles(*p, prec, bxb, byc) != hipSuccess) status = FEF_E_HIP;
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  (void)hipFree(e2);
  (void)hipFree(tot);
  (void)hipFree(flags);
  if (status != FEF_OK) return status;
  *best_xb = bxb;
  *best_yc = byc;
  *best_us = best;
  return FEF_OK;
}

}  // extern "C"
