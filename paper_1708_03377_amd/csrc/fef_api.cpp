// Host side of the C ABI: argument checks, plan construction (fragment
// offsets, oriented pairs, work items, neighbour lists) and dispatch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fef_internal.h"

using namespace fef;

namespace {

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return hipSuccess;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

void free_plan(fef_plan_s* p) {
  if (!p) return;
  for (auto& t : p->tiles) free_tiles(t);
  for (auto& t : p->retired_tiles) free_tiles(t);
  void* ptrs[] = {p->d_frag, p->d_pair, p->d_slot_pair, p->d_ht, p->d_ht_fused, p->d_ht_generic,
                  p->d_off_G, p->d_naux_cls_off,
                  p->d_nbr_ptr, p->d_nbr_idx, p->d_nbr_s, p->d_eig_small,
                  p->d_eig_mid, p->d_eig_large, p->d_gfrag, p->d_glist, p->d_off_Bp,
                  p->d_off_tri, p->d_chunk_C, p->d_chunk_Bp, p->d_cp_list, p->d_rec_off,
                  p->d_off_oo, p->d_off_vv, p->d_inc_ptr, p->d_inc_base};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (hipEvent_t& e : p->stage_ev)
    if (e) (void)hipEventDestroy(e);
  delete p;
}

OpsGeom geom_of(int prec, int P0) {
  switch (prec) {
    case FEF_F64: return {8, (int)round_up(P0, 4), 0, 1};
    case FEF_F32: return {4, (int)round_up(P0, 4), 0, 1};
    default: {
      // contraction length the MFMA chains run over
      const int pw = (int)round_up(P0, 8), nt = split_nterm(prec);
      int kp = 0;
      if (nt == 2)
        kp = (int)round_up(3 * pw, 32);
      else
        for (int l = 0; l < nt; ++l) kp += 32 * split_chain(l, pw);
      return {2, kp, pw, nt};
    }
  }
}

// operand block bytes of one fragment (one role)
int64_t operand_bytes(const OpsGeom& g, int prec, int64_t ld) {
  if (prec == FEF_F64 || prec == FEF_F32) return round_up((int64_t)g.kpad * ld * g.elem_bytes, 256);
  return round_up(ld * (g.nterm * g.pw + 8) * g.elem_bytes, 256);
}

// default pair-kernel tiling per mode: (x units per block, entries per item)
void default_tiles(int prec, int& xb, int& yc) {
  xb = (prec == FEF_F64 || prec == FEF_F32) ? 1 : prec == FEF_BF16X3 ? 2 : 4;
  yc = 16;
}

bool valid_prec(int prec) { return prec >= 0 && prec < FEF_NPREC; }

}  // namespace

namespace fef {

int64_t half_ws_bytes(const fef_plan_s& p, fef_prec) {
  return (p.nBov + p.nW) * (int64_t)sizeof(double) + 256;
}
// partial sums [nslot], the persistent queue head, per-fragment gaps [sum ld],
// 256 block sums of the total
int64_t pair_ws_bytes(const fef_plan_s& p, fef_prec) {
  return round_up(std::max<int64_t>(p.nslot, 1) * (int64_t)sizeof(double), 256) + 256 +
         round_up(round_up(std::max<int64_t>(p.nGap, 1), 32) * (int64_t)sizeof(double), 256) +
         256 * (int64_t)sizeof(double);
}
int64_t naux_total(const fef_plan_s& p) {
  int64_t t = 0;
  for (const auto& f : p.frag) t += f.naux;
  return t;
}
int64_t field_ws_bytes(const fef_plan_s& p) {
  return round_up(2 * std::max<int64_t>(naux_total(p), 1) * (int64_t)sizeof(double), 256);
}
// pair workspace, then the masked copies of the entries and work items
int64_t masked_ws_bytes(const fef_plan_s& p, fef_prec prec) {
  const TileSet& t = p.tiles[prec];
  return pair_ws_bytes(p, prec) +
         round_up(std::max<int64_t>(t.nentries, 1) * (int64_t)sizeof(Entry), 256) +
         round_up(std::max<int64_t>(t.nitems, 1) * (int64_t)sizeof(WorkItem), 256);
}
// coupling modes: V, eps, Dnew, Dold [P0^2 or P0], max, flags, two Jacobi
// slots; invariants: the moments [sum P_c]
int64_t surr_ws_bytes(const fef_plan_s& p) {
  const int64_t n = p.P0;
  const int64_t modes = (3 * n * n + n + 2) * (int64_t)sizeof(double) + 256 +
                        2 * (n + 1) * (n + 1) * (int64_t)sizeof(double) + 4 * 256;
  const int64_t inv = round_up(std::max<int64_t>(naux_total(p), 1) * (int64_t)sizeof(double), 256);
  return std::max(modes, inv);
}
int64_t scf_ws_bytes(const fef_plan_s& p) {
  const int64_t large = (int64_t)p.eig_large.size() * eig_large_slot(p.eig_large_max_nbf);
  // Dold, F, Dnew [nC] each, the eigensolver slots, the weighted packed
  // density [nTri]
  int64_t n = 3 * std::max<int64_t>(p.nC, 1) + large + std::max<int64_t>(p.nTri, 1);
  return field_ws_bytes(p) + round_up(n * (int64_t)sizeof(double), 256);
}

}  // namespace fef

extern "C" {

const char* fef_status_string(fef_status s) {
  switch (s) {
    case FEF_OK: return "ok";
    case FEF_E_ARG: return "invalid argument";
    case FEF_E_SHAPE: return "inconsistent sizes or unsupported pair";
    case FEF_E_PREC: return "unknown precision mode";
    case FEF_E_WORKSPACE: return "workspace too small";
    case FEF_E_HIP: return "HIP runtime error";
    case FEF_E_UNSUPPORTED: return "unsupported request";
    case FEF_E_IO: return "file could not be written";
    default: return "unknown status";
  }
}

fef_status fef_plan_create(const fef_system_desc* d, fef_plan* out) {
  if (!d || !out) return FEF_E_ARG;
  *out = nullptr;
  if (d->nfrag < 0 || d->nclass < 1 || d->npair < 0) return FEF_E_ARG;
  if (d->nfrag > 0 && (!d->nbf || !d->nocc || !d->cls)) return FEF_E_ARG;
  if (!d->naux) return FEF_E_ARG;
  if (d->npair > 0 && (!d->pair_x || !d->pair_y || !d->pair_s)) return FEF_E_ARG;
  if (d->npair > (int64_t)INT32_MAX) return FEF_E_UNSUPPORTED;
  for (int c = 0; c < d->nclass; ++c)
    if (d->naux[c] < 1) return FEF_E_SHAPE;
  if (d->naux[0] > 80) return FEF_E_UNSUPPORTED;  // pair-kernel LDS / register staging bound
  for (int f = 0; f < d->nfrag; ++f) {
    if (d->nbf[f] < 1 || d->nocc[f] < 0 || d->nocc[f] > d->nbf[f]) return FEF_E_SHAPE;
    if (d->cls[f] < 0 || d->cls[f] >= d->nclass) return FEF_E_SHAPE;
    // element indices inside one fragment's coefficient slab are 32-bit
    if ((int64_t)d->naux[d->cls[f]] * d->nbf[f] * d->nbf[f] > (int64_t)INT32_MAX)
      return FEF_E_UNSUPPORTED;
  }

  fef_plan_s* p = new (std::nothrow) fef_plan_s();
  if (!p) return FEF_E_UNSUPPORTED;
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return FEF_E_HIP; }
  p->nfrag = d->nfrag;
  p->nclass = d->nclass;
  p->P0 = d->naux[0];
  p->naux_cls.assign(d->naux, d->naux + d->nclass);
  p->off_G.resize(d->nclass + 1);
  p->off_G[0] = 0;
  for (int c = 0; c < d->nclass; ++c)
    p->off_G[c + 1] = p->off_G[c] + (int64_t)d->naux[c] * p->P0;
  p->nG = p->off_G[d->nclass];
  p->naux_cls_off.assign(d->nclass + 1, 0);
  for (int c = 0; c < d->nclass; ++c) p->naux_cls_off[c + 1] = p->naux_cls_off[c] + d->naux[c];
  for (int k = 0; k < FEF_NPREC; ++k) p->geom[k] = geom_of(k, p->P0);
  (void)compute_units();

  // ---- fragment table -----------------------------------------------------
  p->frag.resize(d->nfrag);
  int64_t oB = 0, oC = 0, oE = 0, oBov = 0, oW = 0, oAux = 0, oGap = 0;
  int64_t oOps[FEF_NPREC];
  // the operand pool starts with two scale factors per fragment (left, right)
  p->ops_header = round_up(16 * (int64_t)std::max(d->nfrag, 1), 256);
  for (int k = 0; k < FEF_NPREC; ++k) oOps[k] = p->ops_header;
  for (int f = 0; f < d->nfrag; ++f) {
    FragInfo& fi = p->frag[f];
    std::memset(&fi, 0, sizeof(fi));
    fi.nbf = d->nbf[f];
    fi.nocc = d->nocc[f];
    fi.nvir = fi.nbf - fi.nocc;
    fi.ov = fi.nocc * fi.nvir;
    fi.cls = d->cls[f];
    fi.naux = d->naux[fi.cls];
    fi.ntile = (int32_t)((fi.ov + kTile - 1) / kTile);
    fi.ld = (int64_t)fi.ntile * kTile;
    fi.off_B = oB;  oB += (int64_t)fi.naux * fi.nbf * fi.nbf;
    fi.off_C = oC;  oC += (int64_t)fi.nbf * fi.nbf;
    fi.off_eps = oE; oE += fi.nbf;
    fi.off_bov = oBov; oBov += (int64_t)fi.naux * fi.ov;
    fi.off_w = oW;  oW += (int64_t)p->P0 * fi.ov;
    fi.off_aux = oAux; oAux += fi.naux;
    fi.off_gap = oGap; oGap += fi.ld;
    for (int k = 0; k < FEF_NPREC; ++k) {
      const int64_t blk = operand_bytes(p->geom[k], k, fi.ld);
      fi.off_L[k] = oOps[k];
      oOps[k] += blk;
      if (fi.cls == 0) { fi.off_R[k] = oOps[k]; oOps[k] += blk; }
      else fi.off_R[k] = -1;
    }
    p->max_nbf = std::max(p->max_nbf, fi.nbf);
    p->max_naux = std::max(p->max_naux, fi.naux);
    p->max_ov = std::max(p->max_ov, fi.ov);
    p->max_on = std::max<int64_t>(p->max_on, (int64_t)fi.nocc * fi.nbf);
  }
  p->nB = oB; p->nC = oC; p->nEps = oE; p->nBov = oBov; p->nW = oW; p->nGap = oGap;
  for (int k = 0; k < FEF_NPREC; ++k) p->ops_bytes[k] = oOps[k];

  // ---- pairs, neighbours ---------------------------------------------------
  p->npair = d->npair;
  p->pairs.resize(d->npair);
  std::vector<std::vector<std::pair<int32_t, double>>> nbr(d->nfrag);
  for (int64_t k = 0; k < d->npair; ++k) {
    const int32_t x = d->pair_x[k], y = d->pair_y[k];
    const double s = d->pair_s[k];
    if (x < 0 || y < 0 || x >= d->nfrag || y >= d->nfrag || x == y || !std::isfinite(s)) {
      free_plan(p);
      return FEF_E_SHAPE;
    }
    if (p->frag[x].cls != 0 && p->frag[y].cls != 0) { free_plan(p); return FEF_E_SHAPE; }
    PairInfo& pi = p->pairs[k];
    std::memset(&pi, 0, sizeof(pi));
    pi.x = x; pi.y = y; pi.s = s;
    nbr[x].push_back({y, s});
    nbr[y].push_back({x, s});
  }
  order_and_orient(*p);
  if (p->nslot > (int64_t)INT32_MAX) { free_plan(p); return FEF_E_UNSUPPORTED; }
  std::vector<int32_t> slot_pair(p->nslot);
  for (int64_t k = 0; k < d->npair; ++k) {
    const PairInfo& pi = p->pairs[k];
    for (int t = 0; t < pi.ntx * pi.nty; ++t) slot_pair[pi.slot_first + t] = (int32_t)k;
  }
  std::vector<int32_t> nptr(d->nfrag + 1, 0), nidx;
  std::vector<double> ns;
  for (int f = 0; f < d->nfrag; ++f) {
    auto& v = nbr[f];
    std::sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    nptr[f + 1] = nptr[f] + (int32_t)v.size();
    for (auto& e : v) { nidx.push_back(e.first); ns.push_back(e.second); }
  }
  p->nbr_total = (int64_t)nidx.size();

  // ---- half-transform tasks and eigen-solver groups --------------------------
  // small fragments take the fused half transform, the rest the generic chain
  std::vector<HtTask> ht;
  int64_t mx_nn = 1, mx_on = 1, mx_pov = 1;
  for (int f = 0; f < d->nfrag; ++f) {
    const FragInfo& fi = p->frag[f];
    if (fi.ov == 0) continue;
    if (fi.nbf <= 32 && fi.ntile == 1 && fi.naux <= 80) {
      p->ht_fused.push_back(f);
      p->max_naux_small = std::max(p->max_naux_small, fi.naux);
      mx_nn = std::max<int64_t>(mx_nn, (int64_t)fi.nbf * fi.nbf);
      mx_on = std::max<int64_t>(mx_on, (int64_t)fi.nocc * fi.nbf);
      mx_pov = std::max<int64_t>(mx_pov, (int64_t)fi.naux * fi.ov);
      continue;
    }
    p->ht_generic.push_back(f);
    // factor slices per task: large fragments one slice each (parallelism)
    const int per = fi.nbf > 64 ? 1 : 8;
    for (int p0 = 0; p0 < fi.naux; p0 += per) ht.push_back({f, p0, std::min(per, fi.naux - p0), 0});
  }
  p->ht_ntasks = (int64_t)ht.size();
  p->fuse_lds[0] = (int32_t)mx_nn;   // largest nbf^2 among small fragments
  p->fuse_lds[1] = (int32_t)mx_on;   // largest nocc * nbf
  p->fuse_lds[2] = (int32_t)mx_pov;  // largest P_c * ov
  for (int f = 0; f < d->nfrag; ++f) {
    const int n = p->frag[f].nbf;
    if (n <= 32) p->eig_small.push_back(f);
    else if (n <= 48) p->eig_mid.push_back(f);
    else { p->eig_large.push_back(f); p->eig_large_max_nbf = std::max(p->eig_large_max_nbf, n); }
  }
  {  // group the n <= 32 fragments by register-kernel size class (8, 16, 24, 32)
    auto cls_of = [&](int f) { const int n = p->frag[f].nbf; return n <= 8 ? 0 : n <= 16 ? 1 : n <= 24 ? 2 : 3; };
    std::stable_sort(p->eig_small.begin(), p->eig_small.end(),
                     [&](int a, int b) { return cls_of(a) < cls_of(b); });
    int32_t cnt[4] = {0, 0, 0, 0};
    for (int f : p->eig_small) ++cnt[cls_of(f)];
    p->eig_w_off[0] = 0;
    for (int c = 0; c < 4; ++c) p->eig_w_off[c + 1] = p->eig_w_off[c] + cnt[c];
  }

  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload(&p->d_frag, p->frag);
  if (e == hipSuccess) e = upload(&p->d_pair, p->pairs);
  if (e == hipSuccess) e = upload(&p->d_slot_pair, slot_pair);
  for (int k = 0; k < FEF_NPREC && e == hipSuccess; ++k) {
    int xb, yc;
    default_tiles(k, xb, yc);
    e = build_tiles(*p, k, xb, yc);
  }
  if (e == hipSuccess) e = upload(&p->d_ht, ht);
  if (e == hipSuccess) e = upload(&p->d_ht_fused, p->ht_fused);
  if (e == hipSuccess) e = upload(&p->d_ht_generic, p->ht_generic);
  if (e == hipSuccess) e = upload(&p->d_off_G, p->off_G);
  if (e == hipSuccess) e = upload(&p->d_naux_cls_off, p->naux_cls_off);
  if (e == hipSuccess) e = upload(&p->d_nbr_ptr, nptr);
  if (e == hipSuccess) e = upload(&p->d_nbr_idx, nidx);
  if (e == hipSuccess) e = upload(&p->d_nbr_s, ns);
  if (e == hipSuccess) e = upload(&p->d_eig_small, p->eig_small);
  if (e == hipSuccess) e = upload(&p->d_eig_mid, p->eig_mid);
  if (e == hipSuccess) e = upload(&p->d_eig_large, p->eig_large);
  if (e == hipSuccess) {
    FragInfo g;
    std::memset(&g, 0, sizeof(g));
    g.nbf = p->P0;
    g.naux = 1;
    e = upload(&p->d_gfrag, std::vector<FragInfo>{g});
  }
  if (e == hipSuccess) e = upload(&p->d_glist, std::vector<int32_t>{0});
  if (e == hipSuccess) e = coupled_setup(*p);
  if (e == hipSuccess) {
    // nfrag + 1 entries: the last is the pool size
    std::vector<int64_t> offp(d->nfrag + 1, 0);
    int64_t o = 0;
    for (int f = 0; f < d->nfrag; ++f) {
      offp[f] = o;
      o += (int64_t)p->frag[f].naux * p->frag[f].nbf * (p->frag[f].nbf + 1) / 2;
    }
    offp[d->nfrag] = o;
    p->nBp = o;
    e = upload(&p->d_off_Bp, offp);
  }
  if (e == hipSuccess) {
    std::vector<int64_t> offt(d->nfrag + 1, 0);
    int64_t o = 0;
    for (int f = 0; f < d->nfrag; ++f) {
      offt[f] = o;
      o += (int64_t)p->frag[f].nbf * (p->frag[f].nbf + 1) / 2;
    }
    offt[d->nfrag] = o;
    p->nTri = o;
    e = upload(&p->d_off_tri, offt);
  }
  if (e == hipSuccess) {
    // chunks of the density pool (nbf^2 per fragment) and of the packed pool
    // (naux nbf (nbf + 1) / 2 per fragment), cut at fragment boundaries
    std::vector<Chunk> cc, cb;
    int64_t oc = 0, ob = 0;
    for (int f = 0; f < d->nfrag; ++f) {
      const FragInfo& fi = p->frag[f];
      const int64_t nc = (int64_t)fi.nbf * fi.nbf;
      const int64_t nb = (int64_t)fi.naux * fi.nbf * (fi.nbf + 1) / 2;
      for (int64_t s = 0; s < nc; s += kDensityChunk)
        cc.push_back({oc + s, oc + std::min<int64_t>(s + kDensityChunk, nc), f, 0});
      for (int64_t s = 0; s < nb; s += kPackChunk)
        cb.push_back({ob + s, ob + std::min<int64_t>(s + kPackChunk, nb), f, 0});
      oc += nc;
      ob += nb;
    }
    p->n_chunk_C = (int64_t)cc.size();
    p->n_chunk_Bp = (int64_t)cb.size();
    if (!cc.empty()) e = upload(&p->d_chunk_C, cc);
    if (e == hipSuccess && !cb.empty()) e = upload(&p->d_chunk_Bp, cb);
  }
  if (e != hipSuccess) { free_plan(p); return FEF_E_HIP; }
  // set-up of fef_pair_energies_noalloc on this device (an address lookup;
  // on failure that entry point retries and reports it)
  (void)noalloc_setup(p->device);
  *out = p;
  return FEF_OK;
}

fef_status fef_plan_destroy(fef_plan p) {
  if (!p) return FEF_E_ARG;
  free_plan(p);
  return FEF_OK;
}

fef_status fef_plan_query(fef_plan p, fef_query what, fef_prec prec, int64_t* out) {
  if (!p || !out) return FEF_E_ARG;
  const bool needs_prec = what == FEF_Q_OPS_BYTES || what == FEF_Q_HALF_WS_BYTES ||
                          what == FEF_Q_PAIR_WS_BYTES || what == FEF_Q_NITEMS ||
                          what == FEF_Q_NENTRIES || what == FEF_Q_MASKED_WS_BYTES;
  if (needs_prec && !valid_prec(prec)) return FEF_E_PREC;
  switch (what) {
    case FEF_Q_OPS_BYTES: *out = p->ops_bytes[prec]; break;
    case FEF_Q_HALF_WS_BYTES: *out = half_ws_bytes(*p, prec); break;
    case FEF_Q_PAIR_WS_BYTES: *out = pair_ws_bytes(*p, prec); break;
    case FEF_Q_FIELD_WS_BYTES: *out = field_ws_bytes(*p); break;
    case FEF_Q_SCF_WS_BYTES: *out = scf_ws_bytes(*p); break;
    case FEF_Q_BOV_ELEMS: *out = p->nBov; break;
    case FEF_Q_W_ELEMS: *out = p->nW; break;
    case FEF_Q_NITEMS: *out = p->tiles[prec].nitems; break;
    case FEF_Q_B_ELEMS: *out = p->nB; break;
    case FEF_Q_C_ELEMS: *out = p->nC; break;
    case FEF_Q_EPS_ELEMS: *out = p->nEps; break;
    case FEF_Q_G_ELEMS: *out = p->nG; break;
    case FEF_Q_NPAIR: *out = p->npair; break;
    case FEF_Q_NSLOT: *out = p->nslot; break;
    case FEF_Q_NENTRIES: *out = p->tiles[prec].nentries; break;
    case FEF_Q_MASKED_WS_BYTES: *out = masked_ws_bytes(*p, prec); break;
    case FEF_Q_SURR_WS_BYTES: *out = surr_ws_bytes(*p); break;
    case FEF_Q_BPACK_ELEMS: *out = p->nBp; break;
    case FEF_Q_COUPLED_WS_BYTES: *out = coupled_ws_bytes(*p); break;
    case FEF_Q_DRESSING_WS_BYTES: *out = dressing_ws_bytes(*p); break;
    case FEF_Q_HOO_ELEMS: *out = p->n_oo; break;
    case FEF_Q_HVV_ELEMS: *out = p->n_vv; break;
    default: return FEF_E_ARG;
  }
  return FEF_OK;
}

static fef_status hip_status(hipError_t e) { return e == hipSuccess ? FEF_OK : FEF_E_HIP; }

fef_status fef_plan_set_tiles(fef_plan p, fef_prec prec, int32_t xb, int32_t yc) {
  if (!p) return FEF_E_ARG;
  if (!valid_prec(prec)) return FEF_E_PREC;
  const bool plain = prec == FEF_F64 || prec == FEF_F32;
  if (plain ? (xb != 1 && xb != 2) : (xb != 2 && xb != 4)) return FEF_E_UNSUPPORTED;
  if (yc < 1 || yc > 4096) return FEF_E_ARG;
  return hip_status(build_tiles(*p, prec, xb, yc));
}

fef_status fef_plan_get_tiles(fef_plan p, fef_prec prec, int32_t* xb, int32_t* yc) {
  if (!p || !xb || !yc) return FEF_E_ARG;
  if (!valid_prec(prec)) return FEF_E_PREC;
  *xb = p->tiles[prec].xb;
  *yc = p->tiles[prec].yc;
  return FEF_OK;
}

fef_status fef_half_transform(fef_plan p, const double* B, const double* C, const double* G,
                              double* Bov, double* W, void* ops, fef_prec prec, void* ws,
                              size_t ws_bytes, void* stream) {
  if (!p) return FEF_E_ARG;
  if (!valid_prec(prec)) return FEF_E_PREC;
  if (p->nfrag > 0 && (!B || !C || !G || !ops)) return FEF_E_ARG;
  if ((int64_t)ws_bytes < half_ws_bytes(*p, prec) || (!ws && ws_bytes)) return FEF_E_WORKSPACE;
  if (p->nfrag == 0) return FEF_OK;
  if ((Bov == nullptr) != (W == nullptr)) return FEF_E_ARG;
  double* bov = Bov ? Bov : static_cast<double*>(ws);
  double* w = W ? W : static_cast<double*>(ws) + p->nBov;
  return hip_status(launch_half_transform(*p, B, C, G, bov, w, ops, prec,
                                          static_cast<hipStream_t>(stream), Bov != nullptr));
}

fef_status fef_pair_energies(fef_plan p, const void* ops, const double* eps, fef_prec prec,
                             double* E2_pair, double* E2_total, int32_t* flags, void* ws,
                             size_t ws_bytes, void* stream) {
  if (!p) return FEF_E_ARG;
  if (!valid_prec(prec)) return FEF_E_PREC;
  if (!E2_total || !flags) return FEF_E_ARG;
  if (p->npair > 0 && (!ops || !eps || !E2_pair)) return FEF_E_ARG;
  if ((int64_t)ws_bytes < pair_ws_bytes(*p, prec) || !ws) return FEF_E_WORKSPACE;
  return hip_status(launch_pair_energies(*p, ops, eps, prec, nullptr, E2_pair, E2_total, flags, ws,
                                         static_cast<hipStream_t>(stream)));
}

fef_status fef_coulomb_field(fef_plan p, const double* B, const double* G, const double* D,
                             double* J, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return FEF_E_ARG;
  if (p->nfrag > 0 && (!B || !G || !D || !J)) return FEF_E_ARG;
  if ((int64_t)ws_bytes < field_ws_bytes(*p) || !ws) return FEF_E_WORKSPACE;
  if (p->nfrag == 0) return FEF_OK;
  double* wd = static_cast<double*>(ws);
  double* wphi = wd + naux_total(*p);
  return hip_status(launch_field(*p, B, G, D, nullptr, nullptr, J, wd, wphi,
                                 static_cast<hipStream_t>(stream)));
}

// Workspace of an SCF step (doubles): field scratch, then Dold [nC], F [nC],
// a spare density pool [nC] (Dnew when the caller passes no D), the
// eigensolver slots, the weighted packed density Dw.
struct ScfWs {
  double *wd, *wphi, *Dold, *F, *Dspare, *eigws, *Dw;
};
static ScfWs scf_ws(const fef_plan_s& p, void* ws) {
  ScfWs w;
  w.wd = static_cast<double*>(ws);
  w.wphi = w.wd + naux_total(p);
  w.Dold = static_cast<double*>(ws) + field_ws_bytes(p) / (int64_t)sizeof(double);
  w.F = w.Dold + std::max<int64_t>(p.nC, 1);
  w.Dspare = w.F + std::max<int64_t>(p.nC, 1);
  w.eigws = w.F + 2 * std::max<int64_t>(p.nC, 1);
  w.Dw = w.eigws + (int64_t)p.eig_large.size() * eig_large_slot(p.eig_large_max_nbf);
  return w;
}

// One SCF step.  B_pack / Bp_out: the moments kernel packs B into Bp on the
// way.  carry_out: the eigensolver also writes Dw of its orbitals.  Dprev
// non-null: D and Dw of the current orbitals are already in Dprev and the
// workspace (the previous step carried them), no density kernel.  Dout
// non-null: the new density goes there (never the same pool as Dprev).
static fef_status scf_step_impl(fef_plan p, const double* B, const double* Bp, const double* G,
                                const double* F0, const double* htilde, double* C, double* eps,
                                double* D, double* dD_max, int32_t* flags, void* ws,
                                size_t ws_bytes, void* stream, const double* B_pack = nullptr,
                                double* Bp_out = nullptr, bool carry_out = false,
                                const double* Dprev = nullptr, double* Dout = nullptr,
                                bool moments_in = false, bool moments_out = false) {
  if (!p) return FEF_E_ARG;
  if (!dD_max || !flags) return FEF_E_ARG;
  if (p->nfrag > 0 && (!(B || Bp) || !G || !F0 || !C || !eps)) return FEF_E_ARG;
  if ((int64_t)ws_bytes < scf_ws_bytes(*p) || !ws) return FEF_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const ScfWs w = scf_ws(*p, ws);
  const double* Dold = Dprev ? Dprev : w.Dold;
  double* Dnew = Dout ? Dout : (D ? D : w.Dspare);
  // with a carried density the moments kernel clears the maximum that the
  // eigensolver accumulates (no kernel of its own)
  const bool clear_in_moments = Dprev && Bp && p->nfrag > 0;
  // moments_in: the previous step's eigensolver left this step's moments in
  // the workspace (no moments kernel; the field kernel clears the maximum);
  // moments_out: this step's eigensolver leaves the next step's there
  moments_in = moments_in && clear_in_moments;
  moments_out = moments_out && carry_out && Bp && p->nfrag > 0;
  stage_mark(*p, 0, st);
  hipError_t e = !Dprev ? launch_density(*p, C, w.Dold, Bp ? w.Dw : nullptr, dD_max, st)
                 : clear_in_moments ? hipSuccess
                                    : launch_zero_scalar(dD_max, st);
  stage_mark(*p, 1, st);
  if (e == hipSuccess && p->nfrag > 0)
    e = Bp ? launch_field_packed(*p, Bp, G, w.Dw, F0, htilde, w.F, w.wd, w.wphi, st, B_pack,
                                 Bp_out, clear_in_moments ? dD_max : nullptr, moments_in)
           : launch_field(*p, B, G, Dold, F0, htilde, w.F, w.wd, w.wphi, st);
  stage_mark(*p, 3, st);
  if (e == hipSuccess && p->nfrag > 0)
    e = launch_eigh(*p, w.F, Dold, C, eps, Dnew, dD_max, flags, w.eigws, st,
                    carry_out ? w.Dw : nullptr, moments_out ? (Bp_out ? Bp_out : Bp) : nullptr,
                    moments_out ? w.wd : nullptr);
  stage_mark(*p, 4, st);
  return hip_status(e);
}

fef_status fef_plan_stage_timing(fef_plan p, int32_t enable) {
  if (!p) return FEF_E_ARG;
  if (enable) {
    for (hipEvent_t& e : p->stage_ev)
      if (!e && hipEventCreate(&e) != hipSuccess) return FEF_E_HIP;
  }
  p->stage_timing = enable != 0;
  return FEF_OK;
}

fef_status fef_plan_stage_ms(fef_plan p, double* ms) {
  if (!p || !ms) return FEF_E_ARG;
  if (!p->stage_ev[0]) return FEF_E_ARG;
  if (hipEventSynchronize(p->stage_ev[kStageMarks - 1]) != hipSuccess) return FEF_E_HIP;
  for (int i = 0; i + 1 < kStageMarks; ++i) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, p->stage_ev[i], p->stage_ev[i + 1]) != hipSuccess)
      return FEF_E_HIP;
    ms[i] = t;
  }
  return FEF_OK;
}

fef_status fef_scf_step(fef_plan p, const double* B, const double* G, const double* F0,
                        const double* htilde, double* C, double* eps, double* D,
                        double* dD_max, int32_t* flags, void* ws, size_t ws_bytes,
                        void* stream) {
  return scf_step_impl(p, B, nullptr, G, F0, htilde, C, eps, D, dD_max, flags, ws, ws_bytes,
                       stream);
}

fef_status fef_pack_coefficients(fef_plan p, const double* B, double* Bp, void* stream) {
  if (!p) return FEF_E_ARG;
  if (p->nfrag > 0 && (!B || !Bp)) return FEF_E_ARG;
  return hip_status(launch_pack_coefficients(*p, B, Bp, static_cast<hipStream_t>(stream)));
}

fef_status fef_scf_step_packed(fef_plan p, const double* Bp, const double* G, const double* F0,
                               const double* htilde, double* C, double* eps, double* D,
                               double* dD_max, int32_t* flags, void* ws, size_t ws_bytes,
                               void* stream) {
  if (p && p->nfrag > 0 && !Bp) return FEF_E_ARG;
  return scf_step_impl(p, nullptr, Bp, G, F0, htilde, C, eps, D, dD_max, flags, ws, ws_bytes,
                       stream);
}

}  // extern "C"

namespace fef {

fef_status scf_step_packing(fef_plan p, const double* B, double* Bp, const double* G,
                            const double* F0, const double* htilde, double* C, double* eps,
                            double* D, double* dD_max, int32_t* flags, void* ws, size_t ws_bytes,
                            void* stream) {
  if (p && p->nfrag > 0 && (!B || !Bp)) return FEF_E_ARG;
  return scf_step_impl(p, nullptr, Bp, G, F0, htilde, C, eps, D, dD_max, flags, ws, ws_bytes,
                       stream, B, Bp);
}

bool density_carry_ok(const fef_plan_s& p) { return p.max_nbf <= 32; }

bool moments_carry_ok(const fef_plan_s& p) {
  if (!density_carry_ok(p) || !small_fragments(p)) return false;
  for (const FragInfo& fi : p.frag) {
    const int nt = fi.nbf * (fi.nbf + 1) / 2;
    if ((nt & 1) != 0 || nt > 384) return false;
  }
  return true;
}

fef_status scf_step_carry(fef_plan p, const double* B_pack, double* Bp, const double* G,
                          const double* F0, const double* htilde, double* C, double* eps,
                          double* D, double* dD_max, int32_t* flags, void* ws, size_t ws_bytes,
                          void* stream, int step, int nsteps) {
  if (!p || !D || !ws || !density_carry_ok(*p) || step < 0 || step >= nsteps) return FEF_E_ARG;
  if (p->nfrag > 0 && !Bp) return FEF_E_ARG;
  if (step > 0 && B_pack) return FEF_E_ARG;  // the packing step starts a pass
  if ((int64_t)ws_bytes < scf_ws_bytes(*p)) return FEF_E_WORKSPACE;
  // the new densities alternate between the spare pool and D so that the
  // last step's lands in D and no step reads the pool it writes
  double* spare = scf_ws(*p, ws).Dspare;
  auto target = [&](int s) { return ((nsteps - 1 - s) % 2 == 0) ? D : spare; };
  // with moments_carry_ok every step but the last also forms the next
  // step's moments in its eigensolver, and every step but the first uses them
  const bool mc = moments_carry_ok(*p);
  return scf_step_impl(p, nullptr, Bp, G, F0, htilde, C, eps, D, dD_max, flags, ws, ws_bytes,
                       stream, B_pack, B_pack ? Bp : nullptr, true,
                       step > 0 ? target(step - 1) : nullptr, target(step), mc && step > 0,
                       mc && step + 1 < nsteps);
}

}  // namespace fef
