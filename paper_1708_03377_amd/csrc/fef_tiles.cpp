// Pair-kernel work decomposition, built once per plan on the host.
//
// 1. Locality order: reverse Cuthill-McKee over the pair graph gives a
//    breadth-first sweep through the box; walking it, every fragment not yet
//    placed seeds a cluster with its (up to) three nearest unplaced
//    neighbours (largest s_xy = 1/R).  Clusters are laid out one after the
//    other, so runs of 4 (or 2) consecutive fragments are spatially tight and
//    share most of their partners.  No coordinates are needed.
// 2. Orientation: the streamed ("y") side of a pair must be a class-0
//    fragment; between two class-0 fragments the one earlier in the order is
//    x.  E2_xy is symmetric, so orientation changes no result.
// 3. Slots: each pair's (row tile, column tile) output tiles own consecutive
//    partial-sum slots; E2_pair sums them in a fixed order.
// 4. Tiles (per precision mode): x units (fragment, row tile) taken in
//    locality order are grouped xb at a time into x-blocks; each block's
//    entries are the union of its units' partners (column tiles), in locality
//    order; entries are chunked into work items of at most yc; the items are
//    split into eight runs of x-blocks of about equal work (one queue per
//    XCD), each sorted longest first (LPT).
#include <algorithm>
#include <cstring>
#include <numeric>
#include <queue>
#include <vector>

#include "fef_internal.h"

namespace fef {

void order_and_orient(fef_plan_s& p) {
  const int n = p.nfrag;
  std::vector<std::vector<int32_t>> adj(n);
  for (const auto& pr : p.pairs) {
    adj[pr.x].push_back(pr.y);
    adj[pr.y].push_back(pr.x);
  }
  std::vector<int32_t> deg(n);
  for (int f = 0; f < n; ++f) {
    auto& a = adj[f];
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
    deg[f] = (int32_t)a.size();
  }
  // Cuthill-McKee from a minimum-degree start in every component, then reverse.
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<char> seen(n, 0);
  std::vector<int32_t> byDeg(n);
  std::iota(byDeg.begin(), byDeg.end(), 0);
  std::stable_sort(byDeg.begin(), byDeg.end(), [&](int a, int b) { return deg[a] < deg[b]; });
  for (int s : byDeg) {
    if (seen[s]) continue;
    std::queue<int32_t> q;
    q.push(s);
    seen[s] = 1;
    while (!q.empty()) {
      const int u = q.front();
      q.pop();
      order.push_back(u);
      std::vector<int32_t> nb;
      for (int v : adj[u])
        if (!seen[v]) { seen[v] = 1; nb.push_back(v); }
      std::stable_sort(nb.begin(), nb.end(), [&](int a, int b) { return deg[a] < deg[b]; });
      for (int v : nb) q.push(v);
    }
  }
  std::reverse(order.begin(), order.end());
  // nearest-neighbour clusters of kCluster fragments along the RCM sweep;
  // fragments with several row tiles form clusters of their own
  constexpr int kCluster = 4;
  std::vector<std::vector<std::pair<double, int32_t>>> near(n);
  for (const auto& pr : p.pairs) {
    near[pr.x].push_back({pr.s, pr.y});
    near[pr.y].push_back({pr.s, pr.x});
  }
  std::vector<char> placed(n, 0);
  std::vector<int32_t> clustered;
  clustered.reserve(n);
  for (int u : order) {
    if (placed[u]) continue;
    placed[u] = 1;
    clustered.push_back(u);
    if (p.frag[u].ntile > 1) continue;
    auto& c = near[u];
    std::stable_sort(c.begin(), c.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    int taken = 1;
    for (const auto& sv : c) {
      if (taken == kCluster) break;
      const int v = sv.second;
      if (placed[v] || p.frag[v].ntile > 1) continue;
      placed[v] = 1;
      clustered.push_back(v);
      ++taken;
    }
  }
  order.swap(clustered);
  p.rank.assign(n, 0);
  for (int i = 0; i < n; ++i) p.rank[order[i]] = i;
  for (int f = 0; f < n; ++f) p.frag[f].rank = p.rank[f];

  // orientation and slots
  int64_t slot = 0;
  for (auto& pr : p.pairs) {
    int32_t x = pr.x, y = pr.y;
    const bool cx0 = p.frag[x].cls == 0, cy0 = p.frag[y].cls == 0;
    if (!cy0 || (cx0 && p.rank[y] < p.rank[x])) std::swap(x, y);
    pr.x = x;
    pr.y = y;
    pr.ntx = p.frag[x].ntile;
    pr.nty = p.frag[y].ntile;
    pr.slot_first = (int32_t)slot;
    slot += (int64_t)pr.ntx * pr.nty;
  }
  p.nslot = slot;
}

void free_tiles(TileSet& t) {
  if (t.d_items) (void)hipFree(t.d_items);
  if (t.d_entries) (void)hipFree(t.d_entries);
  if (t.d_xblocks) (void)hipFree(t.d_xblocks);
  if (t.d_grp_off) (void)hipFree(t.d_grp_off);
  t = TileSet();
}

template <class T>
static hipError_t upload_vec(T** dst, const std::vector<T>& v) {
  *dst = nullptr;
  if (v.empty()) return hipSuccess;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), v.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

hipError_t build_tiles(fef_plan_s& p, int prec, int xb, int yc) {
  const int n = p.nfrag;
  // partners of every x fragment: (y, pair index), in locality order of y
  std::vector<std::vector<std::pair<int32_t, int32_t>>> part(n);
  for (int32_t k = 0; k < (int32_t)p.pairs.size(); ++k) {
    const auto& pr = p.pairs[k];
    if (pr.ntx == 0 || pr.nty == 0) continue;
    part[pr.x].push_back({pr.y, k});
  }
  for (auto& v : part)
    std::sort(v.begin(), v.end(), [&](const auto& a, const auto& b) {
      return p.rank[a.first] < p.rank[b.first];
    });
  std::vector<int32_t> byRank(n);
  for (int f = 0; f < n; ++f) byRank[p.rank[f]] = f;

  struct Unit { int32_t f, mt; };
  std::vector<Unit> units;
  for (int r = 0; r < n; ++r) {
    const int f = byRank[r];
    if (part[f].empty()) continue;
    for (int mt = 0; mt < p.frag[f].ntile; ++mt) units.push_back({f, mt});
  }

  std::vector<XBlock> blocks;
  std::vector<Entry> entries;
  std::vector<WorkItem> items;
  struct Cand { int32_t rk, y, nt, u, slot; double s; };
  const bool plain = prec == FEF_F64 || prec == FEF_F32;
  const int64_t elem = p.geom[prec].elem_bytes;
  // split modes: stored row length (16-bit elements), nterm planes and 8 zeros
  const int64_t xs = (int64_t)p.geom[prec].nterm * p.geom[prec].pw + 8;
  for (size_t u0 = 0; u0 < units.size(); u0 += xb) {
    XBlock blk;
    for (int u = 0; u < kMaxXB; ++u) { blk.f[u] = -1; blk.mt[u] = 0; }
    std::vector<Cand> c;
    for (int u = 0; u < xb && u0 + u < units.size(); ++u) {
      const Unit un = units[u0 + u];
      blk.f[u] = un.f;
      blk.mt[u] = un.mt;
      for (const auto& yp : part[un.f]) {
        const PairInfo& pr = p.pairs[yp.second];
        for (int nt = 0; nt < pr.nty; ++nt)
          c.push_back({p.rank[yp.first], yp.first, nt, u, pr.slot_first + un.mt * pr.nty + nt,
                       pr.s});
      }
    }
    std::sort(c.begin(), c.end(), [](const Cand& a, const Cand& b) {
      return a.rk != b.rk ? a.rk < b.rk : a.nt < b.nt;
    });
    const int32_t bid = (int32_t)blocks.size();
    blocks.push_back(blk);
    const int32_t first = (int32_t)entries.size();
    for (size_t i = 0; i < c.size();) {
      Entry e;
      std::memset(&e, 0, sizeof(e));
      e.y = c[i].y;
      e.nt = c[i].nt;
      const FragInfo& fy = p.frag[e.y];
      e.ld_y = (int32_t)fy.ld;
      // plain modes: column block nt of [kpad][ld]; split modes: row block
      // nt of [ld][nterm pw + 8]
      e.off_R = fy.off_R[prec] + (plain ? (int64_t)e.nt * kTile * elem
                                        : (int64_t)e.nt * kTile * xs * elem);
      e.off_gap = fy.off_gap + (int64_t)e.nt * kTile;
      for (int u = 0; u < kMaxXB; ++u) { e.slot[u] = -1; e.s[u] = 0.0; }
      size_t j = i;
      for (; j < c.size() && c[j].y == c[i].y && c[j].nt == c[i].nt; ++j) {
        e.slot[c[j].u] = c[j].slot;
        e.s[c[j].u] = c[j].s;
      }
      entries.push_back(e);
      i = j;
    }
    const int32_t cnt = (int32_t)entries.size() - first;
    for (int32_t e0 = 0; e0 < cnt; e0 += yc) items.push_back({bid, first + e0, std::min(yc, cnt - e0), 0});
  }
  // queue groups: contiguous runs of items (x-blocks in locality order) of
  // about equal total work, then longest first inside each group
  std::vector<int32_t> grp(items.size());
  {
    int64_t total = 0;
    for (const auto& it : items) total += it.ne;
    int64_t before = 0;
    for (size_t i = 0; i < items.size(); ++i) {
      grp[i] = total > 0 ? (int32_t)std::min<int64_t>(kQueues - 1, before * kQueues / total) : 0;
      before += items[i].ne;
    }
  }
  std::vector<int32_t> order(items.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return grp[a] != grp[b] ? grp[a] < grp[b] : items[a].ne > items[b].ne;
  });
  std::vector<WorkItem> sorted(items.size());
  std::vector<int32_t> grp_off(kQueues + 1, 0);
  for (size_t i = 0; i < order.size(); ++i) {
    sorted[i] = items[order[i]];
    ++grp_off[grp[order[i]] + 1];
  }
  for (int g = 0; g < kQueues; ++g) grp_off[g + 1] += grp_off[g];
  items.swap(sorted);

  TileSet t;
  t.xb = xb;
  t.yc = yc;
  t.nitems = (int64_t)items.size();
  t.nentries = (int64_t)entries.size();
  t.nxblocks = (int64_t)blocks.size();
  hipError_t e = upload_vec(&t.d_items, items);
  if (e == hipSuccess) e = upload_vec(&t.d_entries, entries);
  if (e == hipSuccess) e = upload_vec(&t.d_xblocks, blocks);
  if (e == hipSuccess) e = upload_vec(&t.d_grp_off, grp_off);
  if (e != hipSuccess) { free_tiles(t); return e; }
  if (p.graphs_live[prec] > 0)
    p.retired_tiles.push_back(p.tiles[prec]);  // a captured pass still reads them
  else
    free_tiles(p.tiles[prec]);
  p.tiles[prec] = t;
  return hipSuccess;
}

}  // namespace fef
