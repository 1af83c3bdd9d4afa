// Union-find decoder of syndrome detection events (host code of libstn).
//
// The paper decodes its memory experiments by minimum-weight matching over a
// Pauli error model built from the Pauli-twirled noise (Sec. III.D); this
// library's decoder is the union-find decoder of Delfosse and Nickerson
// (almost-linear time, close to matching at low error rates) with weighted
// cluster growth.  Input: a detector graph whose edges are independent error
// mechanisms (two detectors, or one detector and the boundary), each with a
// weight log((1 - p) / p) and a flag telling whether it flips the logical
// observable; per shot, the detectors that fired.  Output per shot: the
// predicted observable flip (the parity of the flagged edges of the
// correction) and, optionally, the correction itself.
//
// Per shot:
//  1. every fired detector starts an odd cluster; the boundary is one extra
//     vertex, and a cluster that contains it counts as even;
//  2. growth: each odd cluster advances every edge on its border by the
//     smallest amount that completes one of them (an edge of weight w is
//     complete at 2 w, grown from both ends at once when both are odd); a
//     completed edge merges the clusters at its ends (union by size, path
//     halving); repeat until no cluster is odd;
//  3. peeling: a spanning forest of the completed edges of each cluster,
//     rooted at the boundary when the cluster holds it, is peeled from the
//     leaves: a leaf whose vertex is marked puts its edge into the
//     correction and moves the mark to its parent.  The correction's
//     boundary is then exactly the set of fired detectors.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/stn.h"

namespace {

struct Dsu {
  std::vector<int> parent, size, parity, has_bnd;
  explicit Dsu(int n) : parent(n), size(n, 1), parity(n, 0), has_bnd(n, 0) {
    for (int i = 0; i < n; ++i) parent[i] = i;
  }
  int find(int x) {
    while (parent[x] != x) {
      parent[x] = parent[parent[x]];
      x = parent[x];
    }
    return x;
  }
  int unite(int a, int b) {
    a = find(a);
    b = find(b);
    if (a == b) return a;
    if (size[a] < size[b]) std::swap(a, b);
    parent[b] = a;
    size[a] += size[b];
    parity[a] ^= parity[b];
    has_bnd[a] |= has_bnd[b];
    return a;
  }
  bool odd(int x) {
    const int r = find(x);
    return parity[r] && !has_bnd[r];
  }
};

struct Graph {
  int nv;                                  // detectors + 1 (the boundary, index n_nodes)
  std::vector<int> ea, eb;                 // edge ends
  std::vector<double> w;                   // weights (> 0)
  std::vector<std::vector<int>> inc;       // incident edges per vertex
};

// Decodes one shot; corr (n_edges bytes) receives the correction.
int decode_one(const Graph &g, const uint8_t *ev, int n_nodes, uint8_t *corr) {
  const int nv = g.nv, ne = (int)g.w.size();
  Dsu d(nv);
  d.has_bnd[n_nodes] = 1;
  bool any = false;
  for (int v = 0; v < n_nodes; ++v)
    if (ev[v]) { d.parity[v] = 1; any = true; }
  std::memset(corr, 0, (size_t)ne);
  if (!any) return 0;
  std::vector<double> grown(ne, 0.0);
  std::vector<uint8_t> done(ne, 0);
  // 2. growth
  for (int iter = 0; iter < 4 * ne + 8; ++iter) {
    // rate of each edge: number of odd clusters at its ends (0, 1 or 2)
    double step = INFINITY;
    std::vector<uint8_t> rate(ne, 0);
    bool odd_left = false;
    for (int e = 0; e < ne; ++e) {
      if (done[e]) continue;
      const int ra = d.find(g.ea[e]), rb = d.find(g.eb[e]);
      if (ra == rb) { done[e] = 1; continue; }          // inside one cluster already
      const int k = (d.odd(ra) ? 1 : 0) + (d.odd(rb) ? 1 : 0);
      rate[e] = (uint8_t)k;
      if (k) {
        odd_left = true;
        const double left = 2.0 * g.w[e] - grown[e];
        step = std::fmin(step, left / k);
      }
    }
    if (!odd_left) break;
    std::vector<int> fused;
    for (int e = 0; e < ne; ++e) {
      if (!rate[e]) continue;
      grown[e] += step * rate[e];
      if (grown[e] >= 2.0 * g.w[e] * (1.0 - 1e-12)) fused.push_back(e);
    }
    for (int e : fused) {
      done[e] = 2;                                       // completed and kept for peeling
      d.unite(g.ea[e], g.eb[e]);
    }
  }
  // 3. peeling over the completed edges (done == 2), one forest per cluster
  std::vector<int> par_edge(nv, -1), order;
  std::vector<uint8_t> seen(nv, 0), mark(nv, 0);
  for (int v = 0; v < n_nodes; ++v) mark[v] = ev[v] ? 1 : 0;
  auto bfs = [&](int root) {
    size_t head = order.size();
    order.push_back(root);
    seen[root] = 1;
    while (head < order.size()) {
      const int v = order[head++];
      for (int e : g.inc[v]) {
        if (done[e] != 2) continue;
        const int u = g.ea[e] == v ? g.eb[e] : g.ea[e];
        if (seen[u]) continue;
        seen[u] = 1;
        par_edge[u] = e;
        order.push_back(u);
      }
    }
  };
  bfs(n_nodes);                                          // the boundary's cluster first
  for (int v = 0; v < n_nodes; ++v)
    if (!seen[v] && ev[v]) bfs(v);
  for (size_t i = order.size(); i-- > 0;) {
    const int v = order[i];
    const int e = par_edge[v];
    if (e < 0 || !mark[v]) continue;
    corr[e] = 1;
    mark[v] = 0;
    const int u = g.ea[e] == v ? g.eb[e] : g.ea[e];
    mark[u] ^= 1;
  }
  return 0;
}

}  // namespace

extern "C" stn_status stn_decode(const stn_dem_edge *edges, int n_edges, int n_nodes, const uint8_t *events,
                                 int n_shots, uint8_t *pred, uint8_t *corrections) {
  if (!edges || n_edges < 1 || n_nodes < 1 || !events || n_shots < 0 || !pred) return STN_EINVAL;
  Graph g;
  g.nv = n_nodes + 1;
  g.ea.resize(n_edges);
  g.eb.resize(n_edges);
  g.w.resize(n_edges);
  g.inc.assign(g.nv, {});
  for (int e = 0; e < n_edges; ++e) {
    const int a = edges[e].a, b = edges[e].b;
    if (a < 0 || a > n_nodes || b < 0 || b > n_nodes || a == b) return STN_EINVAL;
    if (!(edges[e].weight > 0) || std::isinf(edges[e].weight)) return STN_EINVAL;
    g.ea[e] = a;
    g.eb[e] = b;
    g.w[e] = edges[e].weight;
    g.inc[a].push_back(e);
    g.inc[b].push_back(e);
  }
  std::vector<uint8_t> corr(n_edges);
  for (int s = 0; s < n_shots; ++s) {
    uint8_t *c = corrections ? corrections + (size_t)s * n_edges : corr.data();
    decode_one(g, events + (size_t)s * n_nodes, n_nodes, c);
    int flip = 0;
    for (int e = 0; e < n_edges; ++e) flip ^= (c[e] & edges[e].obs) ? 1 : 0;
    pred[s] = (uint8_t)flip;
  }
  return STN_OK;
}
