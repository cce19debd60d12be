// CPU oracle for the dynamic slab-hash graph path -- TEST INFRASTRUCTURE ONLY.
//
// This file is the plain, slow, single-threaded reference that the GPU path is checked
// against.  Only the tests, the smoke entry point and the benchmark's CPU-baseline leg
// may load it; the product path never calls it.  It shares no code, header, table or
// constant with the HIP library.
//
// State is a sorted adjacency per vertex.  Every algorithm is recomputed from scratch
// on the current state with its textbook definition; none of the paper's incremental
// machinery appears here:
//   * edge insert / delete / search semantics: the graph-operation discussion of the
//     experimental section (insert stores an edge only if it is absent; delete turns a
//     present edge into a tombstone; search probes for membership and the weight);
//   * BFS levels and SSSP distances with the dependence-tree parent of the dynamic SSSP
//     section (section 4.2): parent(v) = the smallest-id predecessor u with
//     dist(u) + w(u,v) = dist(v), the order a 64-bit atomicMin on <dist,parent> induces
//     (the footnote on the packed tree node);
//   * weakly connected components by sequential union-find (section 4.4), labelled by
//     the smallest vertex id of each component;
//   * PageRank by FP64 power iteration of the section 4.1 equation, with the
//     teleport term for zero-out-degree vertices of the same section;
//   * triangle count of the undirected simple graph underlying the arc set
//     (section 4.3 counts triangles of an undirected graph), by degree-ordered
//     sorted-list intersection, and by a triple loop for tiny graphs.
//
// Parity is pinned by the tests against closed forms and brute force; see the
// "not gpu" tests.  Build: g++ -O2 -std=c++17 -shared -fPIC oracle.cpp -o liboracle.so

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <queue>
#include <utility>
#include <vector>
#include <cmath>

namespace {

constexpr uint32_t kInf = 0xFFFFFFFFu;        // unreachable distance / level
constexpr uint32_t kNoVertex = 0xFFFFFFFFu;   // no parent
constexpr uint32_t kReservedLow = 0xFFFFFFFDu; // ids at or above are reserved sentinels

struct Arc {
  uint32_t dst;
  uint32_t w;
};

struct Graph {
  uint32_t n = 0;
  std::vector<std::vector<Arc>> out;  // sorted by dst, no duplicates
};

bool arc_less(const Arc& a, uint32_t d) { return a.dst < d; }

// Status byte of one update: 1 applied, 0 no-op, 2 rejected.
uint8_t validate(const Graph& g, uint32_t s, uint32_t d) {
  if (s >= g.n || d >= g.n || s == d || s >= kReservedLow || d >= kReservedLow) return 2;
  return 0;
}

uint8_t insert_one(Graph& g, uint32_t s, uint32_t d, uint32_t w) {
  if (validate(g, s, d) == 2) return 2;
  auto& a = g.out[s];
  auto it = std::lower_bound(a.begin(), a.end(), d, arc_less);
  if (it != a.end() && it->dst == d) return 0;  // present: weight unchanged
  a.insert(it, Arc{d, w});
  return 1;
}

uint8_t delete_one(Graph& g, uint32_t s, uint32_t d) {
  if (validate(g, s, d) == 2) return 2;
  auto& a = g.out[s];
  auto it = std::lower_bound(a.begin(), a.end(), d, arc_less);
  if (it == a.end() || it->dst != d) return 0;
  a.erase(it);
  return 1;
}

// Undirected simple graph under the arc set: sorted neighbour lists, no self-loops.
std::vector<std::vector<uint32_t>> undirected(const Graph& g) {
  std::vector<std::vector<uint32_t>> nb(g.n);
  for (uint32_t u = 0; u < g.n; ++u)
    for (const Arc& a : g.out[u]) {
      nb[u].push_back(a.dst);
      nb[a.dst].push_back(u);
    }
  for (auto& l : nb) {
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
  }
  return nb;
}

}  // namespace

extern "C" {

void* orc_create(uint32_t n, const uint32_t* src, const uint32_t* dst, const uint32_t* w,
                 uint64_t m) {
  Graph* g = new Graph();
  g->n = n;
  g->out.assign(n, {});
  // Arcs are taken in input order with insert semantics (first copy wins).
  std::vector<uint64_t> cnt(n, 0);
  for (uint64_t i = 0; i < m; ++i)
    if (src[i] < n) cnt[src[i]]++;
  for (uint32_t v = 0; v < n; ++v) g->out[v].reserve(cnt[v]);
  for (uint64_t i = 0; i < m; ++i) {
    uint32_t s = src[i], d = dst[i];
    if (validate(*g, s, d) == 2) continue;
    g->out[s].push_back(Arc{d, w ? w[i] : 1u});
  }
  for (auto& a : g->out) {
    std::stable_sort(a.begin(), a.end(), [](const Arc& x, const Arc& y) { return x.dst < y.dst; });
    a.erase(std::unique(a.begin(), a.end(), [](const Arc& x, const Arc& y) { return x.dst == y.dst; }),
            a.end());
  }
  return g;
}

void orc_destroy(void* h) { delete static_cast<Graph*>(h); }

uint64_t orc_num_arcs(void* h) {
  const Graph& g = *static_cast<Graph*>(h);
  uint64_t m = 0;
  for (const auto& a : g.out) m += a.size();
  return m;
}

void orc_out_degree(void* h, uint32_t* deg) {
  const Graph& g = *static_cast<Graph*>(h);
  for (uint32_t v = 0; v < g.n; ++v) deg[v] = static_cast<uint32_t>(g.out[v].size());
}

// Sequential batch application, ops in array order.
void orc_insert(void* h, const uint32_t* src, const uint32_t* dst, const uint32_t* w, uint64_t b,
                uint8_t* status) {
  Graph& g = *static_cast<Graph*>(h);
  for (uint64_t i = 0; i < b; ++i) {
    uint8_t s = insert_one(g, src[i], dst[i], w ? w[i] : 1u);
    if (status) status[i] = s;
  }
}

void orc_delete(void* h, const uint32_t* src, const uint32_t* dst, uint64_t b, uint8_t* status) {
  Graph& g = *static_cast<Graph*>(h);
  for (uint64_t i = 0; i < b; ++i) {
    uint8_t s = delete_one(g, src[i], dst[i]);
    if (status) status[i] = s;
  }
}

void orc_query(void* h, const uint32_t* src, const uint32_t* dst, uint64_t b, uint8_t* found,
               uint32_t* wout) {
  const Graph& g = *static_cast<Graph*>(h);
  for (uint64_t i = 0; i < b; ++i) {
    uint32_t s = src[i], d = dst[i];
    uint8_t f = 0;
    uint32_t wv = 0;
    if (s < g.n) {
      const auto& a = g.out[s];
      auto it = std::lower_bound(a.begin(), a.end(), d, arc_less);
      if (it != a.end() && it->dst == d) {
        f = 1;
        wv = it->w;
      }
    }
    found[i] = f;
    if (wout) wout[i] = wv;
  }
}

// Export all arcs (sorted by src then dst).  Returns the count written.
uint64_t orc_export(void* h, uint32_t* src, uint32_t* dst, uint32_t* w) {
  const Graph& g = *static_cast<Graph*>(h);
  uint64_t k = 0;
  for (uint32_t u = 0; u < g.n; ++u)
    for (const Arc& a : g.out[u]) {
      src[k] = u;
      dst[k] = a.dst;
      if (w) w[k] = a.w;
      ++k;
    }
  return k;
}

// Parent rule shared by BFS and SSSP: the smallest-id in-neighbour u achieving
// dist(u) + w(u,v) == dist(v); the source is its own parent.
static void min_parent(const Graph& g, uint32_t source, const std::vector<uint64_t>& dist,
                       bool unit, uint32_t* parent) {
  for (uint32_t v = 0; v < g.n; ++v) parent[v] = kNoVertex;
  for (uint32_t u = 0; u < g.n; ++u) {
    if (dist[u] == UINT64_MAX) continue;
    for (const Arc& a : g.out[u]) {
      uint64_t cand = dist[u] + (unit ? 1u : a.w);
      if (a.dst != source && cand == dist[a.dst] && u < parent[a.dst]) parent[a.dst] = u;
    }
  }
  parent[source] = source;
}

// Breadth-first search levels from `source` (queue-based).
void orc_bfs(void* h, uint32_t source, uint32_t* level, uint32_t* parent) {
  const Graph& g = *static_cast<Graph*>(h);
  std::vector<uint64_t> dist(g.n, UINT64_MAX);
  std::queue<uint32_t> q;
  dist[source] = 0;
  q.push(source);
  while (!q.empty()) {
    uint32_t u = q.front();
    q.pop();
    for (const Arc& a : g.out[u])
      if (dist[a.dst] == UINT64_MAX) {
        dist[a.dst] = dist[u] + 1;
        q.push(a.dst);
      }
  }
  for (uint32_t v = 0; v < g.n; ++v) level[v] = dist[v] == UINT64_MAX ? kInf : uint32_t(dist[v]);
  min_parent(g, source, dist, true, parent);
}

// Dijkstra with 64-bit accumulators; returns 0, or 1 if a distance does not fit u32.
int orc_sssp(void* h, uint32_t source, uint32_t* distance, uint32_t* parent) {
  const Graph& g = *static_cast<Graph*>(h);
  std::vector<uint64_t> dist(g.n, UINT64_MAX);
  using Item = std::pair<uint64_t, uint32_t>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> pq;
  dist[source] = 0;
  pq.push({0, source});
  while (!pq.empty()) {
    auto [du, u] = pq.top();
    pq.pop();
    if (du != dist[u]) continue;
    for (const Arc& a : g.out[u]) {
      uint64_t nd = du + a.w;
      if (nd < dist[a.dst]) {
        dist[a.dst] = nd;
        pq.push({nd, a.dst});
      }
    }
  }
  int overflow = 0;
  for (uint32_t v = 0; v < g.n; ++v) {
    if (dist[v] != UINT64_MAX && dist[v] >= kInf) overflow = 1;
    distance[v] = dist[v] == UINT64_MAX ? kInf : uint32_t(dist[v]);
  }
  min_parent(g, source, dist, false, parent);
  return overflow;
}

// Weakly connected components: sequential union-find over every arc, direction ignored.
void orc_wcc(void* h, uint32_t* label) {
  const Graph& g = *static_cast<Graph*>(h);
  std::vector<uint32_t> up(g.n);
  for (uint32_t v = 0; v < g.n; ++v) up[v] = v;
  auto find = [&](uint32_t x) {
    while (up[x] != x) {
      up[x] = up[up[x]];
      x = up[x];
    }
    return x;
  };
  for (uint32_t u = 0; u < g.n; ++u)
    for (const Arc& a : g.out[u]) {
      uint32_t ru = find(u), rv = find(a.dst);
      if (ru != rv) up[std::max(ru, rv)] = std::min(ru, rv);
    }
  // label = smallest id in the component
  std::vector<uint32_t> minid(g.n, kNoVertex);
  for (uint32_t v = 0; v < g.n; ++v) {
    uint32_t r = find(v);
    minid[r] = std::min(minid[r], v);
  }
  for (uint32_t v = 0; v < g.n; ++v) label[v] = minid[find(v)];
}

// FP64 PageRank power iteration: x' = (1-d)/N + d * (sum_{u->v} x[u]/out[u]
// + (sum_{out(z)=0} x[z]) / N), from x = 1/N (or from `rank` when warm != 0), until
// the L1 change is below `tol` or `max_iter` iterations.  Returns the iteration count.
uint32_t orc_pagerank(void* h, double d, double tol, uint32_t max_iter, int warm, double* rank) {
  const Graph& g = *static_cast<Graph*>(h);
  const uint32_t n = g.n;
  std::vector<double> x(n), y(n);
  for (uint32_t v = 0; v < n; ++v) x[v] = warm ? rank[v] : 1.0 / n;
  uint32_t it = 0;
  while (it < max_iter) {
    double dangling = 0.0;
    for (uint32_t v = 0; v < n; ++v) {
      y[v] = 0.0;
      if (g.out[v].empty()) dangling += x[v];
    }
    for (uint32_t u = 0; u < n; ++u) {
      if (g.out[u].empty()) continue;
      double c = x[u] / double(g.out[u].size());
      for (const Arc& a : g.out[u]) y[a.dst] += c;
    }
    double delta = 0.0;
    for (uint32_t v = 0; v < n; ++v) {
      y[v] = (1.0 - d) / n + d * (y[v] + dangling / n);
      delta += std::fabs(y[v] - x[v]);
    }
    std::swap(x, y);
    ++it;
    if (delta < tol) break;
  }
  for (uint32_t v = 0; v < n; ++v) rank[v] = x[v];
  return it;
}

// Triangles of the underlying undirected simple graph: orient each edge from the
// endpoint of smaller (degree, id) to the larger and intersect sorted out-lists.
uint64_t orc_triangles(void* h) {
  const Graph& g = *static_cast<Graph*>(h);
  auto nb = undirected(g);
  auto before = [&](uint32_t a, uint32_t b) {
    return nb[a].size() < nb[b].size() || (nb[a].size() == nb[b].size() && a < b);
  };
  std::vector<std::vector<uint32_t>> fw(g.n);
  for (uint32_t u = 0; u < g.n; ++u)
    for (uint32_t v : nb[u])
      if (before(u, v)) fw[u].push_back(v);  // stays sorted by id
  uint64_t t = 0;
  for (uint32_t u = 0; u < g.n; ++u)
    for (uint32_t v : fw[u]) {
      const auto& a = fw[u];
      const auto& b = fw[v];
      size_t i = 0, j = 0;
      while (i < a.size() && j < b.size()) {
        if (a[i] < b[j]) ++i;
        else if (a[i] > b[j]) ++j;
        else { ++t; ++i; ++j; }
      }
    }
  return t;
}

// Triple loop over vertex triples (tiny graphs only): adjacency of the undirected graph.
uint64_t orc_triangles_brute(void* h) {
  const Graph& g = *static_cast<Graph*>(h);
  std::vector<std::vector<uint8_t>> adj(g.n, std::vector<uint8_t>(g.n, 0));
  for (uint32_t u = 0; u < g.n; ++u)
    for (const Arc& a : g.out[u]) adj[u][a.dst] = adj[a.dst][u] = 1;
  uint64_t t = 0;
  for (uint32_t a = 0; a < g.n; ++a)
    for (uint32_t b = a + 1; b < g.n; ++b)
      if (adj[a][b])
        for (uint32_t c = b + 1; c < g.n; ++c)
          if (adj[a][c] && adj[b][c]) ++t;
  return t;
}

// Triangles of the underlying undirected simple graph that have at least one edge among
// the k listed vertex pairs {a[i], b[i]} (order inside a pair, repeats, self-pairs and pairs
// that are not edges are ignored).  Every such triangle is counted once: from the smallest
// of its listed edges, so no triangle needs to be stored.  With the edges a batch added
// (removed), this is the count after (before) the batch minus the count before (after).
uint64_t orc_triangles_touching(void* h, const uint32_t* a, const uint32_t* b, uint64_t k) {
  const Graph& g = *static_cast<Graph*>(h);
  auto nb = undirected(g);
  auto key = [](uint32_t x, uint32_t y) {
    return x < y ? ((uint64_t)x << 32) | y : ((uint64_t)y << 32) | x;
  };
  auto is_edge = [&](uint32_t x, uint32_t y) { return std::binary_search(nb[x].begin(), nb[x].end(), y); };
  std::vector<uint64_t> listed;
  for (uint64_t i = 0; i < k; ++i)
    if (a[i] < g.n && b[i] < g.n && a[i] != b[i] && is_edge(a[i], b[i])) listed.push_back(key(a[i], b[i]));
  std::sort(listed.begin(), listed.end());
  listed.erase(std::unique(listed.begin(), listed.end()), listed.end());
  auto is_listed = [&](uint64_t e) { return std::binary_search(listed.begin(), listed.end(), e); };
  uint64_t t = 0;
  for (uint64_t e : listed) {
    const uint32_t u = uint32_t(e >> 32), v = uint32_t(e);
    const auto& x = nb[u];
    const auto& y = nb[v];
    size_t i = 0, j = 0;
    while (i < x.size() && j < y.size()) {
      if (x[i] < y[j]) { ++i; continue; }
      if (x[i] > y[j]) { ++j; continue; }
      const uint32_t w = x[i];
      ++i;
      ++j;
      const uint64_t e1 = key(u, w), e2 = key(v, w);
      if ((e1 < e && is_listed(e1)) || (e2 < e && is_listed(e2))) continue;  // counted from a smaller edge
      ++t;
    }
  }
  return t;
}

// Undirected degree of every vertex in the underlying simple graph.
void orc_undirected_degree(void* h, uint32_t* deg) {
  const Graph& g = *static_cast<Graph*>(h);
  auto nb = undirected(g);
  for (uint32_t v = 0; v < g.n; ++v) deg[v] = uint32_t(nb[v].size());
}

}  // extern "C"
