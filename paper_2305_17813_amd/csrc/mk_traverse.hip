// Dynamic BFS and SSSP (section 4.2, the batch-dynamic SSSP algorithm; BFS uses the same
// kernels with unit weights).
//
// Each vertex keeps a 64-bit tree node <distance, parent> (the footnote on the packed
// pair) updated by a 64-bit atomic minimum, so among equal distances the smallest parent
// id wins and the fixed point is unique.  A batch is applied by a prologue followed by
// the common frontier epilogue:
//   insert prologue : relax every effective inserted arc (u, v, w) with a finite u;
//   delete prologue : invalidate v for each deleted tree arc (parent(v) == u), invalidate
//                     the whole dependence subtree below it, then pull each invalidated
//                     vertex's best candidate from its valid in-neighbours (reverse view);
//                     this is the decremental frontier of valid -> invalid arcs;
//   epilogue        : expand the frontier until it is empty.
//
// Differences from the paper's kernels (same fixed point): the frontier holds vertices,
// not edges (a per-iteration stamp keeps each vertex once); subtree invalidation walks
// the tree top-down through the forward view instead of walking every vertex's parent
// chain to the source; vertices with many buckets are expanded by a whole block.
#include <algorithm>

#include "mk_internal.h"

using namespace mk;

namespace {

constexpr uint32_t kExpandBlocks = 2048;  // 256 CUs x 8 resident blocks
constexpr int kSyncEvery = 4;            // frontier launches between size read-backs

__device__ inline uint64_t tree_node(uint64_t dist, uint32_t parent) {
  if (dist >= 0xFFFFFFFFull) dist = 0xFFFFFFFEull;  // saturate below INF
  return (dist << 32) | parent;
}

constexpr uint32_t kGiantBuckets = 512;  // vertices with more buckets are split over 256 groups
constexpr uint32_t kGiantSplit = 256;

// Where pushed vertices go: light (<= kHeavyBuckets buckets), heavy (<= kGiantBuckets)
// and giant queues with their size counters.
struct PushQ {
  uint32_t* q[3];
  uint32_t* c[3];
};

__device__ inline void push_vertex(const uint32_t* nbk, const PushQ& Q, uint32_t* mark, uint32_t stamp,
                                   bool p, uint32_t v) {
  bool take = false;
  if (p) take = atomicExch(mark + v, stamp) != stamp;
  uint32_t nb = 0;
  if (take) nb = nbk[v];
  wave_push(Q.q[0], Q.c[0], take && nb <= kHeavyBuckets, v);
  wave_push(Q.q[1], Q.c[1], take && nb > kHeavyBuckets && nb <= kGiantBuckets, v);
  wave_push(Q.q[2], Q.c[2], take && nb > kGiantBuckets, v);
}

struct Queues {
  const uint32_t* cur[3];  // light, heavy, giant
  PushQ next;
  uint32_t* cnt;  // [3k .. 3k+2]: rotating sizes of queue k
  int icur, iclear;
};

// Relax every out-arc of u held in one slab word per lane.
template <bool kUnit>
__device__ inline void relax_word(const DView& F, uint64_t* D, uint32_t u, uint64_t du, uint64_t x,
                                  bool data, const Queues& q, uint32_t* mark, uint32_t stamp) {
  const uint32_t v = (uint32_t)x;
  bool improve = false;
  if (data && valid_key(v)) {
    const uint64_t w = kUnit ? 1ull : (x >> 32);
    const uint64_t cand = tree_node(du + w, u);
    if (cand < D[v]) improve = amin64(D + v, cand) > cand;
  }
  push_vertex(F.nbk, q.next, mark, stamp, improve, v);
}

template <bool kUnit>
__global__ void __launch_bounds__(kBlock) k_expand(DView F, uint64_t* D, Queues q, uint32_t* mark,
                                                   uint32_t stamp) {
  const uint32_t nl = q.cnt[q.icur], nh = q.cnt[3 + q.icur], ngi = q.cnt[6 + q.icur];
  if (blockIdx.x == 0 && threadIdx.x < 3) q.cnt[3 * threadIdx.x + q.iclear] = 0;
  if (nl == 0 && nh == 0 && ngi == 0) return;
  // single-bucket frontier vertices: one lane each (64 slab reads in flight per wave)
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += gridDim.x * blockDim.x) {
    const uint32_t u = q.cur[0][i];
    if (F.nbk[u] != 1) continue;
    const uint64_t du = ld_u64_coherent(D + u) >> 32;
    Slab sl;
    uint32_t t = u;
    while (true) {
      load_slab(F, t, sl);
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j) relax_word<kUnit>(F, D, u, du, sl.w[j], true, q, mark, stamp);
      t = (uint32_t)sl.w[15];
      if (t == kInvalid) break;
    }
  }
  // other light vertices: one 16-lane group each
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  for (uint32_t i = g0; i < nl; i += ng) {
    const uint32_t u = q.cur[0][i];
    if (F.nbk[u] == 1) continue;
    const uint64_t du = ld_u64_coherent(D + u) >> 32;
    for_each_slab(F, u, [&](uint64_t x, bool data) { relax_word<kUnit>(F, D, u, du, x, data, q, mark, stamp); });
  }
  const uint32_t gib = threadIdx.x / kGroup;
  for (uint32_t j = blockIdx.x; j < nh; j += gridDim.x) {
    const uint32_t u = q.cur[1][j];
    const uint64_t du = ld_u64_coherent(D + u) >> 32;
    for_each_slab_strided(F, u, gib, kGroupsPerBlock, [&](uint64_t x, bool data) {
      relax_word<kUnit>(F, D, u, du, x, data, q, mark, stamp);
    });
  }
  for (uint32_t it = g0; it < ngi * kGiantSplit; it += ng) {  // giant: kGiantSplit groups each
    const uint32_t u = q.cur[2][it / kGiantSplit];
    const uint64_t du = ld_u64_coherent(D + u) >> 32;
    for_each_slab_strided(F, u, it % kGiantSplit, kGiantSplit, [&](uint64_t x, bool data) {
      relax_word<kUnit>(F, D, u, du, x, data, q, mark, stamp);
    });
  }
}

__global__ void k_trav_init(uint64_t* D, uint32_t nv, uint32_t src) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x)
    D[v] = v == src ? (uint64_t)src : kTreeNone;
}

// Reset the rotating counters so that slot 0 is the current frontier.
__global__ void k_queue_reset(uint32_t* cnt, uint32_t* inval_cnt) {
  if (threadIdx.x < 9) cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0 && inval_cnt) *inval_cnt = 0;
}

__global__ void k_seed_source(DView F, uint32_t src, PushQ Q, uint32_t* mark, uint32_t stamp) {
  if (threadIdx.x != 0) return;
  mark[src] = stamp;
  const uint32_t nb = F.nbk[src];
  const int k = nb <= kHeavyBuckets ? 0 : (nb <= kGiantBuckets ? 1 : 2);
  Q.q[k][0] = src;
  *Q.c[k] = 1;
}

// Insert prologue: relax each effective inserted arc.
template <bool kUnit>
__global__ void k_relax_batch(DView F, uint64_t* D, Log lg, uint64_t n, PushQ Q, uint32_t* mark,
                              uint32_t stamp) {
  // whole waves step together so that the wave-wide push sees every lane
  const uint64_t lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; base < n;
       base += stride) {
    const uint64_t i = base + lane;
    bool improve = false;
    uint32_t v = 0;
    if (i < n && lg.st[i] == 1) {
      const uint32_t u = lg.s[i];
      v = lg.d[i];
      const uint64_t du = ld_u64_coherent(D + u);
      if (du != kTreeNone) {
        const uint64_t cand = tree_node((du >> 32) + (kUnit ? 1u : lg.w[i]), u);
        if (cand < D[v]) improve = amin64(D + v, cand) > cand;
      }
    }
    push_vertex(F.nbk, Q, mark, stamp, improve, v);
  }
}

// Delete prologue, step 1: a deleted arc (u, v) of the dependence tree invalidates v.
__global__ void k_invalidate(DView F, uint64_t* D, Log lg, uint64_t n, PushQ Q, uint32_t* inval,
                             uint32_t* inval_cnt, uint32_t* mark, uint32_t stamp) {
  const uint64_t lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; base < n;
       base += stride) {
    const uint64_t i = base + lane;
    bool hit = false;
    uint32_t v = 0;
    if (i < n && lg.st[i] == 1) {
      const uint32_t u = lg.s[i];
      v = lg.d[i];
      const uint64_t dv = ld_u64_coherent(D + v);
      if (dv != kTreeNone && (uint32_t)dv == u) hit = cas64(D + v, dv, kTreeNone) == dv;
    }
    wave_push(inval, inval_cnt, hit, v);
    push_vertex(F.nbk, Q, mark, stamp, hit, v);
  }
}

// Delete prologue, step 2: invalidate the subtree below each invalidated vertex x (its
// tree children are the out-neighbours y whose parent is x).
__device__ inline void inval_word(const DView& F, uint64_t* D, uint32_t x_parent, uint64_t w,
                                  bool data, const Queues& q, uint32_t* inval, uint32_t* inval_cnt,
                                  uint32_t* mark, uint32_t stamp) {
  const uint32_t y = (uint32_t)w;
  bool hit = false;
  if (data && valid_key(y)) {
    const uint64_t dy = ld_u64_coherent(D + y);
    if (dy != kTreeNone && (uint32_t)dy == x_parent) hit = cas64(D + y, dy, kTreeNone) == dy;
  }
  wave_push(inval, inval_cnt, hit, y);
  push_vertex(F.nbk, q.next, mark, stamp, hit, y);
}

__global__ void __launch_bounds__(kBlock) k_propagate(DView F, uint64_t* D, Queues q, uint32_t* inval,
                                                      uint32_t* inval_cnt, uint32_t* mark,
                                                      uint32_t stamp) {
  const uint32_t nl = q.cnt[q.icur], nh = q.cnt[3 + q.icur], ngi = q.cnt[6 + q.icur];
  if (blockIdx.x == 0 && threadIdx.x < 3) q.cnt[3 * threadIdx.x + q.iclear] = 0;
  if (nl == 0 && nh == 0 && ngi == 0) return;
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  for (uint32_t i = g0; i < nl; i += ng) {
    const uint32_t x = q.cur[0][i];
    for_each_slab(F, x, [&](uint64_t w, bool data) {
      inval_word(F, D, x, w, data, q, inval, inval_cnt, mark, stamp);
    });
  }
  const uint32_t gib = threadIdx.x / kGroup;
  for (uint32_t j = blockIdx.x; j < nh; j += gridDim.x) {
    const uint32_t x = q.cur[1][j];
    for_each_slab_strided(F, x, gib, kGroupsPerBlock, [&](uint64_t w, bool data) {
      inval_word(F, D, x, w, data, q, inval, inval_cnt, mark, stamp);
    });
  }
  for (uint32_t it = g0; it < ngi * kGiantSplit; it += ng) {
    const uint32_t x = q.cur[2][it / kGiantSplit];
    for_each_slab_strided(F, x, it % kGiantSplit, kGiantSplit, [&](uint64_t w, bool data) {
      inval_word(F, D, x, w, data, q, inval, inval_cnt, mark, stamp);
    });
  }
}

// Delete prologue, step 3: each invalidated vertex takes the best candidate offered by
// its still-valid in-neighbours (reverse view) and, if reached, joins the frontier.
template <bool kUnit>
__global__ void __launch_bounds__(kBlock) k_dec_pull(DView F, DView R, uint64_t* D,
                                                     const uint32_t* inval, const uint32_t* inval_cnt,
                                                     PushQ Q, uint32_t* mark, uint32_t stamp) {
  const uint32_t n = *inval_cnt;
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  for (uint32_t i = g0; i < n; i += ng) {
    const uint32_t y = inval[i];
    uint64_t best = kTreeNone;
    for_each_slab(R, y, [&](uint64_t x, bool data) {
      const uint32_t u = (uint32_t)x;
      if (data && valid_key(u)) {
        const uint64_t du = ld_u64_coherent(D + u);
        if (du != kTreeNone) {
          const uint64_t cand = tree_node((du >> 32) + (kUnit ? 1ull : (x >> 32)), u);
          best = cand < best ? cand : best;
        }
      }
    });
    best = gmin_u64(best);
    bool improve = false;
    if (glane() == 0 && best != kTreeNone) improve = amin64(D + y, best) > best;
    push_vertex(F.nbk, Q, mark, stamp, improve, y);
  }
}

__global__ void k_fill_mark(uint32_t* mark, uint32_t nv) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) mark[v] = 0;
}

__global__ void k_split(const uint64_t* D, uint32_t nv, uint32_t* dist, uint32_t* parent) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    const uint64_t x = D[v];
    dist[v] = (uint32_t)(x >> 32);
    if (parent) parent[v] = (uint32_t)x;
  }
}

inline uint32_t blocks_for(uint64_t n, uint32_t cap = 4096) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + kBlock - 1) / kBlock, cap));
}

// Where a traversal keeps its state: the graph's own arrays for the maintained BFS/SSSP,
// or a caller workspace for a one-off traversal that other reads may overlap.
struct TravCtx {
  uint64_t* D;
  uint32_t* fq[6];  // light, heavy and giant queues, two of each
  uint32_t* mark;
  uint32_t* inval;
  uint32_t* cnt;        // rotating frontier sizes [9]
  uint32_t* inval_cnt;  // invalidated-list size
  uint32_t* stamp;      // host-side stamp counter
  uint64_t* h_pin;      // pinned host words for size read-backs
};

TravCtx graph_ctx(mk_graph* g, uint64_t* D) {
  TravCtx c;
  c.D = D;
  for (int i = 0; i < 6; ++i) c.fq[i] = g->fq[i];
  c.mark = g->mark;
  c.inval = g->inval;
  c.cnt = g->ctr->frontier;
  c.inval_cnt = &g->ctr->inval;
  c.stamp = &g->stamp;
  c.h_pin = g->h_pin;
  return c;
}

// The queues of iteration 0 (and of every prologue): fq[0], fq[2], fq[4] with slot 0.
PushQ first_push(const TravCtx& c) {
  PushQ Q;
  for (int k = 0; k < 3; ++k) {
    Q.q[k] = c.fq[2 * k];
    Q.c[k] = c.cnt + 3 * k;
  }
  return Q;
}

Queues queues(const TravCtx& c, uint64_t it) {
  Queues q;
  const int a = (int)(it & 1);
  const int inext = (int)((it + 1) % 3);
  for (int k = 0; k < 3; ++k) {
    q.cur[k] = c.fq[2 * k + a];
    q.next.q[k] = c.fq[2 * k + (a ^ 1)];
    q.next.c[k] = c.cnt + 3 * k + inext;
  }
  q.cnt = c.cnt;
  q.icur = (int)(it % 3);
  q.iclear = (int)((it + 2) % 3);
  return q;
}

// Run frontier iterations (expand or propagate) until the frontier is empty.  Iteration
// `it` reads slot it%3; the frontier of iteration 0 sits in fq[0] / fq[2] and slot 0.
template <class Launch>
mk_status run_frontier(mk_graph* g, const TravCtx& c, hipStream_t stream, Launch&& launch) {
  uint64_t it = 0;
  while (true) {
    for (int k = 0; k < kSyncEvery; ++k, ++it) {
      launch(queues(c, it), ++*c.stamp);
      MK_LAUNCH(g, "frontier kernel");
    }
    const int slot = (int)(it % 3);
    MK_HIP(g, hipMemcpyAsync(c.h_pin, c.cnt, 9 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    MK_HIP(g, hipStreamSynchronize(stream));
    const uint32_t* h = reinterpret_cast<const uint32_t*>(c.h_pin);
    if (h[slot] == 0 && h[3 + slot] == 0 && h[6 + slot] == 0) break;
  }
  return MK_OK;
}

template <bool kUnit>
mk_status run_expand(mk_graph* g, const TravCtx& c, hipStream_t stream) {
  const DView F = g->view[VF].d;
  return run_frontier(g, c, stream, [&](Queues q, uint32_t stamp) {
    hipLaunchKernelGGL(k_expand<kUnit>, dim3(kExpandBlocks), dim3(kBlock), 0, stream, F, c.D, q, c.mark,
                       stamp);
  });
}

template <bool kUnit>
mk_status static_from(mk_graph* g, const TravCtx& c, uint32_t source, hipStream_t stream) {
  const DView F = g->view[VF].d;
  const uint32_t stamp0 = ++*c.stamp;
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, stream, c.cnt, c.inval_cnt);
  hipLaunchKernelGGL(k_trav_init, dim3(blocks_for(g->n)), dim3(kBlock), 0, stream, c.D, g->n, source);
  hipLaunchKernelGGL(k_seed_source, dim3(1), dim3(64), 0, stream, F, source, first_push(c), c.mark,
                     stamp0);
  MK_LAUNCH(g, "traversal init");
  return run_expand<kUnit>(g, c, stream);
}

template <bool kUnit>
mk_status traverse(mk_graph* g, AlgoState& st, uint64_t* D, uint32_t source, uint32_t* d_out,
                   uint32_t* d_parent, mk_mode mode, hipStream_t stream) {
  if (source >= g->n || !d_out) return MK_ERR_INVALID_ARG;
  const DView F = g->view[VF].d;
  const uint32_t N = g->n;
  const TravCtx c = graph_ctx(g, D);
  Pending p = pending_for(g, st);
  const bool can_dec = g->view[VR].on;
  const bool full = mode == MK_RECOMPUTE || !st.valid || st.source != source || p.lost ||
                    p.kinds == 3 || (p.kinds == 2 && !can_dec);
  if (full) {
    mk_status s = static_from<kUnit>(g, c, source, stream);
    if (s != MK_OK) return s;
  } else if (!p.list.empty()) {
    const uint32_t stamp0 = ++g->stamp;
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, stream, c.cnt, c.inval_cnt);
    if (p.kinds == 1) {
      for (const BatchRec* b : p.list) {
        Log lg = g->log;
        lg.s += b->off; lg.d += b->off; lg.w += b->off; lg.st += b->off; lg.uf += b->off;
        hipLaunchKernelGGL(k_relax_batch<kUnit>, dim3(blocks_for(b->n)), dim3(kBlock), 0, stream, F, D,
                           lg, b->n, first_push(c), c.mark, stamp0);
      }
    } else {  // deletions only
      for (const BatchRec* b : p.list) {
        Log lg = g->log;
        lg.s += b->off; lg.d += b->off; lg.w += b->off; lg.st += b->off; lg.uf += b->off;
        hipLaunchKernelGGL(k_invalidate, dim3(blocks_for(b->n)), dim3(kBlock), 0, stream, F, D, lg, b->n,
                           first_push(c), c.inval, c.inval_cnt, c.mark, stamp0);
      }
      MK_LAUNCH(g, "k_invalidate");
      mk_status s = run_frontier(g, c, stream, [&](Queues q, uint32_t stamp) {
        hipLaunchKernelGGL(k_propagate, dim3(kExpandBlocks), dim3(kBlock), 0, stream, F, D, q, c.inval,
                           c.inval_cnt, c.mark, stamp);
      });
      if (s != MK_OK) return s;
      hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, stream, c.cnt, nullptr);
      const uint32_t stamp1 = ++g->stamp;
      hipLaunchKernelGGL(k_dec_pull<kUnit>, dim3(kExpandBlocks), dim3(kBlock), 0, stream, F,
                         g->view[VR].d, D, c.inval, c.inval_cnt, first_push(c), c.mark, stamp1);
    }
    MK_LAUNCH(g, "traversal prologue");
    mk_status s = run_expand<kUnit>(g, c, stream);
    if (s != MK_OK) return s;
  }
  hipLaunchKernelGGL(k_split, dim3(blocks_for(N)), dim3(kBlock), 0, stream, D, N, d_out, d_parent);
  MK_LAUNCH(g, "k_split");
  st.valid = true;
  st.source = source;
  mark_seen(g, st);
  return MK_OK;
}

size_t ws_bytes_for(uint32_t n) {
  // D (8 B), six queues, stamps and the invalidated list (4 B each), counters
  return (size_t)n * (8 + 8 * 4) + 512 + 10 * 256;
}

}  // namespace

extern "C" {

mk_status mk_incr_bfs(mk_graph* g, uint32_t source, uint32_t* d_level, uint32_t* d_parent,
                      mk_mode mode, hipStream_t stream) {
  if (!g) return MK_ERR_INVALID_ARG;
  return traverse<true>(g, g->bfs, g->bfs_D, source, d_level, d_parent, mode, stream);
}

mk_status mk_incr_sssp(mk_graph* g, uint32_t source, uint32_t* d_dist, uint32_t* d_parent,
                       mk_mode mode, hipStream_t stream) {
  if (!g) return MK_ERR_INVALID_ARG;
  return traverse<false>(g, g->sssp, g->sssp_D, source, d_dist, d_parent, mode, stream);
}

size_t mk_traversal_workspace_bytes(const mk_graph* g) { return g ? ws_bytes_for(g->n) : 0; }

mk_status mk_traverse_from(mk_graph* g, uint32_t source, int weighted, void* d_ws, size_t ws_bytes,
                           uint32_t slot, uint32_t* d_dist, uint32_t* d_parent, hipStream_t stream) {
  if (!g || !d_ws || !d_dist || source >= g->n || slot >= kSlots) return MK_ERR_INVALID_ARG;
  if (ws_bytes < ws_bytes_for(g->n)) return MK_ERR_CAPACITY;
  if (!g->slot_pin[slot]) {
    if (hipHostMalloc((void**)&g->slot_pin[slot], 64 * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess)
      return MK_ERR_HIP;
  }
  const uint32_t N = g->n;
  char* p = reinterpret_cast<char*>(((uintptr_t)d_ws + 255) & ~uintptr_t(255));
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~size_t(255);
    return r;
  };
  TravCtx c;
  c.D = reinterpret_cast<uint64_t*>(take((size_t)N * 8));
  for (int i = 0; i < 6; ++i) c.fq[i] = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  c.mark = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  c.inval = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  c.cnt = reinterpret_cast<uint32_t*>(take(64));
  c.inval_cnt = c.cnt + 12;
  uint32_t stamp = 0;
  c.stamp = &stamp;
  c.h_pin = g->slot_pin[slot];
  hipLaunchKernelGGL(k_fill_mark, dim3(blocks_for(N)), dim3(kBlock), 0, stream, c.mark, N);
  mk_status s = weighted ? static_from<false>(g, c, source, stream) : static_from<true>(g, c, source, stream);
  if (s != MK_OK) return s;
  hipLaunchKernelGGL(k_split, dim3(blocks_for(N)), dim3(kBlock), 0, stream, c.D, N, d_dist, d_parent);
  MK_LAUNCH(g, "k_split");
  return MK_OK;
}

}  // extern "C"
