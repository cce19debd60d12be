// Distance-only ("vanilla") traversals: BFS levels, level-synchronous and
// direction-optimizing, and SSSP distances by near-far relaxation (further down).
//
// The experimental section runs BFS in two variants: a vanilla one with 32-bit atomics that
// computes only distances, and the tree variant (64-bit <distance, parent> nodes) that the
// dynamic algorithms need; its static BFS is level-based.  This file is the vanilla variant:
// one u32 level per vertex, one level per step.  A step is either top-down (the frontier's
// out-arcs claim unreached vertices by CAS) or bottom-up (every unreached vertex scans its
// in-arcs, through the reverse view, for a vertex of the current level and stops at the
// first one).  A one-thread kernel picks the direction of each step on the device from the
// frontier's size and out-arc count against the number of unreached vertices, so the host
// only reads sizes back after 4, 8, 16 and 32 levels, then every 16.
//
// The rule is Beamer's direction optimization recast for slabs.  A top-down step reads a slab
// per frontier vertex and makes a random level read (and, for an unreached target, a CAS) per
// out-arc; a bottom-up step reads at least one slab per unreached vertex and a level per
// in-arc it scans until it meets the current level, and every bottom-up step also reads the
// level of every vertex.  Counting a slab as two random accesses, bottom-up is taken when
// 2 nf + mf > 6 nu + N / 2  (nf, mf: frontier vertices and out-arcs; nu: unreached
// vertices).  On a power-law graph the hub's neighbourhood passes this at once (few vertices,
// very many arcs).  On a road network the frontier has as few arcs per vertex as the
// unreached part and most unreached vertices find no parent, so bottom-up steps there cost
// more than top-down ones (measured); the N / 2 term keeps such a graph top-down.
#include <rocprim/device/device_scan.hpp>

#include <algorithm>

#include "mk_internal.h"

using namespace mk;

namespace {

constexpr uint32_t kLevelInf = 0xFFFFFFFFu;
constexpr uint32_t kChunk = kGroup;       // buckets of a multi-bucket vertex per work item
constexpr uint32_t kSyncFirst = 4, kSyncMax = 16;  // steps between size read-backs: 4, 4,
                                                    // then doubling while the traversal lasts

// Device counters of one call (in the caller's workspace).  Level L uses slot L mod 4.
struct LvCnt {
  uint32_t n[4];                // frontier sizes
  uint32_t nm[4];               // multi-bucket work items of the level's top-down step
  uint32_t mode;                // direction of the current step: 0 top-down, 1 bottom-up
  uint32_t bu_steps;            // bottom-up steps taken
  uint32_t reached;             // vertices reached before the current frontier
  uint32_t pad[5];
  unsigned long long arcs[4];   // out-arcs of each frontier
};
static_assert(sizeof(LvCnt) <= 256, "counter block");

__global__ void k_lv_fill(uint32_t* level, uint32_t nv) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x)
    level[v] = kLevelInf;
}

__global__ void k_zero_marks(uint32_t* a, uint32_t* b, uint32_t nv) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    a[v] = 0;
    b[v] = 0;
  }
}

__global__ void k_lv_clear(LvCnt* c) {
  uint32_t* w = reinterpret_cast<uint32_t*>(c);
  for (uint32_t i = threadIdx.x; i < sizeof(LvCnt) / 4; i += blockDim.x) w[i] = 0;
}

__global__ void k_lv_seed(uint32_t* level, uint32_t* q0, LvCnt* c, const uint32_t* deg, uint32_t src) {
  if (threadIdx.x != 0) return;
  level[src] = 0;
  q0[0] = src;
  c->n[0] = 1;
  c->arcs[0] = deg[src];
  c->mode = 0;
  c->reached = 0;
}

// Direction of level L's step, and the counters it fills.
__global__ void k_lv_decide(LvCnt* c, uint32_t L, uint32_t nv, int allow_bu) {
  if (threadIdx.x != 0) return;
  const uint32_t s = L & 3, nx = (L + 1) & 3;
  c->n[nx] = 0;
  c->arcs[nx] = 0;
  c->nm[s] = 0;
  const uint64_t nf = c->n[s], mf = c->arcs[s];
  if (L > 0) c->reached += c->n[(L - 1) & 3];
  const uint64_t nu = (uint64_t)nv - c->reached - nf;
  const uint32_t mode = allow_bu && nu > 0 && 2 * nf + mf > 6 * nu + nv / 2 ? 1u : 0u;
  c->mode = mode;
  if (nf) c->bu_steps += mode;
}

// Append the words of `sl` flagged in `found` (<= 15) to the staged next frontier.
__device__ inline void push_found(Stage& S, uint32_t found, const Slab& sl) {
  bool any;
  const StageSlots t = stage_reserve(S, (uint32_t)__popc(found), any);
  if (!any) return;
  uint32_t k = 0;
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j)
    if (found >> j & 1) stage_put(S, t, t.pos + k++, (uint32_t)sl.w[j]);
}

// Top-down on one slab: claim every unreached neighbour for level cur + 1 (the CAS winner
// pushes it and counts its out-arcs).
__device__ inline uint32_t claim_slab(const Slab& sl, int nd, uint32_t* level, const uint32_t* deg,
                                      uint32_t cur, unsigned long long& arcs) {
  uint32_t lv[kKeysPerSlab];
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j) {
    const uint32_t v = (uint32_t)sl.w[j];
    lv[j] = (j < nd && valid_key(v)) ? ld_u32(level + v) : 0u;
  }
  uint32_t found = 0;
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j) {
    const uint32_t v = (uint32_t)sl.w[j];
    if (lv[j] == kLevelInf && atomicCAS(level + v, kLevelInf, cur + 1) == kLevelInf) {
      found |= 1u << j;
      arcs += deg[v];
    }
  }
  return found;
}

// Wave-wide exclusive prefix of k and one atomic per wave on *ctr: this lane's first slot.
__device__ inline uint32_t wave_reserve(uint32_t* ctr, uint32_t k) {
  const int lane = lane64();
  uint32_t incl = k;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  const uint32_t total = __shfl(incl, 63);
  uint32_t base = 0;
  if (lane == 63 && total) base = atomicAdd(ctr, total);
  base = __shfl(base, 63);
  return base + incl - k;
}

__device__ inline void block_add(unsigned long long* acc, unsigned long long v, unsigned long long* out) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(acc, v);
  __syncthreads();
  if (threadIdx.x == 0 && *acc) atomicAdd(out, *acc);
}

// Top-down step, single-bucket frontier vertices: a lane walks its vertex's chain.  A vertex
// with several buckets becomes ceil(nb / 16) work items for k_lv_td_multi.
__global__ void __launch_bounds__(kBlock) k_lv_td(DView F, LvCnt* c, uint32_t L, uint32_t* level,
                                                  const uint32_t* fin, uint32_t* fout, uint32_t* mu_,
                                                  uint32_t* mc_) {
  const uint32_t s = L & 3;
  if (c->mode != 0) return;
  const uint32_t n = c->n[s];
  if (n == 0) return;
  __shared__ Stage S[1];
  __shared__ unsigned long long acc;
  stage_open(S[0], fout, &c->n[(L + 1) & 3]);
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  unsigned long long arcs = 0;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
    const uint32_t i = base + threadIdx.x;
    uint32_t u = 0, nb = 0;
    if (i < n) {
      u = fin[i];
      nb = F.nbk[u];
    }
    const uint32_t k = nb > 1 ? (nb + kChunk - 1) / kChunk : 0u;
    const uint32_t pos = wave_reserve(&c->nm[s], k);
    for (uint32_t j = 0; j < k; ++j) {
      mu_[pos + j] = u;
      mc_[pos + j] = j;
    }
    bool active = i < n && nb == 1 && F.deg[u] > 0;
    uint32_t t = u;
    while (__ballot(active)) {
      Slab sl;
      uint32_t found = 0;
      if (active) {
        load_slab(F, t, sl);
        found = claim_slab(sl, kKeysPerSlab, level, F.deg, L, arcs);
        t = (uint32_t)sl.w[15];
        active = t != kInvalid;
      }
      push_found(S[0], found, sl);
    }
  }
  stage_close(S);
  block_add(&acc, arcs, &c->arcs[(L + 1) & 3]);
}

// Top-down step, multi-bucket frontier vertices: a 16-lane group per work item (16 buckets),
// a lane per bucket chain.
__global__ void __launch_bounds__(kBlock) k_lv_td_multi(DView F, LvCnt* c, uint32_t L, uint32_t* level,
                                                        uint32_t* fout, const uint32_t* mu_,
                                                        const uint32_t* mc_) {
  const uint32_t s = L & 3;
  if (c->mode != 0) return;
  const uint32_t nm = c->nm[s];
  if (nm == 0) return;
  __shared__ Stage S[1];
  __shared__ unsigned long long acc;
  stage_open(S[0], fout, &c->n[(L + 1) & 3]);
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  unsigned long long arcs = 0;
  const uint32_t gib = threadIdx.x / kGroup;
  for (uint32_t base = blockIdx.x * kGroupsPerBlock; base < nm; base += gridDim.x * kGroupsPerBlock) {
    const uint32_t it = base + gib;  // one item per 16-lane group, a lane per bucket
    uint32_t u = 0, nb = 0, xb = 0, b = 0;
    if (it < nm) {
      u = mu_[it];
      nb = (uint32_t)(slab_ptr(F, u)[15] >> 32);
      xb = (uint32_t)slab_ptr(F, u)[14];
      b = mc_[it] * kChunk + glane();
    }
    bool active = it < nm && b < nb;
    uint32_t t = b == 0 ? u : xb + b - 1;
    int nd = b == 0 ? kKeysPerSlab - 1 : kKeysPerSlab;
    while (__ballot(active)) {
      Slab sl;
      uint32_t found = 0;
      if (active) {
        load_slab(F, t, sl);
        found = claim_slab(sl, nd, level, F.deg, L, arcs);
        t = (uint32_t)sl.w[15];
        nd = kKeysPerSlab;
        active = t != kInvalid;
      }
      push_found(S[0], found, sl);
    }
  }
  stage_close(S);
  block_add(&acc, arcs, &c->arcs[(L + 1) & 3]);
}

// Does some in-neighbour of v (reverse view) sit on level cur?  A lane walks v's buckets
// and stops at the first slab that holds one.
__device__ inline bool has_parent_at(const DView& R, uint32_t v, const uint32_t* level, uint32_t cur) {
  Slab sl;
  load_slab(R, v, sl);
  const uint32_t nb = (uint32_t)(sl.w[15] >> 32);
  const uint32_t xb = nb > 1 ? (uint32_t)sl.w[14] : 0u;
  int nd = nb > 1 ? kKeysPerSlab - 1 : kKeysPerSlab;
  for (uint32_t b = 0; b < nb; ++b) {
    if (b > 0) {
      load_slab(R, xb + b - 1, sl);
      nd = kKeysPerSlab;
    }
    while (true) {
      uint32_t lv[kKeysPerSlab];
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j) {
        const uint32_t u = (uint32_t)sl.w[j];
        lv[j] = (j < nd && valid_key(u)) ? ld_u32(level + u) : kLevelInf;
      }
      bool hit = false;
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j) hit |= lv[j] == cur;
      if (hit) return true;
      const uint32_t t = (uint32_t)sl.w[15];
      if (t == kInvalid) break;
      load_slab(R, t, sl);
      nd = kKeysPerSlab;
    }
  }
  return false;
}

// Bottom-up step: every unreached vertex with in-arcs looks for a parent on level L.  Only
// the vertex's own lane writes its level, and no level changes to L during the step.
__global__ void __launch_bounds__(kBlock) k_lv_bu(DView F, DView R, LvCnt* c, uint32_t L, uint32_t* level,
                                                  uint32_t* fout, uint32_t nv) {
  const uint32_t s = L & 3;
  if (c->mode != 1 || c->n[s] == 0) return;
  __shared__ Stage S[1];
  __shared__ unsigned long long acc;
  stage_open(S[0], fout, &c->n[(L + 1) & 3]);
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  unsigned long long arcs = 0;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < nv; base += stride) {
    const uint32_t v = base + threadIdx.x;
    bool found = false;
    if (v < nv && ld_u32(level + v) == kLevelInf && R.deg[v] > 0 && has_parent_at(R, v, level, L)) {
      level[v] = L + 1;
      arcs += F.deg[v];
      found = true;
    }
    stage_push(S[0], found, v);
  }
  stage_close(S);
  block_add(&acc, arcs, &c->arcs[(L + 1) & 3]);
}

inline uint32_t blocks_for(uint64_t n, uint32_t cap) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + kBlock - 1) / kBlock, cap));
}

size_t levels_ws_bytes(const mk_graph* g) {
  return 256 + 2 * ((size_t)g->n * 4 + 256) + 2 * (levels_multi_cap(g) * 4 + 256) + 256;
}

// ----------------------------------------------------------------- tree nodes from levels
// <level, INVALID> for every reached vertex but the source (<0, source>); unreached ones
// get <INF, INVALID>.
__global__ void k_lv_tree_init(const uint32_t* level, uint64_t* D, uint32_t nv, uint32_t src) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    const uint32_t lv = level[v];
    D[v] = lv == kLevelInf ? kTreeNone : v == src ? (uint64_t)src : ((uint64_t)lv << 32) | kInvalid;
  }
}

// Reached vertices (other than the source) with more than kHeavyBuckets buckets in the
// reverse view, and their work items of kPrItem buckets.
constexpr uint32_t kPrItem = 4;
__global__ void k_lv_heavy(const uint32_t* nbk, const uint32_t* level, uint32_t nv, uint32_t src,
                           uint32_t* out, uint32_t* cnt) {
  __shared__ Stage S[1];
  stage_open(S[0], out, cnt);
  __syncthreads();
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < nv; base += stride) {
    const uint32_t v = base + threadIdx.x;
    stage_push(S[0], v < nv && v != src && nbk[v] > kHeavyBuckets && level[v] != kLevelInf, v);
  }
  stage_close(S);
}

__global__ void k_lv_items(const uint32_t* nbk, const uint32_t* heavy, const uint32_t* nheavy, uint32_t* cnt) {
  const uint32_t nh = *nheavy;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nh; j += gridDim.x * blockDim.x)
    cnt[j] = (nbk[heavy[j]] + kPrItem - 1) / kPrItem;
}

// Is u (distance du, arc weight w) a parent of a vertex at distance dv: du + w == dv, with
// the sum saturated below INF as the tree traversal does; BFS counts every arc as 1.
template <bool kUnit>
__device__ inline bool parent_arc(uint32_t du, uint64_t word, uint32_t dv) {
  if (du == kLevelInf) return false;
  const uint64_t w = kUnit ? 1ull : (word >> 32);
  return (uint32_t)min<uint64_t>((uint64_t)du + w, 0xFFFFFFFEull) == dv;
}

// Parent of every reached vertex: the smallest in-neighbour u with dist(u) + w(u, v) =
// dist(v) (the parent rule of the tree variant).  One lane per single-bucket vertex, a
// 16-lane group per vertex of 2 .. kHeavyBuckets buckets, and the heavy vertices' bucket
// items spread over every group, which fold their minima in with a 64-bit atomic minimum.
template <bool kUnit>
__global__ void __launch_bounds__(kBlock) k_lv_parents(DView R, const uint32_t* level, uint64_t* D, uint32_t nv,
                                                       uint32_t src, const uint32_t* heavy,
                                                       const uint32_t* nheavy, const uint32_t* hoff,
                                                       const uint32_t* hcnt) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    if (R.nbk[v] != 1 || v == src) continue;
    const uint32_t lv = level[v];
    if (lv == kLevelInf) continue;
    uint32_t best = kInvalid, t = v;
    Slab sl;
    while (true) {
      load_slab(R, t, sl);
      uint32_t lu[kKeysPerSlab];
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j) {
        const uint32_t u = (uint32_t)sl.w[j];
        lu[j] = valid_key(u) ? level[u] : kLevelInf;
      }
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j)
        if (parent_arc<kUnit>(lu[j], sl.w[j], lv)) best = min(best, (uint32_t)sl.w[j]);
      t = (uint32_t)sl.w[15];
      if (t == kInvalid) break;
    }
    D[v] = ((uint64_t)lv << 32) | best;
  }
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  for (uint32_t v = g0; v < nv; v += ng) {
    const uint32_t nb = R.nbk[v];
    if (nb == 1 || nb > kHeavyBuckets || v == src) continue;
    const uint32_t lv = level[v];
    if (lv == kLevelInf) continue;
    uint64_t best = kTreeNone;
    for_each_slab(R, v, [&](uint64_t w, bool data) {
      const uint32_t u = (uint32_t)w;
      if (data && valid_key(u) && parent_arc<kUnit>(level[u], w, lv)) best = min(best, (uint64_t)u);
    });
    best = gmin_u64(best);
    if (glane() == 0) D[v] = ((uint64_t)lv << 32) | (uint32_t)best;
  }
  const uint32_t nh = *nheavy;
  if (nh == 0) return;
  const uint32_t items = hoff[nh - 1] + hcnt[nh - 1];
  for (uint32_t it = g0; it < items; it += ng) {
    uint32_t lo = 0, hi = nh;  // the last j with hoff[j] <= it
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (hoff[mid] <= it) lo = mid;
      else hi = mid;
    }
    const uint32_t v = heavy[lo];
    const uint32_t lv = level[v];
    const uint32_t b0 = (it - hoff[lo]) * kPrItem;
    uint64_t best = kTreeNone;
    for_each_bucket_range(R, v, b0, b0 + kPrItem, [&](uint64_t w, bool data) {
      const uint32_t u = (uint32_t)w;
      if (data && valid_key(u) && parent_arc<kUnit>(level[u], w, lv)) best = min(best, (uint64_t)u);
    });
    best = gmin_u64(best);
    if (glane() == 0 && best != kTreeNone) amin64(D + v, ((uint64_t)lv << 32) | best);
  }
}


// ----------------------------------------------------------------- distance-only SSSP
// The vanilla SSSP: one u32 distance per vertex relaxed by 32-bit atomic minimum, no
// parents.  Scheduling is near-far: a relaxed vertex whose new distance is below the band
// limit T joins the next near frontier, any other the far pile; when the near frontier runs
// dry, the far pile is split at T = (its smallest distance) + delta.  Every decision is made
// on the device, so the host only reads sizes back every few steps.  Any schedule reaches the
// same distances (label correcting), so the band width only changes the work.
struct DsCnt {
  uint32_t n[4];     // near frontier sizes by step mod 4
  uint32_t nm[4];    // multi-bucket work items by step mod 4
  uint32_t nfar[2];  // far pile sizes
  uint32_t fpar;     // index of the current far pile
  uint32_t T;        // band limit
  uint32_t band;     // band number (far-pile duplicate stamps)
  uint32_t fmin;     // smallest distance on the far pile (before a split)
  uint32_t done;     // blocks of the running split that have finished
  uint32_t pad[5];
};
static_assert(sizeof(DsCnt) <= 256, "counter block");

__global__ void k_ds_seed(uint32_t* dist, uint32_t* q0, DsCnt* c, uint32_t src, uint32_t delta) {
  if (threadIdx.x != 0) return;
  dist[src] = 0;
  q0[0] = src;
  c->n[0] = 1;
  c->T = delta;
  c->band = 1;
  c->fmin = kLevelInf;
}

// Relax one slab of u (distance du): a neighbour whose distance drops goes to the near
// frontier (once per step, by the step stamp) or to the far pile (once per band).
__device__ inline void relax_ds(const Slab& sl, int nd, uint32_t du, uint32_t* dist, uint32_t* mark,
                                uint32_t* fmark, uint32_t stamp, uint32_t band, uint32_t T, uint32_t& near,
                                uint32_t& far) {
  uint32_t dv[kKeysPerSlab];
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j) {
    const uint32_t v = (uint32_t)sl.w[j];
    dv[j] = (j < nd && valid_key(v)) ? ld_u32(dist + v) : 0u;
  }
  near = far = 0;
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j) {
    const uint32_t v = (uint32_t)sl.w[j];
    const uint32_t nd_ = (uint32_t)min<uint64_t>((uint64_t)du + (sl.w[j] >> 32), 0xFFFFFFFEull);
    if (nd_ < dv[j] && nd_ < atomicMin(dist + v, nd_)) {
      if (nd_ < T) {
        if (atomicExch(mark + v, stamp) != stamp) near |= 1u << j;
      } else if (atomicExch(fmark + v, band) != band) {
        far |= 1u << j;
      }
    }
  }
}

__device__ inline void wave_min_to(uint32_t* out, uint32_t m) {
  for (int o = 32; o > 0; o >>= 1) m = min(m, (uint32_t)__shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0 && m != kLevelInf) atomicMin(out, m);
}

struct DsArgs {
  uint32_t *dist, *mark, *fmark, *far[2], *multi_v, *multi_c;
};

// Near step, single-bucket frontier vertices (a lane each); others become 16-bucket items.
__global__ void __launch_bounds__(kBlock) k_ds_relax(DView F, DsCnt* c, uint32_t S, DsArgs a, const uint32_t* fin,
                                                     uint32_t* fout) {
  const uint32_t s = S & 3;
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // counters of the next step (unused in this one)
    c->n[(S + 2) & 3] = 0;
    c->nm[(S + 1) & 3] = 0;
  }
  const uint32_t n = c->n[s];
  if (n == 0) return;
  const uint32_t T = c->T, band = c->band, fp = c->fpar, stamp = S + 1;
  __shared__ Stage St[2];
  stage_open(St[0], fout, &c->n[(S + 1) & 3]);
  stage_open(St[1], a.far[fp], &c->nfar[fp]);
  __syncthreads();
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
    const uint32_t i = base + threadIdx.x;
    uint32_t u = 0, nb = 0, du = 0;
    if (i < n) {
      u = fin[i];
      nb = F.nbk[u];
      du = ld_u32(a.dist + u);
    }
    const uint32_t k = nb > 1 ? (nb + kChunk - 1) / kChunk : 0u;
    const uint32_t pos = wave_reserve(&c->nm[s], k);
    for (uint32_t j = 0; j < k; ++j) {
      a.multi_v[pos + j] = u;
      a.multi_c[pos + j] = j;
    }
    bool active = i < n && nb == 1 && F.deg[u] > 0;
    uint32_t t = u;
    while (__ballot(active)) {
      Slab sl;
      uint32_t nr = 0, fr = 0;
      if (active) {
        load_slab(F, t, sl);
        relax_ds(sl, kKeysPerSlab, du, a.dist, a.mark, a.fmark, stamp, band, T, nr, fr);
        t = (uint32_t)sl.w[15];
        active = t != kInvalid;
      }
      push_found(St[0], nr, sl);
      push_found(St[1], fr, sl);
    }
  }
  stage_close(St);
}

// Near step, multi-bucket frontier vertices: a 16-lane group per item, a lane per bucket.
__global__ void __launch_bounds__(kBlock) k_ds_relax_multi(DView F, DsCnt* c, uint32_t S, DsArgs a,
                                                           uint32_t* fout) {
  const uint32_t s = S & 3;
  const uint32_t nm = c->nm[s];
  if (nm == 0) return;
  const uint32_t T = c->T, band = c->band, fp = c->fpar, stamp = S + 1;
  __shared__ Stage St[2];
  stage_open(St[0], fout, &c->n[(S + 1) & 3]);
  stage_open(St[1], a.far[fp], &c->nfar[fp]);
  __syncthreads();
  const uint32_t gib = threadIdx.x / kGroup;
  for (uint32_t base = blockIdx.x * kGroupsPerBlock; base < nm; base += gridDim.x * kGroupsPerBlock) {
    const uint32_t it = base + gib;  // one item per 16-lane group, a lane per bucket
    uint32_t u = 0, du = 0, nb = 0, xb = 0, b = 0;
    if (it < nm) {
      u = a.multi_v[it];
      du = ld_u32(a.dist + u);
      nb = (uint32_t)(slab_ptr(F, u)[15] >> 32);
      xb = (uint32_t)slab_ptr(F, u)[14];
      b = a.multi_c[it] * kChunk + glane();
    }
    bool active = it < nm && b < nb;
    uint32_t t = b == 0 ? u : xb + b - 1;
    int nd = b == 0 ? kKeysPerSlab - 1 : kKeysPerSlab;
    while (__ballot(active)) {
      Slab sl;
      uint32_t nr = 0, fr = 0;
      if (active) {
        load_slab(F, t, sl);
        relax_ds(sl, nd, du, a.dist, a.mark, a.fmark, stamp, band, T, nr, fr);
        t = (uint32_t)sl.w[15];
        nd = kKeysPerSlab;
        active = t != kInvalid;
      }
      push_found(St[0], nr, sl);
      push_found(St[1], fr, sl);
    }
  }
  stage_close(St);
}

// When a step leaves the near frontier empty: the smallest distance on the far pile ...
__global__ void k_ds_far_min(DsCnt* c, uint32_t S, DsArgs a) {
  if (c->n[(S + 1) & 3] != 0) return;
  const uint32_t fp = c->fpar, nf = c->nfar[fp];
  uint32_t m = kLevelInf;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += gridDim.x * blockDim.x)
    m = min(m, ld_u32(a.dist + a.far[fp][i]));
  wave_min_to(&c->fmin, m);
}

// ... and the split at T' = fmin + delta: vertices below T' start the next near frontier,
// the others move to the other pile, stamped with the next band.  The last block to finish
// commits the new band limit, band number and pile (no block waits for another).
__global__ void k_ds_split(DsCnt* c, uint32_t S, DsArgs a, uint32_t* fout, uint32_t delta) {
  if (c->n[(S + 1) & 3] != 0) return;
  const uint32_t fp = c->fpar, nf = c->nfar[fp];
  if (nf == 0) return;
  const uint32_t T2 = (uint32_t)min<uint64_t>((uint64_t)c->fmin + delta, 0xFFFFFFFFull);
  const uint32_t nb = c->band + 1;
  __shared__ Stage St[2];
  __shared__ bool last;
  stage_open(St[0], fout, &c->n[(S + 1) & 3]);
  stage_open(St[1], a.far[fp ^ 1], &c->nfar[fp ^ 1]);
  __syncthreads();
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < nf; base += stride) {
    const uint32_t i = base + threadIdx.x;
    bool to_near = false, keep = false;
    uint32_t v = 0;
    if (i < nf) {
      v = a.far[fp][i];
      const uint32_t d = ld_u32(a.dist + v);
      to_near = d < T2;
      keep = !to_near;
      if (keep) a.fmark[v] = nb;
    }
    stage_push(St[0], to_near, v);
    stage_push(St[1], keep, v);
  }
  stage_close(St);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(&c->done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    c->T = T2;
    c->band = nb;
    c->nfar[fp] = 0;
    c->fpar = fp ^ 1;
    c->fmin = kLevelInf;
    c->done = 0;
  }
}

size_t dist_ws_bytes(const mk_graph* g) {
  return 256 + 6 * ((size_t)g->n * 4 + 256) + 2 * (levels_multi_cap(g) * 4 + 256) + 256;
}

}  // namespace

namespace mk {

size_t levels_multi_cap(const mk_graph* g) { return (size_t)g->n + g->view[VF].n_head / kChunk + 64; }

mk_status levels_run(mk_graph* g, uint32_t source, bool allow_bu, const LevelBufs& b, uint32_t* level,
                     uint64_t* pin, uint32_t* h_bottom_up_steps, hipStream_t stream) {
  const uint32_t N = g->n;
  LvCnt* c = reinterpret_cast<LvCnt*>(b.cnt);
  const DView F = g->view[VF].d;
  const DView R = g->view[VR].on ? g->view[VR].d : F;
  allow_bu = allow_bu && g->view[VR].on;
  hipLaunchKernelGGL(k_lv_clear, dim3(1), dim3(64), 0, stream, c);
  hipLaunchKernelGGL(k_lv_fill, dim3(blocks_for(N, 4096)), dim3(kBlock), 0, stream, level, N);
  hipLaunchKernelGGL(k_lv_seed, dim3(1), dim3(64), 0, stream, level, b.q[0], c, F.deg, source);
  MK_LAUNCH(g, "k_lv_seed");
  uint64_t every = kSyncFirst, next_sync = kSyncFirst;
  for (uint32_t L = 0;; ++L) {
    uint32_t* fin = b.q[L & 1];
    uint32_t* fout = b.q[(L + 1) & 1];
    hipLaunchKernelGGL(k_lv_decide, dim3(1), dim3(64), 0, stream, c, L, N, (int)allow_bu);
    hipLaunchKernelGGL(k_lv_td, dim3(blocks_for(N, 2048)), dim3(kBlock), 0, stream, F, c, L, level, fin,
                       fout, b.multi_v, b.multi_c);
    hipLaunchKernelGGL(k_lv_td_multi, dim3(2048), dim3(kBlock), 0, stream, F, c, L, level, fout, b.multi_v,
                       b.multi_c);
    if (allow_bu)
      hipLaunchKernelGGL(k_lv_bu, dim3(blocks_for(N, 8192)), dim3(kBlock), 0, stream, F, R, c, L, level,
                         fout, N);
    MK_LAUNCH(g, "k_lv step");
    if (L + 1 == next_sync || L + 1 >= N) {
      if (next_sync >= 2 * kSyncFirst) every = std::min<uint64_t>(2 * every, kSyncMax);
      next_sync += every;
      MK_HIP(g, hipMemcpyAsync(pin, &c->n[(L + 1) & 3], 4, hipMemcpyDeviceToHost, stream));
      MK_HIP(g, hipMemcpyAsync(pin + 1, &c->bu_steps, 4, hipMemcpyDeviceToHost, stream));
      MK_HIP(g, hipStreamSynchronize(stream));
      if ((uint32_t)pin[0] == 0 || L + 1 >= N) break;
    }
  }
  if (h_bottom_up_steps) *h_bottom_up_steps = (uint32_t)pin[1];
  return MK_OK;
}

// Tree nodes <dist, smallest parent> from finished distances (BFS levels when kUnit).
template <bool kUnit>
mk_status tree_from_dist(mk_graph* g, uint32_t source, const uint32_t* dist, uint64_t* D, hipStream_t stream) {
  const uint32_t N = g->n;
  const DView R = g->view[VR].d;
  uint32_t* heavy = g->fq[2];
  uint32_t* hcnt = g->fq[3];
  uint32_t* hoff = g->fq[4];
  uint32_t* nh = reinterpret_cast<LvCnt*>(g->lv_cnt)->pad;
  hipLaunchKernelGGL(k_lv_clear, dim3(1), dim3(64), 0, stream, reinterpret_cast<LvCnt*>(g->lv_cnt));
  hipLaunchKernelGGL(k_lv_tree_init, dim3(blocks_for(N, 4096)), dim3(kBlock), 0, stream, dist, D, N, source);
  hipLaunchKernelGGL(k_lv_heavy, dim3(blocks_for(N, 4096)), dim3(kBlock), 0, stream, R.nbk, dist, N, source,
                     heavy, nh);
  hipLaunchKernelGGL(k_lv_items, dim3(blocks_for(N, 1024)), dim3(kBlock), 0, stream, R.nbk, heavy, nh, hcnt);
  size_t tb = g->scan_tmp_bytes;
  if (rocprim::exclusive_scan(g->scan_tmp, tb, hcnt, hoff, 0u, (size_t)N, rocprim::plus<uint32_t>(), stream) !=
      hipSuccess)
    return MK_ERR_HIP;
  hipLaunchKernelGGL(k_lv_parents<kUnit>, dim3(4096), dim3(kBlock), 0, stream, R, dist, D, N, source, heavy, nh,
                     hoff, hcnt);
  MK_LAUNCH(g, "k_lv_parents");
  return MK_OK;
}

mk_status bfs_tree_by_levels(mk_graph* g, uint32_t source, uint32_t* level, uint64_t* D, hipStream_t stream) {
  LevelBufs b;
  b.cnt = g->lv_cnt;
  b.q[0] = g->fq[0];
  b.q[1] = g->fq[1];
  b.multi_v = g->lv_multi[0];
  b.multi_c = g->lv_multi[1];
  mk_status s = levels_run(g, source, true, b, level, g->h_pin, nullptr, stream);
  if (s != MK_OK) return s;
  return tree_from_dist<true>(g, source, level, D, stream);
}

// Every step either relaxes a non-empty near frontier or splits a non-empty far pile, and
// positive weights bound the number of distance drops, so the loop ends; the cap is a guard
// (and keeps the step stamps unique).
mk_status dist_run(mk_graph* g, uint32_t source, void* cnt, uint32_t* const q[2], const DsArgs& a,
                   uint64_t* pin, hipStream_t stream) {
  const uint32_t N = g->n;
  DsCnt* c = reinterpret_cast<DsCnt*>(cnt);
  const DView F = g->view[VF].d;
  const uint32_t delta = std::max<uint32_t>(1u, g->sssp_delta);
  hipLaunchKernelGGL(k_lv_clear, dim3(1), dim3(64), 0, stream, reinterpret_cast<LvCnt*>(c));
  hipLaunchKernelGGL(k_lv_fill, dim3(blocks_for(N, 4096)), dim3(kBlock), 0, stream, a.dist, N);
  hipLaunchKernelGGL(k_zero_marks, dim3(blocks_for(N, 4096)), dim3(kBlock), 0, stream, a.mark, a.fmark, N);
  hipLaunchKernelGGL(k_ds_seed, dim3(1), dim3(64), 0, stream, a.dist, q[0], c, source, delta);
  MK_LAUNCH(g, "k_ds_seed");
  const uint64_t cap = std::min<uint64_t>(64ull * N + 1024, 1ull << 31);
  uint64_t every = kSyncFirst, next_sync = kSyncFirst;
  for (uint64_t S = 0;; ++S) {
    const uint32_t s32 = (uint32_t)S;
    uint32_t* fin = q[S & 1];
    uint32_t* fout = q[(S + 1) & 1];
    hipLaunchKernelGGL(k_ds_relax, dim3(blocks_for(N, 2048)), dim3(kBlock), 0, stream, F, c, s32, a, fin, fout);
    hipLaunchKernelGGL(k_ds_relax_multi, dim3(2048), dim3(kBlock), 0, stream, F, c, s32, a, fout);
    hipLaunchKernelGGL(k_ds_far_min, dim3(blocks_for(N, 1024)), dim3(kBlock), 0, stream, c, s32, a);
    hipLaunchKernelGGL(k_ds_split, dim3(blocks_for(N, 2048)), dim3(kBlock), 0, stream, c, s32, a, fout, delta);
    MK_LAUNCH(g, "k_ds step");
    if (S + 1 == next_sync) {
      if (next_sync >= 2 * kSyncFirst) every = std::min<uint64_t>(2 * every, kSyncMax);
      next_sync += every;
      MK_HIP(g, hipMemcpyAsync(pin, &c->n[(S + 1) & 3], 4, hipMemcpyDeviceToHost, stream));
      MK_HIP(g, hipMemcpyAsync(pin + 1, &c->nfar[0], 8, hipMemcpyDeviceToHost, stream));
      MK_HIP(g, hipStreamSynchronize(stream));
      const uint32_t* h = reinterpret_cast<const uint32_t*>(pin + 1);
      if ((uint32_t)pin[0] == 0 && h[0] == 0 && h[1] == 0) break;
      if (S > cap) return MK_ERR_HIP;
    }
  }
  return MK_OK;
}

mk_status sssp_tree_by_distances(mk_graph* g, uint32_t source, uint32_t* dist, uint64_t* D, hipStream_t stream) {
  uint32_t* q[2] = {g->fq[0], g->fq[1]};
  DsArgs a;
  a.dist = dist;
  a.mark = g->fq[2];  // scratch here; the maintained traversals' stamps stay untouched
  a.fmark = g->fq[3];
  a.far[0] = g->far[0];
  a.far[1] = g->far[1];
  a.multi_v = g->lv_multi[0];
  a.multi_c = g->lv_multi[1];
  mk_status s = dist_run(g, source, g->lv_cnt, q, a, g->h_pin, stream);
  if (s != MK_OK) return s;
  return tree_from_dist<false>(g, source, dist, D, stream);
}

}  // namespace mk

extern "C" {

mk_status mk_bfs_levels(mk_graph* g, uint32_t source, uint32_t flags, void* d_ws, size_t ws_bytes,
                        uint32_t slot, uint32_t* d_level, uint32_t* h_bottom_up_steps, hipStream_t stream) {
  if (!g || !d_ws || !d_level || source >= g->n || slot >= kSlots || (flags & ~MK_BFS_TOP_DOWN_ONLY))
    return MK_ERR_INVALID_ARG;
  if (ws_bytes < levels_ws_bytes(g)) return MK_ERR_CAPACITY;
  if (mk_status gs = graph_guard(g); gs != MK_OK) return gs;
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
  LevelBufs b;
  b.cnt = take(256);
  b.q[0] = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  b.q[1] = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  b.multi_v = reinterpret_cast<uint32_t*>(take(levels_multi_cap(g) * 4));
  b.multi_c = reinterpret_cast<uint32_t*>(take(levels_multi_cap(g) * 4));
  return levels_run(g, source, !(flags & MK_BFS_TOP_DOWN_ONLY), b, d_level, g->slot_pin[slot],
                    h_bottom_up_steps, stream);
}

size_t mk_bfs_levels_workspace_bytes(const mk_graph* g) { return g ? levels_ws_bytes(g) : 0; }

mk_status mk_sssp_distances(mk_graph* g, uint32_t source, void* d_ws, size_t ws_bytes, uint32_t slot,
                            uint32_t* d_dist, hipStream_t stream) {
  if (!g || !d_ws || !d_dist || source >= g->n || slot >= kSlots) return MK_ERR_INVALID_ARG;
  if (ws_bytes < dist_ws_bytes(g)) return MK_ERR_CAPACITY;
  if (mk_status gs = graph_guard(g); gs != MK_OK) return gs;
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
  DsCnt* c = reinterpret_cast<DsCnt*>(take(256));
  uint32_t* q[2];
  q[0] = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  q[1] = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  DsArgs a;
  a.dist = d_dist;
  a.mark = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  a.fmark = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  a.far[0] = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  a.far[1] = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  a.multi_v = reinterpret_cast<uint32_t*>(take(levels_multi_cap(g) * 4));
  a.multi_c = reinterpret_cast<uint32_t*>(take(levels_multi_cap(g) * 4));
  return dist_run(g, source, c, q, a, g->slot_pin[slot], stream);
}

size_t mk_sssp_distances_workspace_bytes(const mk_graph* g) { return g ? dist_ws_bytes(g) : 0; }

}  // extern "C"
