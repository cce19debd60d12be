// Weakly connected components (section 4.4), PageRank (section 4.1) and triangle
// counting (section 4.3) over the slab views.
//
// All-vertex walks follow the paper's IterationScheme1 (one vertex per lane group); the
// few vertices with more than kHeavyBuckets buckets are walked by a whole block so that a
// power-law hub does not serialize one group.
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "mk_internal.h"

using namespace mk;

namespace {

constexpr uint32_t kWalkBlocks = 4096;
constexpr uint32_t kPrContribBlocks = 2048, kPrFinalBlocks = 512;
static_assert(kPrContribBlocks + kWalkBlocks + kPrFinalBlocks <= kPrParts, "PageRank partial sums");
constexpr uint32_t kPrChunk = 4;  // buckets per heavy-vertex work item
constexpr uint32_t kPrBatch = 8;  // head slabs a group loads at once in the PageRank pull
constexpr int kPrSyncEvery = 4;

inline uint32_t blocks_for(uint64_t n, uint32_t cap = 4096) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + kBlock - 1) / kBlock, cap));
}

// Vertices of a view with more than kHeavyBuckets buckets (staged per block: they are
// sparse, and one counter atomic per wave that finds one would serialize).
__global__ void k_collect_heavy(const uint32_t* nbk, uint32_t nv, uint32_t* out, uint32_t* cnt) {
  __shared__ Stage S[1];
  stage_open(S[0], out, cnt);
  __syncthreads();
  const uint64_t lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; base < nv;
       base += stride) {
    const uint64_t v = base + lane;
    const bool heavy = v < nv && nbk[v] > kHeavyBuckets;
    stage_push(S[0], heavy, (uint32_t)v);
  }
  stage_close(S);
}

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// ================================================================= union-find (WCC)
// Hooking rule: the larger root is hooked under the smaller one by CAS, so every parent
// pointer goes to a smaller id and the final root of a component is its minimum id.
__device__ inline uint32_t uf_find(uint32_t* P, uint32_t x) {
  while (true) {
    const uint32_t p = ld_u32(P + x);
    if (p == x) return x;
    const uint32_t gp = ld_u32(P + p);
    if (gp != p) __hip_atomic_store(P + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // halving
    x = gp;
  }
}

__device__ inline void uf_union(uint32_t* P, uint32_t a, uint32_t b) {
  while (true) {
    a = uf_find(P, a);
    b = uf_find(P, b);
    if (a == b) return;
    if (a < b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    const uint32_t r = atomicCAS(P + a, a, b);  // hook the larger root under the smaller
    if (r == a) return;
    a = r;  // a was hooked meanwhile: continue from its true parent (a smaller id)
  }
}

__global__ void k_wcc_init(uint32_t* P, uint32_t nv) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) P[v] = v;
}

// Static WCC: union over every arc.  A neighbour whose parent already is u's root (as
// found once per vertex; a stale root only means an older member of the same component)
// is skipped without a union, and a lane issues the parent loads of a whole slab together.
//
// With `big` set (the sampled static WCC below), a vertex whose root is *big is skipped: its
// arcs are left to their other ends, which then walk both directions (the undirected view).
__global__ void __launch_bounds__(kBlock) k_wcc_all(DView F, uint32_t* P, uint32_t nv,
                                                    const uint32_t* heavy, const uint32_t* nheavy,
                                                    const uint32_t* big) {
  const uint32_t skip = big ? *big : kInvalid;
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  auto body = [&](uint32_t u, uint32_t ru, uint64_t x, bool data) {
    const uint32_t v = (uint32_t)x;
    if (data && valid_key(v) && ld_u32(P + v) != ru) uf_union(P, u, v);
  };
  // single-bucket vertices: one lane each
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < nv; u += gridDim.x * blockDim.x) {
    if (F.nbk[u] != 1 || F.deg[u] == 0) continue;
    const uint32_t ru = uf_find(P, u);
    if (ru == skip) continue;
    Slab sl;
    uint32_t t = u;
    while (true) {
      load_slab(F, t, sl);
      uint32_t pv[kKeysPerSlab];
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j) {
        const uint32_t v = (uint32_t)sl.w[j];
        pv[j] = valid_key(v) ? ld_u32(P + v) : ru;
      }
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j)
        if (pv[j] != ru) uf_union(P, u, (uint32_t)sl.w[j]);
      t = (uint32_t)sl.w[15];
      if (t == kInvalid) break;
    }
  }
  for (uint32_t u = g0; u < nv; u += ng) {
    const uint32_t nb = F.nbk[u];
    if (nb == 1 || nb > kHeavyBuckets || F.deg[u] == 0) continue;
    const uint32_t ru = uf_find(P, u);
    if (ru == skip) continue;
    for_each_slab(F, u, [&](uint64_t x, bool data) { body(u, ru, x, data); });
  }
  const uint32_t nh = *nheavy, gib = threadIdx.x / kGroup;
  for (uint32_t j = blockIdx.x; j < nh; j += gridDim.x) {
    const uint32_t u = heavy[j];
    const uint32_t ru = uf_find(P, u);
    if (ru == skip) continue;
    for_each_slab_strided(F, u, gib, kGroupsPerBlock, [&](uint64_t x, bool data) { body(u, ru, x, data); });
  }
}

// Sampled static WCC (after the subgraph-sampling method of Sutton, Ben-Nun and Barak,
// "Optimizing parallel graph connectivity computation via subgraph sampling", IPDPS 2018).
// First every vertex points its parent at the smallest id among itself and the neighbours in
// its primary slab of the undirected view (at most 15, one 128-byte read, no atomics): a
// forest whose every edge is an arc, which on a power-law graph already holds most of the
// giant component in one tree.  After flattening, the most frequent root among kWccSamples
// sampled vertices is taken as the largest component, and only vertices outside it walk their
// neighbourhoods (both directions, with unions), so the giant component's arcs are not read.
// The partition is the plain one (labels are still component minima): every arc with an end
// outside the largest component is united from that end, and an arc with both ends inside
// joins nothing new.
constexpr uint32_t kWccLinks = 2;
constexpr uint32_t kWccSamples = 1024;

__global__ void k_wcc_link_first(DView U, uint32_t* P, uint32_t nv) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < nv; u += gridDim.x * blockDim.x) {
    if (U.deg[u] == 0) continue;
    const uint64_t* hs = slab_ptr(U, u);
    const int nd = (uint32_t)(ld_word(hs + 15) >> 32) > 1 ? kKeysPerSlab - 1 : kKeysPerSlab;
    const uint32_t ru = uf_find(P, u);
    uint32_t linked = 0;
    for (int i = 0; i < nd && linked < kWccLinks; ++i) {
      const uint32_t v = (uint32_t)ld_word(hs + i);
      if (!valid_key(v)) continue;
      if (ld_u32(P + v) != ru) uf_union(P, u, v);
      ++linked;
    }
  }
}

// Every parent made a root (no labels written); a plain walk to the root, as in k_wcc_compress.
__global__ void k_wcc_flatten(uint32_t* P, uint32_t nv) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    uint32_t r = v;
    for (uint32_t p = ld_u32(P + r); p != r; p = ld_u32(P + r)) r = p;
    __hip_atomic_store(P + v, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One block of kWccSamples threads: the most frequent root among the sampled vertices
// (ties: the smaller root) into *big.  Samples are spread over the ids by a Weyl sequence.
__global__ void __launch_bounds__(kWccSamples) k_wcc_big(const uint32_t* P, uint32_t nv, uint32_t* big) {
  __shared__ uint32_t root[kWccSamples];
  __shared__ unsigned long long best;
  const uint32_t v = (uint32_t)(((uint64_t)threadIdx.x * 0x9E3779B97F4A7C15ull >> 32) % nv);
  root[threadIdx.x] = ld_u32(P + v);
  if (threadIdx.x == 0) best = 0;
  __syncthreads();
  const uint32_t r = root[threadIdx.x];
  uint32_t n = 0;
  for (uint32_t i = 0; i < kWccSamples; ++i) n += root[i] == r;
  // larger count first, then the smaller root
  atomicMax(&best, ((unsigned long long)n << 32) | (0xFFFFFFFFu - r));
  __syncthreads();
  if (threadIdx.x == 0) *big = 0xFFFFFFFFu - (uint32_t)best;
}

// IterationScheme2 (section 3.4): one 16-lane group per bucket chain <v, i>, in a
// grid-stride loop over the pair list.  Bucket i > 0 of v is the extra head slab
// N + off[v] - v + i - 1 = N + k - v - 1 (the extra head slabs were laid out by the same
// scan); bucket 0 is v's primary slab, with 14 data words when v has several buckets.
template <class F>
__device__ inline void walk_pair(const DView& V, const uint32_t* pv, const uint32_t* pi, uint32_t nv,
                                 uint32_t k, uint32_t& v, F&& f) {
  v = pv[k];
  const uint32_t i = pi[k];
  const uint32_t h = i == 0 ? v : nv + k - v - 1;
  const uint64_t x = ld_word(slab_ptr(V, h) + glane());
  int nd = kKeysPerSlab;
  if (i == 0 && (uint32_t)(gbcast64(x, 15) >> 32) > 1) nd = kKeysPerSlab - 1;
  walk_chain(V, h, x, nd, f);
}

// Static WCC under IterationScheme2: union over the arcs of every bucket chain.
__global__ void __launch_bounds__(kBlock) k_wcc_pairs(DView F, uint32_t* P, const uint32_t* pv,
                                                      const uint32_t* pi, uint32_t np, uint32_t nv) {
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  for (uint32_t k = g0; k < np; k += ng) {
    const uint32_t u = pv[k];
    const uint32_t ru = uf_find(P, u);
    uint32_t vv;
    walk_pair(F, pv, pi, nv, k, vv, [&](uint64_t x, bool data) {
      const uint32_t v = (uint32_t)x;
      if (data && valid_key(v) && ld_u32(P + v) != ru) uf_union(P, u, v);
    });
  }
}

__global__ void k_wcc_batch(uint32_t* P, Log lg, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    if (lg.st[i] == 1) uf_union(P, lg.s[i], lg.d[i]);
}

// ----------------------------------------------------------------- incremental WCC schemes
// The vertices that gained out-arcs in a pending insert batch, each listed once (the
// to_union flags of section 4.4): vertices with more than kHeavyBuckets buckets go to a
// second list that is walked a block per vertex.
__global__ void k_wcc_flag(Log lg, uint64_t n, const uint32_t* nbk, uint32_t* flag, uint32_t* light,
                           uint32_t* nlight, uint32_t* heavy, uint32_t* nheavy) {
  __shared__ Stage S[2];
  stage_open(S[0], light, nlight);
  stage_open(S[1], heavy, nheavy);
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    const uint64_t i = base + threadIdx.x;
    bool p = false, hv = false;
    uint32_t u = 0;
    if (i < n && lg.st[i] == 1) {
      u = lg.s[i];
      p = ld_u32(flag + u) == 0u && atomicExch(flag + u, 1u) == 0u;
      hv = p && nbk[u] > kHeavyBuckets;
    }
    stage_push(S[0], p && !hv, u);
    stage_push(S[1], hv, u);
  }
  stage_close(S);
}

__global__ void k_wcc_unflag(uint32_t* flag, const uint32_t* light, const uint32_t* nlight,
                             const uint32_t* heavy, const uint32_t* nheavy) {
  const uint32_t nl = *nlight, nh = *nheavy;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nl + nh; i += gridDim.x * blockDim.x)
    flag[i < nl ? light[i] : heavy[i - nl]] = 0u;
}

// UpdateIterator over one bucket chain (section 3.4).  The chain's mark is <slab + 1, lane>
// of the first word the last pass did not unite (0: the head slab, lane 0).  As a chain's
// filled words always form a prefix, everything inserted since then lies at or past the
// mark, and the first EMPTY word met is the chain's new end: the mark moves there (the
// paper's UpdateSlabPointers, done by the pass itself).  A chain with no new word costs one
// slab read: the paper's per-chain is_updated flag is derived, not stored.
__device__ inline void wcc_update_chain(const DView& F, uint64_t* marks, uint32_t* P, uint32_t h,
                                        int nd0, uint32_t u, uint32_t ru) {
  const int gl = glane();
  const uint64_t m = ld_u64(marks + h);
  uint32_t s = (uint32_t)m ? (uint32_t)m - 1u : h;
  int l = (uint32_t)m ? (int)(m >> 32) : 0;
  int nd = s == h ? nd0 : kKeysPerSlab;
  while (true) {
    const uint64_t x = ld_word(slab_ptr(F, s) + gl);
    const uint32_t v = (uint32_t)x;
    const bool data = gl >= l && gl < nd;
    if (data && valid_key(v) && ld_u32(P + v) != ru) uf_union(P, u, v);
    const uint32_t e = gballot(data && v == kEmptyKey);
    if (e) {
      l = __ffs(e) - 1;
      break;
    }
    const uint32_t nx = gbcast(v, 15);
    if (nx == kInvalid) {
      l = nd;
      break;
    }
    s = nx;
    l = 0;
    nd = kKeysPerSlab;
  }
  const uint64_t nm = ((uint64_t)(uint32_t)l << 32) | (s + 1u);
  if (gl == 0 && nm != m) marks[h] = nm;
}

// Incremental WCC over the listed vertices: every slab of each (SlabIterator scheme, marks
// null) or only the words past each chain's mark (UpdateIterator scheme).  Light vertices
// take a 16-lane group each, heavy ones a block with its groups striding over the buckets.
__global__ void __launch_bounds__(kBlock) k_wcc_listed(DView F, uint32_t* P, uint64_t* marks,
                                                       const uint32_t* light, const uint32_t* nlight,
                                                       const uint32_t* heavy, const uint32_t* nheavy) {
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  const uint32_t gib = threadIdx.x / kGroup;
  auto walk = [&](uint32_t u, uint32_t b0, uint32_t stride) {
    const uint32_t ru = uf_find(P, u);
    if (!marks) {
      for_each_slab_strided(F, u, b0, stride, [&](uint64_t x, bool data) {
        const uint32_t v = (uint32_t)x;
        if (data && valid_key(v) && ld_u32(P + v) != ru) uf_union(P, u, v);
      });
      return;
    }
    const Table t = group_table(F, u);
    for (uint32_t b = b0; b < t.nb; b += stride)
      wcc_update_chain(F, marks, P, b ? t.xb + b - 1 : u,
                       (b == 0 && t.nb > 1) ? kKeysPerSlab - 1 : kKeysPerSlab, u, ru);
  };
  const uint32_t nl = *nlight;
  for (uint32_t i = g0; i < nl; i += ng) walk(light[i], 0, 1);
  const uint32_t nh = *nheavy;
  for (uint32_t j = blockIdx.x; j < nh; j += gridDim.x) walk(heavy[j], gib, kGroupsPerBlock);
}

// UpdateSlabPointers over every chain: each mark moves to its chain's end (the first EMPTY
// word, or past the last slab's data words when the chain is full).  One group per chain.
__global__ void __launch_bounds__(kBlock) k_mark_all(DView F, uint64_t* marks, uint64_t n_head,
                                                     uint32_t nv) {
  const uint64_t g0 = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint64_t ng = (uint64_t)gridDim.x * kGroupsPerBlock;
  const int gl = glane();
  for (uint64_t h = g0; h < n_head; h += ng) {
    uint32_t s = (uint32_t)h;
    uint64_t y = ld_word(slab_ptr(F, s) + gl);
    int nd = (h < nv && (uint32_t)(gbcast64(y, 15) >> 32) > 1) ? kKeysPerSlab - 1 : kKeysPerSlab;
    int l;
    while (true) {
      const uint32_t e = gballot(gl < nd && (uint32_t)y == kEmptyKey);
      if (e) {
        l = __ffs(e) - 1;
        break;
      }
      const uint32_t nx = gbcast((uint32_t)y, 15);
      if (nx == kInvalid) {
        l = nd;
        break;
      }
      s = nx;
      nd = kKeysPerSlab;
      y = ld_word(slab_ptr(F, s) + gl);
    }
    if (gl == 0) marks[h] = ((uint64_t)(uint32_t)l << 32) | (s + 1u);
  }
}

// Full path compression and the labels.  No union runs here, so every root is final and
// any parent a thread reads (the value the union kernels left, or the root another thread
// has just stored) leads to it.  The walk must not halve paths: a halving store computed
// from an earlier read could land after another thread's final store to the same vertex
// and leave it pointing at a non-root.
__global__ void k_wcc_compress(uint32_t* P, uint32_t nv, uint32_t* label) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    uint32_t r = v;
    for (uint32_t p = ld_u32(P + r); p != r; p = ld_u32(P + r)) r = p;
    __hip_atomic_store(P + v, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    label[v] = r;
  }
}

__global__ void k_copy_u32(const uint32_t* a, uint32_t* b, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = a[i];
}

// ================================================================= PageRank
__device__ inline double block_sum(double v, double* lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += lds[i];
  return s;  // valid in thread 0
}

__global__ void k_pr_fill(float* x, uint32_t nv, float v) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) x[i] = v;
}

// Contribution per vertex C[u] = PR[u] / out[u] (the FindContributionPerVertex kernel),
// plus the FP64 sum of the ranks of zero-out-degree vertices (FindTeleportProb).
//
// With `cr` (the packing iteration), the contribution goes beside the vertex's hot-first rank,
// cr[v] = <rank[v], contribution bits>, so the packing pull reads both with one 8-byte load.
__global__ void __launch_bounds__(kBlock) k_pr_contrib(const float* __restrict__ x,
                                                       const uint32_t* __restrict__ outdeg,
                                                       float* __restrict__ c, uint32_t nv,
                                                       double* dpart, const uint32_t* state,
                                                       const uint32_t* __restrict__ rank, uint2* __restrict__ cr) {
  __shared__ double lds[kBlock / 64];
  if (state[0]) return;
  double local = 0;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    const uint32_t o = outdeg[v];
    const float xv = x[v];
    const float cv = o ? xv / (float)o : 0.f;
    if (cr) cr[v] = make_uint2(rank[v], __float_as_uint(cv));
    else c[v] = cv;
    if (!o) local += xv;
  }
  const double s = block_sum(local, lds);
  if (threadIdx.x == 0) dpart[blockIdx.x] = s;
}

// Sum of per-block partial sums in a fixed order (one block): the dangling mass and the L1
// change of an iteration are deterministic and take no same-address atomics.  (The in-arc
// sums of vertices split into bucket work items are the exception: their FP64 partials are
// added by atomics, so the order, and the last bits of those ranks, can vary between runs.)
__device__ inline double sum_parts(const double* part, uint32_t n, double* lds) {
  double v = 0;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
  return block_sum(v, lds);
}

__global__ void __launch_bounds__(kBlock) k_pr_sum(const double* part, uint32_t n, double* out,
                                                   const uint32_t* state) {
  __shared__ double lds[kBlock / 64];
  if (state[0]) return;
  const double s = sum_parts(part, n, lds);
  if (threadIdx.x == 0) *out = s;
}

// Pull over in-arcs (reverse view): PR'[v] = (1-d)/N + d * (sum C[u] + dangling/N),
// and the FP64 L1 change sum |PR'[v] - PR[v]|.
// With `list`, the pull also packs every vertex's in-arc sources, as their ranks in the
// hot-first order (rank[u]), into list[off[v] .. off[v] + deg[v]) for the packed iterations
// (k_pr_pull): single-bucket and 2..16-bucket vertices in slab order, heavy vertices in the
// order their work items reserve room at cur[j] (so their keys' order, and the last bits of
// their FP64 sums, can vary between runs).
__global__ void __launch_bounds__(kBlock) k_pr_gather(DView R, const float* __restrict__ c,
                                                      const float* __restrict__ x,
                                                      float* __restrict__ y, uint32_t nv, float damping,
                                                      const double* dang, double* delta,
                                                      const uint32_t* heavy, const uint32_t* nheavy,
                                                      const uint32_t* hcnt, const uint32_t* hoff,
                                                      double* hacc, const uint32_t* state,
                                                      uint32_t* __restrict__ list, const uint32_t* __restrict__ off,
                                                      uint32_t* cur, const uint2* __restrict__ cr) {
  __shared__ double lds[kBlock / 64];
  if (state[0]) return;
  const double base = (1.0 - (double)damping) / nv + (double)damping * (*dang) / nv;
  double local = 0;
  // u's contribution, and with `list` its hot-first rank r (both from one load of cr[u])
  auto term = [&](uint32_t u, uint32_t& r) -> float {
    if (list) {
      const uint2 q = cr[u];
      r = q.x;
      return __uint_as_float(q.y);
    }
    r = 0;
    return c[u];
  };
  // single-bucket vertices (most of a power-law graph): one lane per vertex, so a wave keeps
  // 64 slab reads and their gathers in flight
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    if (R.nbk[v] != 1) continue;
    double s = 0;
    const uint32_t dv = R.deg[v];
    if (dv != 0) {  // vertices without in-arcs need no slab read
      Slab sl;
      uint32_t t = v;
      uint32_t* out = list ? list + off[v] : nullptr;
      uint32_t n = 0;
      while (true) {
        load_slab(R, t, sl);
#pragma unroll
        for (int j = 0; j < kKeysPerSlab; ++j) {
          const uint32_t u = (uint32_t)sl.w[j];
          if (valid_key(u)) {
            uint32_t r;
            s += (double)term(u, r);
            if (out && n < dv) out[n] = r;
            ++n;
          }
        }
        t = (uint32_t)sl.w[15];
        if (t == kInvalid) break;
      }
    }
    const float nvl = (float)(base + (double)damping * s);
    y[v] = nvl;
    local += fabs((double)nvl - (double)x[v]);
  }
  // vertices with 2 .. kHeavyBuckets buckets: one 16-lane group per vertex.  The group
  // issues the loads of all its head slabs at once, then all their contribution gathers,
  // and only then follows the (rare) chains, rather than one dependent slab at a time.
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  const int gl = glane();
  for (uint32_t v = g0; v < nv; v += ng) {
    const uint32_t nb = R.nbk[v];
    if (nb == 1 || nb > kHeavyBuckets) continue;
    const uint64_t x0 = ld_word(slab_ptr(R, v) + gl);
    const uint32_t xb = gbcast((uint32_t)x0, 14);
    double s = 0;
    uint32_t* out = list ? list + off[v] : nullptr;
    const uint32_t dv = list ? R.deg[v] : 0u;
    uint32_t n = 0;  // keys packed so far (the same in every lane of the group)
    auto pack = [&](bool valid, uint32_t r) {
      const uint32_t m = gballot(valid);
      const uint32_t at = n + (uint32_t)__popc(m & ((1u << gl) - 1u));
      if (valid && at < dv) out[at] = r;
      n += (uint32_t)__popc(m);
    };
    for (uint32_t b0 = 0; b0 < nb; b0 += kPrBatch) {
      uint64_t hw[kPrBatch];
#pragma unroll
      for (uint32_t j = 0; j < kPrBatch; ++j) {
        const uint32_t b = b0 + j;
        hw[j] = b == 0 ? x0 : (b < nb ? ld_word(slab_ptr(R, xb + b - 1) + gl) : kEmptyWord);
      }
#pragma unroll
      for (uint32_t j = 0; j < kPrBatch; ++j) {
        const uint32_t u = (uint32_t)hw[j];
        const bool data = gl < (b0 + j == 0 ? kKeysPerSlab - 1 : kKeysPerSlab);
        uint32_t r = 0;
        if (data && valid_key(u)) s += (double)term(u, r);
        if (out) pack(data && valid_key(u), r);
      }
#pragma unroll
      for (uint32_t j = 0; j < kPrBatch; ++j) {  // chained slabs after a full head slab
        if (b0 + j >= nb) break;
        const uint32_t next = gbcast((uint32_t)hw[j], 15);
        if (next == kInvalid) continue;
        walk_chain(R, next, ld_word(slab_ptr(R, next) + gl), kKeysPerSlab, [&](uint64_t w, bool data) {
          const uint32_t u = (uint32_t)w;
          uint32_t r = 0;
          if (data && valid_key(u)) s += (double)term(u, r);
          if (out) pack(data && valid_key(u), r);
        });
      }
    }
    s = gsum(s);
    if (glane() == 0) {
      const float nvl = (float)(base + (double)damping * s);
      y[v] = nvl;
      local += fabs((double)nvl - (double)x[v]);
    }
  }
  // heavy vertices: work items of kPrChunk buckets spread over every group; partial sums
  // go to hacc[j] and k_pr_heavy_final turns them into ranks
  const uint32_t nh = *nheavy;
  if (nh) {
    const uint32_t items = hoff[nh - 1] + hcnt[nh - 1];
    for (uint32_t it = g0; it < items; it += ng) {
      uint32_t lo = 0, hi = nh;  // last j with hoff[j] <= it
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (hoff[mid] <= it) lo = mid;
        else hi = mid;
      }
      const uint32_t v = heavy[lo];
      const uint32_t b0 = (it - hoff[lo]) * kPrChunk;
      double s = 0;
      const uint32_t end = list ? off[v] + R.deg[v] : 0u;
      for_each_bucket_range(R, v, b0, b0 + kPrChunk, [&](uint64_t w, bool data) {
        const uint32_t u = (uint32_t)w;
        const bool valid = data && valid_key(u);
        uint32_t r = 0;
        if (valid) s += (double)term(u, r);
        if (list) {  // room for this slab's keys in v's segment, one reservation per slab
          const uint32_t m = gballot(valid);
          uint32_t at = 0;
          if (glane() == 0 && m) at = atomicAdd(cur + lo, (uint32_t)__popc(m));
          at = gbcast(at, 0) + (uint32_t)__popc(m & ((1u << glane()) - 1u));
          if (valid && at < end) list[at] = r;
        }
      });
      s = gsum(s);
      if (glane() == 0 && s != 0.0) atomicAdd(hacc + lo, s);
    }
  }
  const double s = block_sum(local, lds);
  if (threadIdx.x == 0) delta[blockIdx.x] = s;
}

// PageRank pull over the packed in-arc lists (iterations after the packing one): the same
// sums as k_pr_gather, reading 4 bytes per in-arc instead of whole slabs.  Each lane issues
// kPullRound list loads, then their contribution gathers, before it adds them (in list
// order), so that many gathers are in flight.  Single-bucket vertices take a lane,
// 2..16-bucket ones a 16-lane group, heavy ones work items of kPullItem in-arcs (partial sums
// into hacc, as in k_pr_gather).
constexpr uint32_t kPullRound = 8;
constexpr uint32_t kPullItem = kGroup * kPullRound * 4;

__global__ void k_pull_items(const uint32_t* deg, const uint32_t* heavy, const uint32_t* nheavy,
                             const uint32_t* off, uint32_t* cnt, uint32_t* cur) {
  const uint32_t nh = *nheavy;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nh; j += gridDim.x * blockDim.x) {
    const uint32_t v = heavy[j];
    cnt[j] = (deg[v] + kPullItem - 1) / kPullItem;
    cur[j] = off[v];
  }
}

// off[nv] = off[nv - 1] + deg[nv - 1]: the end of the last segment.
__global__ void k_pull_end(const uint32_t* deg, uint32_t* off, uint32_t nv) {
  if (threadIdx.x == 0) off[nv] = off[nv - 1] + deg[nv - 1];
}

// Hot-first order of the sources for the packed iterations: a stable sort by out-degree class
// (largest first) puts the sources of most in-arcs in a few MB of the contribution vector,
// which the L2 of each XCD keeps.  Keys 31 - floor(log2(out + 1)), values the vertex ids.
__global__ void k_pr_class(const uint32_t* __restrict__ outdeg, uint32_t nv, uint32_t* key, uint32_t* idx) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    key[v] = (uint32_t)__clz(outdeg[v] + 1u);  // 31 - floor(log2(out + 1)), in [0, 31]
    idx[v] = v;
  }
}
__global__ void k_pr_rank(const uint32_t* __restrict__ perm, uint32_t nv, uint32_t* __restrict__ rank) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) rank[perm[i]] = i;
}

// k_pr_contrib in the hot-first order: cp[i] = PR[perm[i]] / out[perm[i]], and the FP64 sum of
// the ranks of zero-out-degree vertices.
__global__ void __launch_bounds__(kBlock) k_pr_contrib_perm(const float* __restrict__ x,
                                                            const uint32_t* __restrict__ outdeg,
                                                            const uint32_t* __restrict__ perm,
                                                            float* __restrict__ cp, uint32_t nv, double* dpart,
                                                            const uint32_t* state) {
  __shared__ double lds[kBlock / 64];
  if (state[0]) return;
  double local = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
    const uint32_t v = perm[i];
    const uint32_t o = outdeg[v];
    const float xv = x[v];
    cp[i] = o ? xv / (float)o : 0.f;
    if (!o) local += xv;
  }
  const double s = block_sum(local, lds);
  if (threadIdx.x == 0) dpart[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_pr_pull(const uint32_t* __restrict__ nbk,
                                                    const uint32_t* __restrict__ deg,
                                                    const uint32_t* __restrict__ off,
                                                    const uint32_t* __restrict__ list,
                                                    const float* __restrict__ c, const float* __restrict__ x,
                                                    float* __restrict__ y, uint32_t nv, float damping,
                                                    const double* dang, double* delta, const uint32_t* heavy,
                                                    const uint32_t* nheavy, const uint32_t* pcnt,
                                                    const uint32_t* poff, double* hacc, const uint32_t* state) {
  __shared__ double lds[kBlock / 64];
  if (state[0]) return;
  const double base = (1.0 - (double)damping) / nv + (double)damping * (*dang) / nv;
  double local = 0;
  // in-arcs [a + first + k * stride, for k < kPullRound) below a + n (n >= 1), summed in
  // order.  Every load is unconditional (indexes clamped into the segment and the vertex
  // range, out-of-range terms masked afterwards), so a lane has all its loads in flight.
  auto round = [&](uint32_t a, uint32_t n, uint32_t first, uint32_t stride, double& s) {
    uint32_t u[kPullRound];
#pragma unroll
    for (uint32_t k = 0; k < kPullRound; ++k) u[k] = list[a + min(first + k * stride, n - 1)];
    float cv[kPullRound];
#pragma unroll
    for (uint32_t k = 0; k < kPullRound; ++k) cv[k] = c[min(u[k], nv - 1)];
#pragma unroll
    for (uint32_t k = 0; k < kPullRound; ++k)
      if (first + k * stride < n && u[k] < nv) s += (double)cv[k];
  };
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    if (nbk[v] != 1) continue;
    const uint32_t a = off[v], n = deg[v];
    double s = 0;
    for (uint32_t j0 = 0; j0 < n; j0 += kPullRound) round(a + j0, n - j0, 0, 1, s);
    const float nvl = (float)(base + (double)damping * s);
    y[v] = nvl;
    local += fabs((double)nvl - (double)x[v]);
  }
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  const uint32_t gl = (uint32_t)glane();
  for (uint32_t v = g0; v < nv; v += ng) {
    const uint32_t nb = nbk[v];
    if (nb == 1 || nb > kHeavyBuckets) continue;
    const uint32_t a = off[v], n = deg[v];
    double s = 0;
    for (uint32_t j0 = 0; j0 < n; j0 += kGroup * kPullRound) round(a + j0, n - j0, gl, kGroup, s);
    s = gsum(s);
    if (gl == 0) {
      const float nvl = (float)(base + (double)damping * s);
      y[v] = nvl;
      local += fabs((double)nvl - (double)x[v]);
    }
  }
  const uint32_t nh = *nheavy;
  if (nh) {
    const uint32_t items = poff[nh - 1] + pcnt[nh - 1];
    for (uint32_t it = g0; it < items; it += ng) {
      uint32_t lo = 0, hi = nh;  // last j with poff[j] <= it
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (poff[mid] <= it) lo = mid;
        else hi = mid;
      }
      const uint32_t v = heavy[lo];
      const uint32_t j0 = (it - poff[lo]) * kPullItem;
      const uint32_t n = min(deg[v] - j0, kPullItem);
      double s = 0;
      for (uint32_t j = 0; j < n; j += kGroup * kPullRound) round(off[v] + j0 + j, n - j, gl, kGroup, s);
      s = gsum(s);
      if (gl == 0 && s != 0.0) atomicAdd(hacc + lo, s);
    }
  }
  const double s = block_sum(local, lds);
  if (threadIdx.x == 0) delta[blockIdx.x] = s;
}

// PageRank pull under IterationScheme2: the FP64 in-arc sum of every reverse-view bucket
// chain into pp[k]; k_pr_final_s2 adds a vertex's buckets in bucket order.
__global__ void __launch_bounds__(kBlock) k_pr_gather_s2(DView R, const float* __restrict__ c,
                                                         const uint32_t* pv, const uint32_t* pi, uint32_t np,
                                                         uint32_t nv, double* __restrict__ pp,
                                                         const uint32_t* state) {
  if (state[0]) return;
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  for (uint32_t k = g0; k < np; k += ng) {
    double s = 0;
    uint32_t v;
    walk_pair(R, pv, pi, nv, k, v, [&](uint64_t w, bool data) {
      const uint32_t u = (uint32_t)w;
      if (data && valid_key(u)) s += (double)c[u];
    });
    s = gsum(s);
    if (glane() == 0) pp[k] = s;
  }
}

__global__ void __launch_bounds__(kBlock) k_pr_final_s2(const uint32_t* __restrict__ nbk,
                                                        const uint32_t* __restrict__ off,
                                                        const double* __restrict__ pp, const float* __restrict__ x,
                                                        float* __restrict__ y, uint32_t nv, float damping,
                                                        const double* dang, double* delta, const uint32_t* state) {
  __shared__ double lds[kBlock / 64];
  if (state[0]) return;
  const double base = (1.0 - (double)damping) / nv + (double)damping * (*dang) / nv;
  double local = 0;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    const uint32_t o = off[v], nb = nbk[v];
    double s = 0;
    for (uint32_t i = 0; i < nb; ++i) s += pp[o + i];
    const float nvl = (float)(base + (double)damping * s);
    y[v] = nvl;
    local += fabs((double)nvl - (double)x[v]);
  }
  const double s = block_sum(local, lds);
  if (threadIdx.x == 0) delta[blockIdx.x] = s;
}

// Work items per heavy vertex: ceil(buckets / kPrChunk).
__global__ void k_heavy_items(const uint32_t* nbk, const uint32_t* heavy, const uint32_t* nheavy,
                              uint32_t* cnt, double* acc) {
  const uint32_t nh = *nheavy;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nh; j += gridDim.x * blockDim.x) {
    cnt[j] = (nbk[heavy[j]] + kPrChunk - 1) / kPrChunk;
    acc[j] = 0.0;
  }
}

// Ranks of the heavy vertices from their partial sums (and their share of the L1 change).
__global__ void __launch_bounds__(kBlock) k_pr_heavy_final(const uint32_t* heavy, const uint32_t* nheavy,
                                                           double* acc, const float* x, float* y,
                                                           uint32_t nv, float damping, const double* dang,
                                                           double* delta, const uint32_t* state) {
  __shared__ double lds[kBlock / 64];
  if (state[0]) return;
  const double base = (1.0 - (double)damping) / nv + (double)damping * (*dang) / nv;
  const uint32_t nh = *nheavy;
  double local = 0;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nh; j += gridDim.x * blockDim.x) {
    const uint32_t v = heavy[j];
    const float nvl = (float)(base + (double)damping * acc[j]);
    y[v] = nvl;
    acc[j] = 0.0;
    local += fabs((double)nvl - (double)x[v]);
  }
  const double s = block_sum(local, lds);
  if (threadIdx.x == 0) delta[blockIdx.x] = s;
}

// Convergence bookkeeping for one iteration (single thread): stop at delta <= tol, when
// the change has not improved for three iterations (the FP32 noise floor), or at max_iter.
__global__ void __launch_bounds__(kBlock) k_pr_check(Counters* C, int slot, double tol, uint32_t max_iter,
                                                     const double* dpart, uint32_t nparts) {
  __shared__ double lds[kBlock / 64];
  uint32_t* st = C->pr_state;
  if (st[0]) return;
  const double d = sum_parts(dpart, nparts, lds);  // the L1 change of this iteration
  if (threadIdx.x != 0) return;
  C->pr_acc[2 * slot + 1] = d;
  st[1] += 1;
  C->pr_last = d;
  if (d < C->pr_best * 0.999) {
    C->pr_best = d;
    st[2] = 0;
  } else {
    st[2] += 1;
  }
  if (d <= tol || st[2] >= 3 || st[1] >= max_iter) st[0] = 1;
}

__global__ void k_pr_start(Counters* C) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < 8; ++i) C->pr_acc[i] = 0.0;
  C->pr_state[0] = 0;
  C->pr_state[1] = 0;
  C->pr_state[2] = 0;
  C->pr_last = 0;
  C->pr_best = 1e300;
}

// Copy the final vector (buffer iters % 2) to the persistent state and the output.
__global__ void k_pr_final(const Counters* C, const float* a, const float* b, float* keep, float* out,
                           uint32_t nv, uint32_t* iters_out) {
  const uint32_t it = C->pr_state[1];
  const float* src = (it & 1) ? b : a;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
    const float v = src[i];
    if (keep != src) keep[i] = v;
    out[i] = v;
  }
  if (iters_out && blockIdx.x == 0 && threadIdx.x == 0) *iters_out = it;
}

// ================================================================= triangle counting
__device__ inline bool ranks_before(const uint32_t* deg, uint32_t a, uint32_t b) {
  const uint32_t da = deg[a], db = deg[b];
  return da < db || (da == db && a < b);
}

// |N(a) intersect N(b)| counted by the calling group: walk N(a), each lane probes its
// neighbour in b's table.  Returns the group total in every lane.
__device__ inline uint64_t group_intersect(const DView& U, uint32_t a, uint32_t b) {
  const Table tb = group_table(U, b);
  uint64_t c = 0;
  for_each_slab(U, a, [&](uint64_t x, bool data) {
    const uint32_t k = (uint32_t)x;
    if (data && valid_key(k) && k != b) c += lane_has(U, tb, k);
  });
  return gsum_u64(c);
}

// Static count: every undirected edge {u, v} once, from its lower-(degree, id) end.
__global__ void __launch_bounds__(kBlock) k_tc_static(DView U, uint32_t nv, const uint32_t* heavy,
                                                      const uint32_t* nheavy,
                                                      unsigned long long* acc) {
  uint64_t local = 0;
  auto per_vertex = [&](uint32_t u, uint32_t b0, uint32_t stride) {
    for_each_slab_strided(U, u, b0, stride, [&](uint64_t x, bool data) {
      const uint32_t v = (uint32_t)x;
      uint32_t todo = gballot(data && valid_key(v) && ranks_before(U.deg, u, v));
      while (todo) {
        const int l = __builtin_ctz(todo);
        todo &= todo - 1;
        const uint32_t vv = gbcast(v, l);
        const uint64_t c = group_intersect(U, u, vv);
        if (glane() == 0) local += c;
      }
    });
  };
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  for (uint32_t u = g0; u < nv; u += ng) {
    if (U.nbk[u] > kHeavyBuckets || U.deg[u] < 2) continue;
    per_vertex(u, 0, 1);
  }
  const uint32_t nh = *nheavy, gib = threadIdx.x / kGroup;
  for (uint32_t j = blockIdx.x; j < nh; j += gridDim.x) per_vertex(heavy[j], gib, kGroupsPerBlock);
  if (glane() == 0 && local) atomicAdd(acc, (unsigned long long)local);
}

// Keys of the batch graph: both directions of each effective undirected change, or a
// sentinel (vertex N) that sorts last.
__global__ void k_tc_keys(Log lg, uint64_t n, uint32_t nv, uint64_t* keys) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t k0 = (uint64_t)nv << 32, k1 = k0;
    if (lg.uf[i]) {
      const uint32_t a = min(lg.s[i], lg.d[i]), b = max(lg.s[i], lg.d[i]);
      k0 = ((uint64_t)a << 32) | b;
      k1 = ((uint64_t)b << 32) | a;
    }
    keys[2 * i] = k0;
    keys[2 * i + 1] = k1;
  }
}

__device__ inline uint64_t lower_bound_u64(const uint64_t* a, uint64_t n, uint64_t key) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Where each source's arcs start and end in the sorted batch keys (every vertex of a batch
// arc is the source of the reverse arc too, so both ends of an arc have a segment).
__global__ void k_tc_segs(const uint64_t* keys, uint64_t nk, uint32_t nv, uint32_t* seg_lo, uint32_t* seg_hi) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nk;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t src = (uint32_t)(keys[i] >> 32);
    if (src >= nv) continue;  // sentinels sort last
    if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != src) seg_lo[src] = (uint32_t)i;
    if (i + 1 == nk || (uint32_t)(keys[i + 1] >> 32) != src) seg_hi[src] = (uint32_t)(i + 1);
  }
}

// Which end of a canonical batch edge {u, v} (u < v) is walked for S1: the end of smaller
// live degree (ties: u).  The other end, b, is the one whose neighbourhood is looked up.
__device__ inline bool tc_walk_u(const DView& U, uint32_t u, uint32_t v) { return U.deg[u] <= U.deg[v]; }
// The walked end of the batch edge {x, y}, in either order.
__device__ inline uint32_t tc_walked(const DView& U, uint32_t x, uint32_t y) {
  const uint32_t u = min(x, y), v = max(x, y);
  return tc_walk_u(U, u, v) ? u : v;
}

// A vertex b with more than kTcHubDeg neighbours and at least kTcHubEdges batch edges is a
// hub; so is one with more than kTcHubBig neighbours and fewer batch edges when one of its
// batch partners has more than kTcHubDeg neighbours (that edge's walk would otherwise take
// hundreds of slabs on one 16-lane group, the tail of a small batch; a large vertex whose few
// partners are small costs less by probing, the common case after uniform inserts).  Every
// caller sees b's segment [lo, hi) of the sorted batch keys.
// The S1 terms of the batch edges whose looked-up end is a hub, the S2 terms of every batch
// arc leaving a hub and of every arc into a hub from its walked end, are counted by k_tc_hub,
// which loads the hub's neighbourhood into an LDS hash set once for all of them (a smaller
// vertex with few batch edges costs less by probing).  Every other term is counted by
// k_tc_batch, one group per batch arc.
constexpr uint32_t kTcHubDeg = 512;
constexpr uint32_t kTcHubEdges = 4;
constexpr uint32_t kTcHubBig = 2048;
__device__ inline bool tc_is_hub(const DView& U, uint32_t b, const uint64_t* keys, uint32_t lo, uint32_t hi) {
  const uint32_t d = U.deg[b];
  if (d <= kTcHubDeg) return false;
  if (hi - lo >= kTcHubEdges) return true;
  if (d <= kTcHubBig) return false;
  for (uint32_t i = lo; i < hi; ++i)  // fewer than kTcHubEdges entries
    if (U.deg[(uint32_t)keys[i]] > kTcHubDeg) return true;
  return false;
}

// S1, S2 and S3 of the batch identity, one group per batch arc (u, v):
//   S1 += |N_G(u) & N_G(v)|, S2 += |N_G(u) & N_B(v)|, S3 += |N_B(u) & N_B(v)|
// with G the graph after the batch and B the graph of the batch alone (S1 and S3 on the
// canonical direction u < v, counted twice).  The terms k_tc_hub counts are skipped.
__global__ void __launch_bounds__(kBlock) k_tc_batch(DView U, const uint64_t* keys, uint64_t nk,
                                                     const uint32_t* seg_lo, const uint32_t* seg_hi,
                                                     uint32_t nv, bool s2in, unsigned long long* S) {
  const uint64_t g0 = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint64_t ng = (uint64_t)gridDim.x * kGroupsPerBlock;
  uint64_t s1 = 0, s2 = 0, s3 = 0;
  const int gl = glane();
  for (uint64_t i = g0; i < nk; i += ng) {
    const uint64_t key = keys[i];
    const uint32_t u = (uint32_t)(key >> 32), v = (uint32_t)key;
    if (u >= nv) break;  // sentinels sort last
    const bool canon = u < v;
    const uint32_t a = tc_walked(U, u, v), b = a == u ? v : u;
    const bool hub = tc_is_hub(U, b, keys, seg_lo[b], seg_hi[b]);
    uint64_t c1 = 0;
    if (canon && !hub) c1 = 2 * group_intersect(U, a, b);  // walk the smaller side, probe the other
    // batch neighbourhoods: the segments of v and u in the sorted key list
    const uint64_t vlo = seg_lo[v], vhi = seg_hi[v];
    const uint64_t ulo = seg_lo[u], uhi = seg_hi[u];
    auto in_seg = [&](uint64_t lo, uint64_t hi, uint32_t src, uint32_t x) {
      const uint64_t want = ((uint64_t)src << 32) | x;
      const uint64_t q = lower_bound_u64(keys + lo, hi - lo, want);
      return q < hi - lo && keys[lo + q] == want;
    };
    uint64_t c2 = 0, c3 = 0;
    if (tc_is_hub(U, u, keys, (uint32_t)ulo, (uint32_t)uhi)) {
      // S2 of a hub's directions is counted by k_tc_hub against its LDS sets
    } else if (s2in && tc_is_hub(U, v, keys, (uint32_t)vlo, (uint32_t)vhi) && a == u) {
      // so is S2 of an arc into a hub from the end walked against the hub's set
    } else if (2ull * U.deg[u] < vhi - vlo) {
      // S2 from the smaller side: walk N_G(u), look each key up in v's sorted segment
      for_each_slab(U, u, [&](uint64_t w, bool data) {
        const uint32_t x = (uint32_t)w;
        if (data && valid_key(x)) c2 += in_seg(vlo, vhi, v, x);
      });
    } else {
      // S2 by probing: every x of N_B(v) in u's table
      const Table tu = group_table(U, u);
      for (uint64_t j = vlo + gl; j < vhi; j += kGroup) {
        const uint32_t x = (uint32_t)keys[j];
        if (x != u) c2 += lane_has(U, tu, x);
      }
    }
    if (canon) {
      // S3: the smaller segment's entries looked up in the other segment
      const bool u_short = uhi - ulo <= vhi - vlo;
      const uint64_t lo = u_short ? ulo : vlo, hi = u_short ? uhi : vhi;
      const uint64_t olo = u_short ? vlo : ulo, ohi = u_short ? vhi : uhi;
      const uint32_t other = u_short ? v : u;
      for (uint64_t j = lo + gl; j < hi; j += kGroup) {
        const uint32_t x = (uint32_t)keys[j];
        if (x != other) c3 += 2 * in_seg(olo, ohi, other, x);
      }
    }
    c2 = gsum_u64(c2);
    c3 = gsum_u64(c3);
    if (gl == 0) {
      s1 += c1;
      s2 += c2;
      s3 += c3;
    }
  }
  if (gl == 0) {
    if (s1) atomicAdd(S + 0, (unsigned long long)s1);
    if (s2) atomicAdd(S + 1, (unsigned long long)s2);
    if (s3) atomicAdd(S + 2, (unsigned long long)s3);
  }
}

// ---------------------------------------------------------------- hub edges through LDS sets
// A hub b (tc_is_hub, with its segment in the sorted batch keys) owns the batch edges {a, b}
// whose walked end is a.  Its work is split into items <b, pass p, chunk c>: pass p keeps the
// keys of N(b) whose partition hash is p (P_b passes, so that one pass fits the LDS set),
// chunk c is a run of entries of b's segment.  An item loads its part of N(b) into an LDS
// hash set, then reads the packed list of every partner a in its chunk (spread over the
// whole block) and looks each key of the pass up (S1); it also looks up, for the arcs
// (b, a), every entry of a's batch segment that falls in the pass (S2), and, with b's own
// batch segment in the set as tagged keys, counts S2 of the arcs (a, b) on the same lookups.
//
// The set is bucketized: 4 slots (16 bytes, one LDS read) per bucket, linear probing over
// buckets.  At the set's load factor a lookup mostly reads one bucket, so the lanes of a wave
// rarely wait for each other's probe chains (one slot per probe step cost about twice as
// much in the measurements).
//
// Two classes of hubs, one launch each: a small hub (at most HubClass<true>::kKeys
// neighbours) takes a 256-thread block with a 32 KiB set, four blocks to a CU, so that the
// latency of one item's dependent steps overlaps the others'; a large one takes a
// 1024-thread block with a 128 KiB set, one to a CU, in as many passes as it needs.
template <bool Small>
struct HubClass {
  static constexpr uint32_t kThreads = Small ? 256 : 1024;
  static constexpr uint32_t kSlots = Small ? 8192 : 32768;  // u32 keys of the LDS set
  static constexpr uint32_t kKeys = kSlots * 5 / 16;        // keys per pass (load <= 0.3125)
  static constexpr uint32_t kChunk = Small ? 128 : 512;     // segment entries per item
  static constexpr uint32_t kBlocks = Small ? 1024 : 512;   // persistent blocks
  static_assert(kChunk % 64 == 0 && kChunk <= kThreads && kThreads >= 128, "a wave scans a chunk");
};
constexpr uint32_t kTcHubRun = 8;  // list tasks a wave loads at once
__device__ inline bool tc_small_hub(const DView& U, uint32_t b) { return U.deg[b] <= HubClass<true>::kKeys; }

__device__ inline uint32_t tc_part(uint32_t k, uint32_t P) {
  return (uint32_t)(((uint64_t)(k * 0x85EBCA6Bu) * P) >> 32);
}
// Keys of b's batch segment share b's set, tagged with the top bit (vertex ids stay below
// 2^31 when the tag is in use); the bucket hash ignores that bit, so a key and its tagged
// copy share a home bucket and one probe sees both.
constexpr uint32_t kTcTag = 0x80000000u;
__device__ inline uint32_t tc_bucket(uint32_t k, uint32_t bmask) {
  return ((k & ~kTcTag) * 0x9E3779B1u) >> 9 & bmask;
}
template <bool Small>
__device__ inline uint32_t tc_hub_passes(uint32_t deg) {
  return max(1u, (deg + HubClass<Small>::kKeys - 1) / HubClass<Small>::kKeys);
}

// Insert `key` into the bucketized LDS set of bmask + 1 buckets; false when the set is full.
__device__ inline bool lds_insert(uint32_t* tab, uint32_t bmask, uint32_t key) {
  uint32_t h = tc_bucket(key, bmask);
  for (uint32_t n = 0; n <= bmask; ++n) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t old = atomicCAS(&tab[4 * h + i], kInvalid, key);
      if (old == kInvalid || old == key) return true;
    }
    h = (h + 1) & bmask;
  }
  return false;
}
// Whether `key` is in the set, probing from bucket h on (its hash bucket, or a later one
// when the earlier ones are known full and without it).
__device__ inline bool lds_has_from(const uint32_t* tab, uint32_t bmask, uint32_t key, uint32_t h) {
  for (uint32_t n = 0; n <= bmask; ++n) {
    const uint4 q = reinterpret_cast<const uint4*>(tab)[h];
    if (q.x == key || q.y == key || q.z == key || q.w == key) return true;
    if (q.x == kInvalid || q.y == kInvalid || q.z == kInvalid || q.w == kInvalid) return false;
    h = (h + 1) & bmask;
  }
  return false;
}
__device__ inline bool lds_has(const uint32_t* tab, uint32_t bmask, uint32_t key) {
  return lds_has_from(tab, bmask, key, tc_bucket(key, bmask));
}
// Whether `key` (bit 0) and `tkey` (bit 1) are in the set, probing from bucket h on: both
// lie before the first bucket with an empty slot.
__device__ inline uint32_t lds_has2_from(const uint32_t* tab, uint32_t bmask, uint32_t key, uint32_t tkey,
                                         uint32_t h) {
  uint32_t f = 0;
  for (uint32_t n = 0; n <= bmask; ++n) {
    const uint4 q = reinterpret_cast<const uint4*>(tab)[h];
    if (q.x == key || q.y == key || q.z == key || q.w == key) f |= 1u;
    if (q.x == tkey || q.y == tkey || q.z == tkey || q.w == tkey) f |= 2u;
    if (q.x == kInvalid || q.y == kInvalid || q.z == kInvalid || q.w == kInvalid) break;
    h = (h + 1) & bmask;
  }
  return f;
}

// The last position i < n with off[i] <= t, for a non-decreasing off with off[0] <= t,
// searched by a whole wave at once: each round the 64 lanes test 64 evenly spaced
// positions, so a range of n entries takes ceil(log64 n) rounds of dependent loads instead
// of log2 n.  Every lane of the wave must call it; every lane gets the result.
__device__ inline uint64_t wave_last_le(const uint32_t* off, uint64_t n, uint32_t t) {
  const uint64_t lane = __lane_id();
  uint64_t lo = 0, end = n;
  while (end - lo > 1) {
    const uint64_t step = (end - lo + 63) / 64;
    const uint64_t i = lo + lane * step;
    const unsigned long long m = __ballot(i < end && off[i] <= t);  // a prefix of the lanes
    lo += (uint64_t)(63 - __clzll(m)) * step;
    end = min(end, lo + step);
  }
  return lo;
}

// Packed neighbour lists.  A partner's neighbourhood is read once per hub edge and pass, so
// the partners' keys are first copied out of their slabs into contiguous u32 lists: each
// later read is a coalesced 256-byte run instead of a chain of scattered 128-byte slabs
// that are 15/16 filled with 8-byte words.
//
// k_tc_need marks every vertex walked against a hub's set (the walked end of a batch edge
// whose other end is a hub), exactly the partners k_tc_hub reads.
__global__ void k_tc_need(DView U, const uint64_t* keys, uint64_t nk, const uint32_t* seg_lo,
                          const uint32_t* seg_hi, uint32_t nv, uint32_t* need) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nk;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t key = keys[i];
    const uint32_t b = (uint32_t)(key >> 32), a = (uint32_t)key;
    if (b >= nv) continue;  // sentinels
    if (tc_is_hub(U, b, keys, seg_lo[b], seg_hi[b]) && tc_walked(U, a, b) == a) need[a] = 1;
  }
}

constexpr uint32_t kPackBuckets = 256;  // buckets per packing item (one wave, 4 rounds of 64)

// Per vertex: its list length (the live degree when marked, else 0) and its packing items;
// the mark becomes the vertex's write cursor (0).
__global__ void k_tc_pack_count(DView U, uint32_t nv, uint32_t* need, uint32_t* dcnt, uint32_t* icnt) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    const bool on = need[v] != 0 && U.deg[v] > 0;
    need[v] = 0;
    dcnt[v] = on ? U.deg[v] : 0u;
    icnt[v] = on ? (U.nbk[v] + kPackBuckets - 1) / kPackBuckets : 0u;
  }
}

// One wave per item <vertex a, buckets [q * kPackBuckets, ...)>: a lane walks one bucket
// chain, reading whole slabs; per round the wave reserves room for its valid keys (with one
// atomic on a's cursor when a has several items) and each lane writes its keys at its
// prefix (key order in a list is arbitrary).  Writes stay inside a's range
// [doff[a], doff[a] + deg(a)).
__global__ void __launch_bounds__(kBlock) k_tc_pack(DView U, uint32_t nv, const uint64_t* doff,
                                                    const uint32_t* icnt, const uint32_t* ioff,
                                                    uint32_t* cur, uint32_t* list) {
  if (nv == 0) return;
  const uint32_t total = ioff[nv - 1] + icnt[nv - 1];
  const uint32_t ln = threadIdx.x & 63;
  const uint32_t nw = gridDim.x * (blockDim.x / 64);
  for (uint32_t t = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; t < total; t += nw) {
    const uint32_t a = (uint32_t)wave_last_le(ioff, nv, t);  // ioff[a] <= t < ioff[a] + icnt[a]
    const uint32_t q = t - ioff[a], dv = U.deg[a];
    const uint64_t* hs = slab_ptr(U, a);
    const uint32_t nb = (uint32_t)(ld_word(hs + 15) >> 32);
    const uint32_t xb = nb > 1 ? (uint32_t)ld_word(hs + 14) : 0u;
    const uint32_t bend = min(nb, (q + 1) * kPackBuckets);
    uint32_t* out = list + doff[a];
    const bool single = icnt[a] == 1;  // one item: no other wave writes a's list
    uint32_t own = 0;
    for (uint32_t b0 = q * kPackBuckets; b0 < bend; b0 += 64) {
      const uint32_t bk = b0 + ln;
      uint32_t s = kInvalid;
      int nd = kKeysPerSlab;
      if (bk < bend) {
        s = bk == 0 ? a : xb + bk - 1;
        nd = (bk == 0 && nb > 1) ? kKeysPerSlab - 1 : kKeysPerSlab;
      }
      while (__ballot(s != kInvalid) != 0) {  // wave-uniform: every lane takes every round
        Slab sl;
        uint32_t n = 0;
        const bool act = s != kInvalid;
        if (act) {
          load_slab(U, s, sl);
#pragma unroll
          for (int i = 0; i < kKeysPerSlab; ++i) n += (i < nd && valid_key((uint32_t)sl.w[i])) ? 1u : 0u;
        }
        uint32_t incl = n;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t y = __shfl_up(incl, o);
          if ((int)ln >= o) incl += y;
        }
        uint32_t base = 0;
        if (single) {  // the wave owns a's whole list
          base = own;
          own += __shfl(incl, 63);
        } else {
          if (ln == 63 && incl) base = atomicAdd(cur + a, incl);
          base = __shfl(base, 63);
        }
        base += incl - n;
        if (act) {
#pragma unroll
          for (int i = 0; i < kKeysPerSlab; ++i) {
            const uint32_t key = (uint32_t)sl.w[i];
            if (i < nd && valid_key(key)) {
              if (base < dv) out[base] = key;
              ++base;
            }
          }
          s = (uint32_t)sl.w[15];
          nd = kKeysPerSlab;
        }
      }
    }
  }
}

// Work items per segment start: P_b * ceil(|segment| / chunk) at the first key of a hub's
// segment when the hub is of the class, 0 elsewhere (an exclusive scan numbers the items).
template <bool Small>
__global__ void k_tc_hub_count(DView U, const uint64_t* keys, uint64_t nk, const uint32_t* seg_hi,
                               uint32_t nv, uint32_t* cnt) {
  using H = HubClass<Small>;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nk;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t b = (uint32_t)(keys[i] >> 32);
    uint32_t c = 0;
    if (b < nv && (i == 0 || (uint32_t)(keys[i - 1] >> 32) != b) && tc_is_hub(U, b, keys, (uint32_t)i, seg_hi[b]) &&
        tc_small_hub(U, b) == Small) {
      const uint64_t len = seg_hi[b] - i;
      c = tc_hub_passes<Small>(U.deg[b]) * (uint32_t)((len + H::kChunk - 1) / H::kChunk);
    }
    cnt[i] = c;
  }
}

// Persistent blocks take items from a counter until none is left.
template <bool Small>
__global__ void __launch_bounds__(HubClass<Small>::kThreads) k_tc_hub(DView U, const uint64_t* keys, uint64_t nk,
                                                         const uint32_t* seg_lo, const uint32_t* seg_hi,
                                                         const uint32_t* cnt,
                                                         const uint32_t* off, uint32_t* next,
                                                         const uint32_t* list, const uint64_t* loff,
                                                         bool s2in, unsigned long long* S) {
  using H = HubClass<Small>;
  __shared__ uint4 tab4[H::kSlots / 4];
  uint32_t* tab = reinterpret_cast<uint32_t*>(tab4);
  // per partner: its packed list (start, length) and its 64-key tasks, scanned into pre
  __shared__ uint64_t pbase[H::kChunk], qb[H::kChunk];
  __shared__ uint32_t plen[H::kChunk], ql[H::kChunk], qpre[H::kChunk + 1], nq_s;
  __shared__ uint32_t pslo[H::kChunk], pre2[H::kChunk + 1];  // partners' batch segments
  __shared__ uint32_t item_s[8];
  __shared__ uint32_t full;  // a key found no free slot: this item looks keys up in b's slabs
  __shared__ unsigned long long part[2][H::kThreads / 64];
  const uint32_t total = nk ? off[nk - 1] + cnt[nk - 1] : 0u;
  uint64_t hits = 0, h2 = 0;  // S1 and S2 matches
  while (true) {
    if (threadIdx.x < 64) {  // wave 0 fetches the next item
      uint32_t t = 0;
      if (threadIdx.x == 0) t = atomicAdd(next, 1u);
      t = __shfl(t, 0);
      // the segment start of item t: the last key position with off <= t
      const uint64_t lo = t < total ? wave_last_le(off, nk, t) : 0;
      if (threadIdx.x == 0) item_s[0] = t;
      if (threadIdx.x == 0 && t < total) {
        const uint32_t b = (uint32_t)(keys[lo] >> 32);
        const uint32_t P = tc_hub_passes<Small>(U.deg[b]);
        const uint32_t C = cnt[lo] / P;
        const uint32_t local = t - off[lo];
        const uint64_t c0 = lo + (uint64_t)(local % C) * H::kChunk;
        item_s[1] = b;
        item_s[2] = P;
        item_s[3] = local / C;
        item_s[4] = (uint32_t)c0;
        item_s[5] = (uint32_t)min<uint64_t>(c0 + H::kChunk, seg_hi[b]) - (uint32_t)c0;
      }
    }
    __syncthreads();
    if (item_s[0] >= total) break;  // every thread reads the same value
    // the item, wave-uniform: in scalar registers
    const uint32_t b = __builtin_amdgcn_readfirstlane(item_s[1]), P = __builtin_amdgcn_readfirstlane(item_s[2]);
    const uint32_t p = __builtin_amdgcn_readfirstlane(item_s[3]), c0 = __builtin_amdgcn_readfirstlane(item_s[4]);
    const uint32_t np = __builtin_amdgcn_readfirstlane(item_s[5]);
    // buckets: a power of two, at least 3.2 slots per key of the pass, within the LDS array (a
    // key's first bucket is then rarely full, and a probe rarely reads a second one)
    const uint32_t blo = seg_lo[b], bhi = seg_hi[b];  // b's batch segment: N_B(b)
    const uint32_t want = (U.deg[b] + P - 1) / P + (s2in ? (bhi - blo + P - 1) / P : 0u);
    uint32_t slots = 64;
    while (slots < H::kSlots && slots * 5 < want * 16) slots <<= 1;
    const uint32_t bmask = __builtin_amdgcn_readfirstlane(slots / 4 - 1);
    for (uint32_t i = threadIdx.x; i < slots; i += H::kThreads) tab[i] = kInvalid;
    if (threadIdx.x == 0) full = 0;
    // partners of this chunk: a is walked when tc_walked picks it over b
    for (uint32_t j = threadIdx.x; j < np; j += H::kThreads) {
      const uint32_t a = (uint32_t)keys[c0 + j];
      const uint32_t len = tc_walked(U, a, b) == a ? U.deg[a] : 0u;
      pbase[j] = len ? loff[a] : 0;
      plen[j] = len;
      pslo[j] = seg_lo[a];
      // S2 of the arc (b, a), over a's segment (its length, scanned below); not when a is a
      // hub that walks b against its own set: a's items count that arc with b's tagged keys
      const bool by_a = s2in && tc_walked(U, a, b) == b && tc_is_hub(U, a, keys, seg_lo[a], seg_hi[a]);
      pre2[j] = by_a ? 0u : seg_hi[a] - seg_lo[a];
    }
    if (threadIdx.x == 64) {  // b's bucket count and first extra head slab
      const uint64_t* ps = slab_ptr(U, b);
      const uint32_t nbb0 = (uint32_t)(ld_word(ps + 15) >> 32);
      item_s[6] = nbb0;
      item_s[7] = nbb0 > 1 ? (uint32_t)ld_word(ps + 14) : 0u;
    }
    __syncthreads();
    if (threadIdx.x < 128) {
      // two scans, one wave each, a lane owning H::kChunk / 64 consecutive partners.
      // Wave 0 compacts the partners with a non-empty list, in order, into qb / ql with the
      // exclusive prefix of their 64-key tasks in qpre (qpre[nq] = all tasks); wave 1 turns
      // the partners' batch-segment lengths in pre2 into their exclusive prefix.
      constexpr uint32_t kPer = H::kChunk / 64;
      const uint32_t ln = threadIdx.x & 63;
      const bool w0 = threadIdx.x < 64;
      uint32_t v[kPer], sum = 0, nz = 0;
#pragma unroll
      for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t j = ln * kPer + k;
        v[k] = j >= np ? 0u : w0 ? (plen[j] + 63) / 64 : pre2[j];
        sum += v[k];
        nz += v[k] != 0;
      }
      uint32_t incl = sum, zincl = nz;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o), z = __shfl_up(zincl, o);
        if ((int)ln >= o) {
          incl += t;
          zincl += z;
        }
      }
      uint32_t acc = incl - sum, q = zincl - nz;
#pragma unroll
      for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t j = ln * kPer + k;
        if (w0) {
          if (v[k]) {
            qpre[q] = acc;
            qb[q] = pbase[j];
            ql[q] = plen[j];
            ++q;
          }
        } else if (j < np) {
          pre2[j] = acc;
        }
        acc += v[k];
      }
      if (ln == 63) {
        if (w0) {
          qpre[zincl] = incl;
          nq_s = zincl;
        } else {
          pre2[np] = incl;
        }
      }
    }
    // this pass's keys of N(b), one bucket chain per lane (each lane reads whole slabs, so a
    // wave keeps 64 slab reads in flight)
    const uint32_t nbb = item_s[6], xbb = item_s[7];
    for (uint32_t k = threadIdx.x; k < nbb; k += H::kThreads) {
      uint32_t s = k == 0 ? b : xbb + k - 1;
      int nd = (k == 0 && nbb > 1) ? kKeysPerSlab - 1 : kKeysPerSlab;
      while (true) {
        Slab sl;
        load_slab(U, s, sl);
#pragma unroll
        for (int i = 0; i < kKeysPerSlab; ++i) {
          const uint32_t key = (uint32_t)sl.w[i];
          if (i >= nd || !valid_key(key) || tc_part(key, P) != p) continue;
          if (!lds_insert(tab, bmask, key)) full = 1;
        }
        s = (uint32_t)sl.w[15];
        if (s == kInvalid) break;
        nd = kKeysPerSlab;
      }
    }
    if (s2in) {  // and this pass's keys of N_B(b), tagged
      for (uint32_t j = blo + threadIdx.x; j < bhi; j += H::kThreads) {
        const uint32_t x = (uint32_t)keys[j];
        if (tc_part(x, P) == p && !lds_insert(tab, bmask, x | kTcTag)) full = 1;
      }
    }
    __syncthreads();
    const bool in_lds = full == 0;
    const Table tb{b, nbb, xbb};
    // S2 of the arcs (b, a): N_B(a) of every partner a against this pass's keys of N(b), one
    // segment entry per lane
    const uint32_t tasks2 = pre2[np];
    for (uint32_t t = threadIdx.x; t < tasks2; t += H::kThreads) {
      uint32_t lo = 0, hi = np;  // the partner j with pre2[j] <= t < pre2[j + 1]
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre2[mid] <= t) lo = mid;
        else hi = mid;
      }
      const uint32_t x = (uint32_t)keys[pslo[lo] + (t - pre2[lo])];
      if (x == b || tc_part(x, P) != p) continue;
      h2 += in_lds ? lds_has(tab, bmask, x) : lane_has(U, tb, x);
    }
    // the partners' packed lists against this pass's keys of N(b).  Wave w takes a run of
    // consecutive 64-key tasks, kTcHubRun at a time: the tasks' partners come from kTcHubRun
    // lookahead prefixes (a partner has at least one task), the keys from one coalesced load
    // per task, and each key's first bucket from one LDS read, all issued before any is used.
    // Everything that selects a task's partner is wave-uniform and kept in scalar registers
    // (readfirstlane), so the vector units only form addresses, hash and compare keys.
    const uint32_t nq = __builtin_amdgcn_readfirstlane(nq_s);
    const uint32_t tasks = __builtin_amdgcn_readfirstlane(qpre[nq]);
    const uint32_t per = (tasks + H::kThreads / 64 - 1) / (H::kThreads / 64);
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t tb0 = min(tasks, wv * per), te = min(tasks, tb0 + per);
    const uint32_t lane = threadIdx.x & 63;
    uint32_t j = 0;  // the partner of task tb0: the last j with qpre[j] <= tb0
    if (tb0 < te) {
      uint32_t hi = nq;
      while (hi - j > 1) {
        const uint32_t mid = (j + hi) >> 1;
        if (__builtin_amdgcn_readfirstlane(qpre[mid]) <= tb0) j = mid;
        else hi = mid;
      }
    }
    // a run's partners are j .. j + kTcHubRun - 1: their prefixes, lengths and list starts are
    // read at once, and each task selects its own by the count of prefixes at or below it
    auto runs = [&](auto&& probe) {
      for (uint32_t t0 = tb0; t0 < te; t0 += kTcHubRun) {
        uint32_t nx[kTcHubRun], ln_[kTcHubRun], blo[kTcHubRun], bhi[kTcHubRun];
#pragma unroll
        for (uint32_t k = 0; k < kTcHubRun; ++k) {
          nx[k] = __builtin_amdgcn_readfirstlane(qpre[min(j + 1 + k, nq)]);
          ln_[k] = __builtin_amdgcn_readfirstlane(ql[min(j + k, nq - 1)]);
          const uint64_t bq = qb[min(j + k, nq - 1)];
          blo[k] = __builtin_amdgcn_readfirstlane((uint32_t)bq);
          bhi[k] = __builtin_amdgcn_readfirstlane((uint32_t)(bq >> 32));
        }
        const uint32_t pj = __builtin_amdgcn_readfirstlane(qpre[j]);
        uint32_t key[kTcHubRun];
#pragma unroll
        for (uint32_t r = 0; r < kTcHubRun; ++r) {
          const uint32_t t = t0 + r;  // its partner is j + c, c <= r (a partner has >= 1 task)
          uint32_t start = pj, len = ln_[0], lo = blo[0], hi = bhi[0];
#pragma unroll
          for (uint32_t k = 0; k + 1 < kTcHubRun; ++k)
            if (nx[k] <= t) {
              start = nx[k];
              len = ln_[k + 1];
              lo = blo[k + 1];
              hi = bhi[k + 1];
            }
          const uint32_t pos = (t - start) * 64 + lane;
          const uint32_t* src = list + (((uint64_t)hi << 32) | lo);
          key[r] = t < te && pos < len ? src[pos] : kInvalid;
        }
        uint32_t cn = 0;  // the partner of the next run's first task, t0 + kTcHubRun: j + cn
#pragma unroll
        for (uint32_t k = 0; k < kTcHubRun; ++k) cn += nx[k] <= t0 + kTcHubRun;
        j = min(j + cn, nq - 1);
        const uint64_t f = probe(key);  // S1 matches, and S2 matches << 32
        hits += (uint32_t)f;
        h2 += f >> 32;
      }
    };
    // keys of this pass: all of them when b takes one pass
    auto wanted = [&](uint32_t x) { return x != kInvalid && x != b && (P == 1 || tc_part(x, P) == p); };
    // With s2in, a key x of N(a) found tagged counts S2 of the arc (a, b): x in N_B(b).
    if (in_lds) {
      runs([&](const uint32_t (&key)[kTcHubRun]) -> uint64_t {
        uint32_t h[kTcHubRun];
        uint4 q4[kTcHubRun];
#pragma unroll
        for (uint32_t r = 0; r < kTcHubRun; ++r) {  // every first bucket, before any is tested
          h[r] = tc_bucket(key[r], bmask);
          q4[r] = tab4[h[r]];
        }
        uint32_t n = 0, n2 = 0, pend = 0, got = 0;
#pragma unroll
        for (uint32_t r = 0; r < kTcHubRun; ++r) {
          const uint32_t x = key[r], tx = s2in ? x | kTcTag : kInvalid;
          if (!wanted(x)) continue;
          const bool f1 = q4[r].x == x || q4[r].y == x || q4[r].z == x || q4[r].w == x;
          const bool f2 = s2in && (q4[r].x == tx || q4[r].y == tx || q4[r].z == tx || q4[r].w == tx);
          n += f1;
          n2 += f2;
          got |= (f1 ? 1u : 0u) << (2 * r) | (f2 ? 2u : 0u) << (2 * r);
          const bool fullb = q4[r].x != kInvalid && q4[r].y != kInvalid && q4[r].z != kInvalid && q4[r].w != kInvalid;
          if (fullb && (!f1 || (s2in && !f2))) pend |= 1u << r;  // a full first bucket
        }
        while (pend) {  // keys whose first bucket was full, all runs of the wave at once
          const uint32_t r = __builtin_ctz(pend);
          pend &= pend - 1;
          uint32_t x = key[0], hh = h[0];
#pragma unroll
          for (uint32_t k = 1; k < kTcHubRun; ++k)
            if (k == r) {
              x = key[k];
              hh = h[k];
            }
          const uint32_t f = lds_has2_from(tab, bmask, x, s2in ? x | kTcTag : kInvalid, (hh + 1) & bmask) &
                             ~(got >> (2 * r));
          n += f & 1u;
          n2 += s2in ? (f >> 1) & 1u : 0u;
        }
        return ((uint64_t)n2 << 32) | n;
      });
    } else {  // the pass overflowed its set: look the keys up in b's slabs and b's segment
      runs([&](const uint32_t (&key)[kTcHubRun]) -> uint64_t {
        uint32_t n = 0, n2 = 0;
#pragma unroll 1
        for (uint32_t r = 0; r < kTcHubRun; ++r) {
          if (!wanted(key[r])) continue;
          n += lane_has(U, tb, key[r]);
          if (s2in) {
            const uint64_t want_k = ((uint64_t)b << 32) | key[r];
            const uint64_t q = lower_bound_u64(keys + blo, bhi - blo, want_k);
            n2 += q < bhi - blo && keys[blo + q] == want_k;
          }
        }
        return ((uint64_t)n2 << 32) | n;
      });
    }
    __syncthreads();  // the set and partner arrays are rebuilt by the next item
  }
  // an S1 match counts twice (S1 adds both directions of an edge)
  uint64_t hs[2] = {2 * hits, h2};
  for (int k = 0; k < 2; ++k) {
    for (int o = 32; o > 0; o >>= 1) hs[k] += __shfl_xor(hs[k], o);
    if ((threadIdx.x & 63) == 0) part[k][threadIdx.x >> 6] = hs[k];
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    unsigned long long t = 0;
    for (uint32_t i = 0; i < H::kThreads / 64; ++i) t += part[threadIdx.x][i];
    if (t) atomicAdd(S + threadIdx.x, t);
  }
}

__global__ void k_tc_begin(Counters* C, bool reset_total) {
  if (threadIdx.x != 0) return;
  C->tc_s[0] = C->tc_s[1] = C->tc_s[2] = 0;
  C->u64tmp[0] = 0;
  if (reset_total) C->tc_total = 0;
}

// insert: T += (S1 - S2 + S3/3) / 2;  delete: T -= (S1 + S2 + S3/3) / 2;  static: T = sum / 3
__global__ void k_tc_finish(Counters* C, int kind, unsigned long long* out) {
  if (threadIdx.x != 0) return;
  const unsigned long long s1 = C->tc_s[0], s2 = C->tc_s[1], s3 = C->tc_s[2];
  if (kind == 0) C->tc_total += (s1 - s2 + s3 / 3) / 2;
  else if (kind == 1) C->tc_total -= (s1 + s2 + s3 / 3) / 2;
  else C->tc_total = C->u64tmp[0] / 3;
  if (out) *out = C->tc_total;
}

Log log_at(const mk_graph* g, uint64_t off) {
  Log l = g->log;
  l.s += off;
  l.d += off;
  l.w += off;
  l.st += off;
  l.uf += off;
  return l;
}

// PageRank iterations under IterationScheme2 from the ranks in g->pr_x (the caller has
// initialized or kept them): contributions, one group per reverse-view bucket chain, then
// the per-vertex sums in bucket order.
mk_status pagerank_scheme2(mk_graph* g, float damping, double tol_l1, uint32_t max_iter, float* d_rank,
                           uint32_t* d_iters, hipStream_t stream) {
  const uint32_t N = g->n;
  if (mk_status st = ensure_pairs(g, VR, stream); st != MK_OK) return st;
  const ViewHost& vh = g->view[VR];
  hipLaunchKernelGGL(k_pr_start, dim3(1), dim3(64), 0, stream, g->ctr);
  float* buf[2] = {g->pr_x, g->pr_y};
  const uint32_t cb = blocks_for(N, kPrContribBlocks);
  double* dpart = g->pr_part + kPrContribBlocks;
  uint32_t it = 0;
  while (true) {
    for (int k = 0; k < kPrSyncEvery; ++k, ++it) {
      const int slot = it & 3;
      const float* x = buf[it & 1];
      float* y = buf[(it + 1) & 1];
      double* dang = &g->ctr->pr_acc[2 * slot];
      hipLaunchKernelGGL(k_pr_contrib, dim3(cb), dim3(kBlock), 0, stream, x, g->view[VF].d.deg, g->pr_c,
                         N, g->pr_part, g->ctr->pr_state, nullptr, nullptr);
      hipLaunchKernelGGL(k_pr_sum, dim3(1), dim3(kBlock), 0, stream, g->pr_part, cb, dang, g->ctr->pr_state);
      hipLaunchKernelGGL(k_pr_gather_s2, dim3(kWalkBlocks), dim3(kBlock), 0, stream, vh.d, g->pr_c,
                         vh.pair_v, vh.pair_i, (uint32_t)vh.n_head, N, g->pr_pair, g->ctr->pr_state);
      hipLaunchKernelGGL(k_pr_final_s2, dim3(kWalkBlocks), dim3(kBlock), 0, stream, vh.nbk, vh.pair_off,
                         g->pr_pair, x, y, N, damping, dang, dpart, g->ctr->pr_state);
      hipLaunchKernelGGL(k_pr_check, dim3(1), dim3(kBlock), 0, stream, g->ctr, slot, tol_l1, max_iter, dpart,
                         kWalkBlocks);
      MK_LAUNCH(g, "pagerank iteration (scheme 2)");
    }
    MK_HIP(g, hipMemcpyAsync(g->h_pin, g->ctr->pr_state, 8, hipMemcpyDeviceToHost, stream));
    MK_HIP(g, hipStreamSynchronize(stream));
    if (reinterpret_cast<const uint32_t*>(g->h_pin)[0]) break;
  }
  hipLaunchKernelGGL(k_pr_final, dim3(blocks_for(N)), dim3(kBlock), 0, stream, g->ctr, g->pr_x,
                     g->pr_y, g->pr_x, d_rank, N, d_iters);
  MK_LAUNCH(g, "pagerank final");
  g->pr.valid = true;
  mark_seen(g, g->pr);
  return MK_OK;
}

}  // namespace

extern "C" {

mk_status mk_incr_wcc(mk_graph* g, uint32_t* d_label, mk_mode mode, hipStream_t stream) {
  return mk_incr_wcc_scheme(g, d_label, mode, MK_WCC_LOG, stream);
}

mk_status mk_incr_wcc_scheme(mk_graph* g, uint32_t* d_label, mk_mode mode, mk_wcc_scheme scheme,
                             hipStream_t stream) {
  if (!g || !d_label || (uint32_t)scheme > (uint32_t)MK_WCC_UPDATE) return MK_ERR_INVALID_ARG;
  if (mk_status gs = graph_guard(g); gs != MK_OK) return gs;
  const uint32_t N = g->n;
  Pending p = pending_for(g, g->wcc);
  bool full = mode == MK_RECOMPUTE || !g->wcc.valid || p.lost || (p.kinds & 2);
  if (!full && mode == MK_AUTO)
    if (mk_status s = auto_prefers_recompute(g, MK_ALGO_WCC, p, stream, &full); s != MK_OK) return s;
  uint32_t* P = g->wcc_parent;
  const DView F = g->view[VF].d;
  auto all_arcs = [&]() -> mk_status {  // union over every arc
    if (g->iter_scheme == MK_ITER_SCHEME2) {  // one group per bucket chain
      if (mk_status st = ensure_pairs(g, VF, stream); st != MK_OK) return st;
      const ViewHost& vh = g->view[VF];
      hipLaunchKernelGGL(k_wcc_pairs, dim3(kWalkBlocks), dim3(kBlock), 0, stream, F, P, vh.pair_v, vh.pair_i,
                         (uint32_t)vh.n_head, N);
      return MK_OK;
    }
    // IterationScheme1, collecting the heavy vertices first
    uint32_t* nh = &g->ctr->n_heavy_wcc;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, nh, 1u);
    hipLaunchKernelGGL(k_collect_heavy, dim3(blocks_for(N)), dim3(kBlock), 0, stream,
                       g->view[VF].nbk, N, g->fq[2], nh);
    hipLaunchKernelGGL(k_wcc_all, dim3(kWalkBlocks), dim3(kBlock), 0, stream, F, P, N, g->fq[2], nh,
                       nullptr);
    return MK_OK;
  };
  // the sampled static WCC: needs the undirected view (both directions of a skipped arc)
  auto sampled = [&]() {
    const DView U = g->view[VU].d;
    uint32_t* nh = &g->ctr->n_heavy_wcc;
    hipLaunchKernelGGL(k_wcc_link_first, dim3(blocks_for(N)), dim3(kBlock), 0, stream, U, P, N);
    hipLaunchKernelGGL(k_wcc_flatten, dim3(blocks_for(N)), dim3(kBlock), 0, stream, P, N);
    hipLaunchKernelGGL(k_wcc_big, dim3(1), dim3(kWccSamples), 0, stream, P, N, &g->ctr->wcc_big);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, nh, 1u);
    hipLaunchKernelGGL(k_collect_heavy, dim3(blocks_for(N)), dim3(kBlock), 0, stream,
                       g->view[VU].nbk, N, g->fq[2], nh);
    hipLaunchKernelGGL(k_wcc_all, dim3(kWalkBlocks), dim3(kBlock), 0, stream, U, P, N, g->fq[2], nh,
                       &g->ctr->wcc_big);
  };
  if (full) {
    hipLaunchKernelGGL(k_wcc_init, dim3(blocks_for(N)), dim3(kBlock), 0, stream, P, N);
    if (g->view[VU].on && g->iter_scheme != MK_ITER_SCHEME2 && N > 0) {
      sampled();
    } else if (mk_status st = all_arcs(); st != MK_OK) {
      return st;
    }
    if (scheme == MK_WCC_UPDATE)
      hipLaunchKernelGGL(k_mark_all, dim3(grid_for_groups(std::min<uint64_t>(g->view[VF].n_head, 1u << 20))),
                         dim3(kBlock), 0, stream, F, g->upd_mark, g->view[VF].n_head, N);
  } else if (!p.list.empty()) {
    if (scheme == MK_WCC_LOG) {
      for (const BatchRec* b : p.list)
        hipLaunchKernelGGL(k_wcc_batch, dim3(blocks_for(b->n)), dim3(kBlock), 0, stream, P,
                           log_at(g, b->off), b->n);
    } else if (scheme == MK_WCC_NAIVE) {
      if (mk_status st = all_arcs(); st != MK_OK) return st;
    } else {
      uint32_t* nl = &g->ctr->n_listed_light;
      uint32_t* nh = &g->ctr->n_listed_heavy;
      hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, nl, 2u);
      uint64_t ops = 0;
      for (const BatchRec* b : p.list) {
        hipLaunchKernelGGL(k_wcc_flag, dim3(blocks_for(b->n)), dim3(kBlock), 0, stream,
                           log_at(g, b->off), b->n, g->view[VF].nbk, g->wcc_flag, g->fq[0], nl,
                           g->fq[1], nh);
        ops += b->n;
      }
      hipLaunchKernelGGL(k_wcc_listed, dim3(blocks_for(ops * kGroup)), dim3(kBlock), 0, stream, F, P,
                         scheme == MK_WCC_UPDATE ? g->upd_mark : nullptr, g->fq[0], nl, g->fq[1], nh);
      hipLaunchKernelGGL(k_wcc_unflag, dim3(blocks_for(ops)), dim3(kBlock), 0, stream, g->wcc_flag,
                         g->fq[0], nl, g->fq[1], nh);
    }
  }
  if (full || !p.list.empty())
    hipLaunchKernelGGL(k_wcc_compress, dim3(blocks_for(N)), dim3(kBlock), 0, stream, P, N, d_label);
  else  // nothing changed: the parents are the compressed labels of the last call
    hipLaunchKernelGGL(k_copy_u32, dim3(blocks_for(N)), dim3(kBlock), 0, stream, P, d_label, N);
  MK_LAUNCH(g, "wcc");
  g->wcc.valid = true;
  mark_seen(g, g->wcc);
  return MK_OK;
}

mk_status mk_incr_pagerank(mk_graph* g, float damping, double tol_l1, uint32_t max_iter,
                           float* d_rank, uint32_t* d_iters, mk_mode mode, hipStream_t stream) {
  if (!g || !d_rank || !(damping >= 0.f && damping < 1.f) || max_iter == 0) return MK_ERR_INVALID_ARG;
  if (!g->view[VR].on) return MK_ERR_STATE;
  const uint32_t N = g->n;
  Pending p = pending_for(g, g->pr);
  if (mk_status gs = graph_guard(g); gs != MK_OK) return gs;
  bool warm = mode != MK_RECOMPUTE && g->pr.valid && !p.lost;
  if (warm && mode == MK_AUTO) {
    bool rec = false;
    if (mk_status s = auto_prefers_recompute(g, MK_ALGO_PAGERANK, p, stream, &rec); s != MK_OK) return s;
    warm = !rec;
  }
  if (warm && p.list.empty()) {
    hipLaunchKernelGGL(k_pr_start, dim3(1), dim3(64), 0, stream, g->ctr);
    hipLaunchKernelGGL(k_pr_final, dim3(blocks_for(N)), dim3(kBlock), 0, stream, g->ctr, g->pr_x,
                       g->pr_y, g->pr_x, d_rank, N, d_iters);
    MK_LAUNCH(g, "pagerank copy");
    return MK_OK;
  }
  if (!warm)
    hipLaunchKernelGGL(k_pr_fill, dim3(blocks_for(N)), dim3(kBlock), 0, stream, g->pr_x, N, 1.f / N);
  if (g->iter_scheme == MK_ITER_SCHEME2) return pagerank_scheme2(g, damping, tol_l1, max_iter, d_rank, d_iters, stream);
  uint32_t* nh = &g->ctr->n_heavy_pr;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, nh, 1u);
  hipLaunchKernelGGL(k_collect_heavy, dim3(blocks_for(N)), dim3(kBlock), 0, stream, g->view[VR].nbk,
                     N, g->heavy_rev, nh);
  // heavy-vertex work items: counts, exclusive offsets, FP64 partial sums (scratch: the
  // traversal queues, which PageRank does not use)
  uint32_t* hcnt = g->fq[0];
  uint32_t* hoff = g->fq[1];
  double* hacc = g->pr_hacc;
  hipLaunchKernelGGL(k_heavy_items, dim3(blocks_for(N)), dim3(kBlock), 0, stream, g->view[VR].nbk,
                     g->heavy_rev, nh, hcnt, hacc);
  {
    size_t tb = g->scan_tmp_bytes;
    if (rocprim::exclusive_scan(g->scan_tmp, tb, hcnt, hoff, 0u, (size_t)N, rocprim::plus<uint32_t>(),
                                stream) != hipSuccess)
      return MK_ERR_HIP;
  }
  // packed iterations: the first one walks the slabs and packs the in-arc keys at the
  // exclusive scan of the in-degrees; the heavy vertices' pull items and packing cursors
  // use three more traversal queues
  const bool packed = g->iter_scheme == MK_ITER_PACKED && g->pr_list;
  const DView& Rd = g->view[VR].d;
  uint32_t* pcnt = g->fq[2];
  uint32_t* poff = g->fq[3];
  uint32_t* pcur = g->fq[4];
  if (packed) {
    size_t tb = g->scan_tmp_bytes;
    if (rocprim::exclusive_scan(g->scan_tmp, tb, Rd.deg, g->pr_off, 0u, (size_t)N, rocprim::plus<uint32_t>(),
                                stream) != hipSuccess)
      return MK_ERR_HIP;
    // hot-first ranks of the sources (out-degrees change with every batch: once per call)
    hipLaunchKernelGGL(k_pr_class, dim3(blocks_for(N)), dim3(kBlock), 0, stream, g->view[VF].d.deg, N,
                       g->pr_skey[0], g->pr_sidx);
    size_t sb = g->pr_sort_bytes;
    if (rocprim::radix_sort_pairs(g->pr_sort_tmp, sb, g->pr_skey[0], g->pr_skey[1], g->pr_sidx, g->pr_perm,
                                  (size_t)N, 0, 6, stream) != hipSuccess)
      return MK_ERR_HIP;
    hipLaunchKernelGGL(k_pr_rank, dim3(blocks_for(N)), dim3(kBlock), 0, stream, g->pr_perm, N, g->pr_rank);
    hipLaunchKernelGGL(k_pull_end, dim3(1), dim3(64), 0, stream, Rd.deg, g->pr_off, N);
    hipLaunchKernelGGL(k_pull_items, dim3(blocks_for(N)), dim3(kBlock), 0, stream, Rd.deg, g->heavy_rev, nh,
                       g->pr_off, pcnt, pcur);
    size_t tb2 = g->scan_tmp_bytes;
    if (rocprim::exclusive_scan(g->scan_tmp, tb2, pcnt, poff, 0u, (size_t)N, rocprim::plus<uint32_t>(),
                                stream) != hipSuccess)
      return MK_ERR_HIP;
  }
  hipLaunchKernelGGL(k_pr_start, dim3(1), dim3(64), 0, stream, g->ctr);
  MK_LAUNCH(g, "pagerank setup");
  float* buf[2] = {g->pr_x, g->pr_y};
  // per-block partial sums: the dangling mass (contribution blocks), then the L1 change
  // (gather blocks, heavy-final blocks)
  const uint32_t cb = blocks_for(N, kPrContribBlocks), hb = blocks_for(N, kPrFinalBlocks);
  double* dpart = g->pr_part + kPrContribBlocks;
  uint32_t it = 0;
  while (true) {
    for (int k = 0; k < kPrSyncEvery; ++k, ++it) {
      const int slot = it & 3;
      const float* x = buf[it & 1];
      float* y = buf[(it + 1) & 1];
      double* dang = &g->ctr->pr_acc[2 * slot];
      if (packed && it > 0)
        hipLaunchKernelGGL(k_pr_contrib_perm, dim3(cb), dim3(kBlock), 0, stream, x, g->view[VF].d.deg,
                           g->pr_perm, g->pr_cp, N, g->pr_part, g->ctr->pr_state);
      else  // the first iteration; with packing, <rank, contribution> pairs
        hipLaunchKernelGGL(k_pr_contrib, dim3(cb), dim3(kBlock), 0, stream, x, g->view[VF].d.deg, g->pr_c,
                           N, g->pr_part, g->ctr->pr_state, packed ? g->pr_rank : nullptr,
                           packed ? reinterpret_cast<uint2*>(g->pr_cr) : nullptr);
      hipLaunchKernelGGL(k_pr_sum, dim3(1), dim3(kBlock), 0, stream, g->pr_part, cb, dang, g->ctr->pr_state);
      if (packed && it > 0)
        hipLaunchKernelGGL(k_pr_pull, dim3(kWalkBlocks), dim3(kBlock), 0, stream, Rd.nbk, Rd.deg, g->pr_off,
                           g->pr_list, g->pr_cp, x, y, N, damping, dang, dpart, g->heavy_rev, nh, pcnt, poff,
                           hacc, g->ctr->pr_state);
      else
        hipLaunchKernelGGL(k_pr_gather, dim3(kWalkBlocks), dim3(kBlock), 0, stream, Rd, g->pr_c, x, y, N,
                           damping, dang, dpart, g->heavy_rev, nh, hcnt, hoff, hacc, g->ctr->pr_state,
                           packed ? g->pr_list : nullptr, g->pr_off, pcur,
                           reinterpret_cast<const uint2*>(g->pr_cr));
      hipLaunchKernelGGL(k_pr_heavy_final, dim3(hb), dim3(kBlock), 0, stream, g->heavy_rev, nh, hacc, x, y,
                         N, damping, dang, dpart + kWalkBlocks, g->ctr->pr_state);
      hipLaunchKernelGGL(k_pr_check, dim3(1), dim3(kBlock), 0, stream, g->ctr, slot, tol_l1, max_iter, dpart,
                         kWalkBlocks + hb);
      MK_LAUNCH(g, "pagerank iteration");
    }
    MK_HIP(g, hipMemcpyAsync(g->h_pin, g->ctr->pr_state, 8, hipMemcpyDeviceToHost, stream));
    MK_HIP(g, hipStreamSynchronize(stream));
    if (reinterpret_cast<const uint32_t*>(g->h_pin)[0]) break;
  }
  hipLaunchKernelGGL(k_pr_final, dim3(blocks_for(N)), dim3(kBlock), 0, stream, g->ctr, g->pr_x,
                     g->pr_y, g->pr_x, d_rank, N, d_iters);
  MK_LAUNCH(g, "pagerank final");
  g->pr.valid = true;
  mark_seen(g, g->pr);
  return MK_OK;
}

mk_status mk_count_triangles(mk_graph* g, uint64_t* d_count, mk_mode mode, hipStream_t stream) {
  if (!g || !d_count) return MK_ERR_INVALID_ARG;
  if (!g->view[VU].on) return MK_ERR_STATE;
  const uint32_t N = g->n;
  const DView U = g->view[VU].d;
  if (mk_status gs = graph_guard(g); gs != MK_OK) return gs;
  Pending p = pending_for(g, g->tc);
  bool full = mode == MK_RECOMPUTE || !g->tc.valid || p.lost || p.kinds == 3;
  if (!full && mode == MK_AUTO)
    if (mk_status s = auto_prefers_recompute(g, MK_ALGO_TC, p, stream, &full); s != MK_OK) return s;
  unsigned long long* out = reinterpret_cast<unsigned long long*>(d_count);
  if (full) {
    uint32_t* nh = &g->ctr->n_heavy_tc;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, nh, 1u);
    hipLaunchKernelGGL(k_collect_heavy, dim3(blocks_for(N)), dim3(kBlock), 0, stream, U.nbk, N,
                       g->fq[2], nh);
    hipLaunchKernelGGL(k_tc_begin, dim3(1), dim3(64), 0, stream, g->ctr, true);
    hipLaunchKernelGGL(k_tc_static, dim3(kWalkBlocks), dim3(kBlock), 0, stream, U, N, g->fq[2], nh,
                       &g->ctr->u64tmp[0]);
    hipLaunchKernelGGL(k_tc_finish, dim3(1), dim3(64), 0, stream, g->ctr, 2, out);
  } else if (p.list.empty()) {
    hipLaunchKernelGGL(k_tc_finish, dim3(1), dim3(64), 0, stream, g->ctr, 3, out);
  } else {
    // all pending batches are of one kind: their union is one effective batch
    uint64_t nk = 0;
    for (const BatchRec* b : p.list) {
      hipLaunchKernelGGL(k_tc_keys, dim3(blocks_for(b->n)), dim3(kBlock), 0, stream,
                         log_at(g, b->off), b->n, N, g->tc_keys[0] + nk);
      nk += 2 * b->n;
    }
    if (nk > 2 * g->log_cap) return MK_ERR_CAPACITY;
    unsigned end_bit = 32;
    while (end_bit < 64 && ((uint64_t)N >> (end_bit - 32)) != 0) ++end_bit;
    size_t tb = g->sort_tmp_bytes;
    if (rocprim::radix_sort_keys(g->sort_tmp, tb, g->tc_keys[0], g->tc_keys[1], (size_t)nk, 0,
                                 end_bit, stream) != hipSuccess)
      return MK_ERR_HIP;
    hipLaunchKernelGGL(k_tc_begin, dim3(1), dim3(64), 0, stream, g->ctr, false);
    // segment bounds per source vertex (scratch: two traversal queues, unused here)
    hipLaunchKernelGGL(k_tc_segs, dim3(blocks_for(nk)), dim3(kBlock), 0, stream, g->tc_keys[1], nk, N,
                       g->fq[4], g->fq[5]);
    // S2 of arcs into hubs goes through the hubs' sets when ids leave the tag bit free
    const bool s2in = N <= 0x7FFFFFFFu;
    hipLaunchKernelGGL(k_tc_batch, dim3(grid_for_groups(std::min<uint64_t>(nk, 1u << 20))),
                       dim3(kBlock), 0, stream, U, g->tc_keys[1], nk, g->fq[4], g->fq[5], N, s2in,
                       g->ctr->tc_s);
    // hub edges: work items numbered by an exclusive scan over the key
    // positions, in the sort's input buffer (free after the sort; 2 * nk u32 fit in it)
    uint32_t* hcnt = reinterpret_cast<uint32_t*>(g->tc_keys[0]);
    uint32_t* hoff = hcnt + nk;
    // packed lists of the hub partners (scratch: the other traversal queues)
    uint32_t *dcnt = g->fq[0], *icnt = g->fq[1], *ioff = g->fq[2], *need = g->fq[3];
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(N)), dim3(kBlock), 0, stream, need, N);
    hipLaunchKernelGGL(k_tc_need, dim3(blocks_for(nk)), dim3(kBlock), 0, stream, U, g->tc_keys[1], nk,
                       g->fq[4], g->fq[5], N, need);
    hipLaunchKernelGGL(k_tc_pack_count, dim3(blocks_for(N)), dim3(kBlock), 0, stream, U, N, need, dcnt, icnt);
    {
      size_t tb2 = g->scan_tmp_bytes;
      if (rocprim::exclusive_scan(g->scan_tmp, tb2, dcnt, g->tc_off, (uint64_t)0, (size_t)N,
                                  rocprim::plus<uint64_t>(), stream) != hipSuccess)
        return MK_ERR_HIP;
      tb2 = g->scan_tmp_bytes;
      if (rocprim::exclusive_scan(g->scan_tmp, tb2, icnt, ioff, 0u, (size_t)N, rocprim::plus<uint32_t>(),
                                  stream) != hipSuccess)
        return MK_ERR_HIP;
    }
    hipLaunchKernelGGL(k_tc_pack, dim3(kWalkBlocks), dim3(kBlock), 0, stream, U, N, g->tc_off, icnt, ioff, need,
                       g->tc_list);
    // the small hubs' items, then the large ones' (the item numbering is redone per class)
    auto hub_launch = [&](auto cls) -> bool {
      constexpr bool kSmall = decltype(cls)::value;
      using H = HubClass<kSmall>;
      hipLaunchKernelGGL(k_tc_hub_count<kSmall>, dim3(blocks_for(nk)), dim3(kBlock), 0, stream, U,
                         g->tc_keys[1], nk, g->fq[5], N, hcnt);
      size_t tb2 = g->scan_tmp_bytes;
      if (rocprim::exclusive_scan(g->scan_tmp, tb2, hcnt, hoff, 0u, (size_t)nk, rocprim::plus<uint32_t>(),
                                  stream) != hipSuccess)
        return false;
      hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, &g->ctr->tc_work, 1u);
      hipLaunchKernelGGL(k_tc_hub<kSmall>, dim3(H::kBlocks), dim3(H::kThreads), 0, stream, U, g->tc_keys[1], nk,
                         g->fq[4], g->fq[5], hcnt, hoff, &g->ctr->tc_work, g->tc_list, g->tc_off, s2in,
                         g->ctr->tc_s);
      return true;
    };
    if (!hub_launch(std::true_type{}) || !hub_launch(std::false_type{})) return MK_ERR_HIP;
    hipLaunchKernelGGL(k_tc_finish, dim3(1), dim3(64), 0, stream, g->ctr,
                       p.kinds == 1 ? 0 : 1, out);
  }
  MK_LAUNCH(g, "triangles");
  g->tc.valid = true;
  mark_seen(g, g->tc);
  return MK_OK;
}

}  // extern "C"
