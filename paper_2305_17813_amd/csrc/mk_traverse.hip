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
//
// Weighted epilogue in distance bands (near-far): an improved vertex joins the frontier
// only if its new distance is below the current band's threshold T, else it waits on a
// far pile.  When the frontier empties, the pile's smallest pending distance f gives the
// next threshold f + delta, the pile entries below it form the next frontier and the
// rest stay.  Any order of relaxations reaches the same unique fixed point; expanding
// nearer vertices first only avoids re-expanding vertices whose distance drops again.
#include <algorithm>

#include "mk_internal.h"

using namespace mk;

namespace {

constexpr uint32_t kExpandBlocks = 2048;  // 256 CUs x 8 resident blocks
constexpr int kSyncFirst = 4, kSyncMax = 16;  // frontier launches between size read-backs: 4,
                                              // then doubling while the frontier lasts

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

// Near-far routing of the weighted epilogue.  T == nullptr: every push is near.
struct Route {
  const uint32_t* T;   // threshold of the current band
  uint32_t* far;       // far pile of the current band and its size
  uint32_t* far_cnt;
  uint32_t* far_mark;  // band id of the last far push of each vertex
  uint32_t band;
};

__device__ inline uint32_t band_limit(const Route& r) { return r.T ? *r.T : 0xFFFFFFFFu; }


// Routed pushes through block stages: a vertex improved to distance `dist` goes to the near
// queues ([0..2] light, heavy, giant of Q) when dist < T, else onto the far pile of r ([3],
// once per band); open_routed opens the four stages.
__device__ inline void open_routed(Stage (&S)[4], const PushQ& Q, const Route& r) {
  for (int k = 0; k < 3; ++k) stage_open(S[k], Q.q[k], Q.c[k]);
  stage_open(S[3], r.far, r.far_cnt);
  __syncthreads();
}

__device__ inline void push_staged(Stage (&S)[4], const uint32_t* nbk, const Route& r, uint32_t T,
                                   uint32_t* mark, uint32_t stamp, bool p, uint32_t v, uint32_t dist) {
  const bool near = p && dist < T;
  bool take = false, take_far = false;
  if (near) take = atomicExch(mark + v, stamp) != stamp;
  else if (p) take_far = atomicExch(r.far_mark + v, r.band) != r.band;
  const uint32_t nb = take ? nbk[v] : 0u;
  stage_push(S[3], take_far, v);
  stage_push(S[0], take && nb <= kHeavyBuckets, v);
  stage_push(S[1], take && nb > kHeavyBuckets && nb <= kGiantBuckets, v);
  stage_push(S[2], take && nb > kGiantBuckets, v);
}

struct Queues {
  const uint32_t* cur[3];  // light, heavy, giant
  PushQ next;
  uint32_t* cnt;  // [3k .. 3k+2]: rotating sizes of queue k
  int icur, iclear;
};

// Stage the keys of the slab words selected by `mask` (bit j: word j) of every active lane.
__device__ inline void stage_words(Stage& S, uint32_t mask, const Slab& sl) {
  bool any;
  const StageSlots t = stage_reserve(S, (uint32_t)__popc(mask), any);
  if (!any) return;
  uint32_t pos = t.pos;
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j)
    if (mask >> j & 1) stage_put(S, t, pos++, (uint32_t)sl.w[j]);
}

// Relax the 15 out-arcs of a whole slab held by one lane.  The distance loads, the atomic
// minima, the frontier marks and the bucket counts are each issued as one independent
// batch, and the pushes of the wave are appended with one counter atomic per queue.
template <bool kUnit>
__device__ inline void relax_slab_lane(const DView& F, uint64_t* D, uint32_t u, uint64_t du, const Slab& sl,
                                       int nd, Stage (&S)[4], const Route& r, uint32_t T, uint32_t* mark,
                                       uint32_t stamp) {
  uint64_t cand[kKeysPerSlab], cur[kKeysPerSlab];
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j) {
    const uint32_t v = (uint32_t)sl.w[j];
    const bool ok = j < nd && valid_key(v);
    cand[j] = ok ? tree_node(du + (kUnit ? 1ull : (sl.w[j] >> 32)), u) : kTreeNone;
    cur[j] = ok ? D[v] : 0ull;
  }
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j)
    cur[j] = cand[j] < cur[j] ? amin64(D + (uint32_t)sl.w[j], cand[j]) : 0ull;
  uint32_t near = 0, far = 0;
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j) {
    if (cur[j] > cand[j]) {
      if ((uint32_t)(cand[j] >> 32) < T) near |= 1u << j;
      else far |= 1u << j;
    }
  }
  uint32_t tk[kKeysPerSlab];
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j) {
    const uint32_t v = (uint32_t)sl.w[j];
    tk[j] = 0;
    if (near >> j & 1) tk[j] = atomicExch(mark + v, stamp);
    else if (far >> j & 1) tk[j] = atomicExch(r.far_mark + v, r.band);
  }
  uint32_t tn = 0, tf = 0;
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j) {
    if ((near >> j & 1) && tk[j] != stamp) tn |= 1u << j;
    if ((far >> j & 1) && tk[j] != r.band) tf |= 1u << j;
  }
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j) tk[j] = (tn >> j & 1) ? F.nbk[(uint32_t)sl.w[j]] : 1u;
  uint32_t heavy = 0, giant = 0;
#pragma unroll
  for (int j = 0; j < kKeysPerSlab; ++j) {
    if (tk[j] > kGiantBuckets) giant |= 1u << j;
    else if (tk[j] > kHeavyBuckets) heavy |= 1u << j;
  }
  stage_words(S[0], tn & ~(heavy | giant), sl);
  stage_words(S[1], heavy, sl);
  stage_words(S[2], giant, sl);
  stage_words(S[3], tf, sl);
}

// Relax every arc in bucket b of u (nb buckets, extra head slabs from xb) with one lane.
template <bool kUnit>
__device__ inline void relax_bucket_lane(const DView& F, uint64_t* D, uint32_t u, uint64_t du, uint32_t b,
                                         uint32_t nb, uint32_t xb, Stage (&S)[4], const Route& r,
                                         uint32_t T, uint32_t* mark, uint32_t stamp) {
  uint32_t t = b == 0 ? u : xb + b - 1;
  int nd = (b == 0 && nb > 1) ? kKeysPerSlab - 1 : kKeysPerSlab;
  Slab sl;
  while (true) {
    load_slab(F, t, sl);
    relax_slab_lane<kUnit>(F, D, u, du, sl, nd, S, r, T, mark, stamp);
    t = (uint32_t)sl.w[15];
    if (t == kInvalid) break;
    nd = kKeysPerSlab;
  }
}

// First extra head slab of a multi-bucket vertex (word 14 of its primary slab).
__device__ inline uint32_t extra_base(const DView& F, uint32_t u) {
  return (uint32_t)ld_word(slab_ptr(F, u) + 14);
}

constexpr uint32_t kGiantLanes = kGiantSplit * kGroup;  // lanes sharing one giant vertex

// Frontier expansion.  Every path gives each lane whole slabs (one bucket chain at a
// time), so the pushes of a wave cover up to 64 x 15 arcs per counter atomic:
//   single-bucket vertices: one lane each;
//   2 .. kHeavyBuckets buckets: one 16-lane group per vertex, a lane per bucket;
//   heavy: one block per vertex, a lane per bucket;
//   giant: kGiantLanes lanes per vertex, striding over its buckets.
template <bool kUnit>
__global__ void __launch_bounds__(kBlock) k_expand(DView F, uint64_t* D, Queues q, Route r, uint32_t* mark,
                                                   uint32_t stamp) {
  const uint32_t nl = q.cnt[q.icur], nh = q.cnt[3 + q.icur], ngi = q.cnt[6 + q.icur];
  if (blockIdx.x == 0 && threadIdx.x < 3) q.cnt[3 * threadIdx.x + q.iclear] = 0;
  if (nl == 0 && nh == 0 && ngi == 0) return;  // the same for the whole grid
  __shared__ Stage S[4];
  open_routed(S, q.next, r);
  const uint32_t T = band_limit(r);
  const uint32_t gtid = blockIdx.x * kBlock + threadIdx.x, nthreads = gridDim.x * kBlock;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  if constexpr (kUnit) {  // one loop per path
    for (uint32_t i = gtid; i < nl; i += nthreads) {
      const uint32_t u = q.cur[0][i];
      if (F.nbk[u] != 1) continue;
      relax_bucket_lane<kUnit>(F, D, u, ld_u64(D + u) >> 32, 0, 1, 0, S, r, T, mark, stamp);
    }
    for (uint32_t i = gtid / kGroup; i < nl; i += ng) {
      const uint32_t u = q.cur[0][i];
      const uint32_t nb = F.nbk[u];
      if (nb == 1 || (uint32_t)glane() >= nb) continue;
      relax_bucket_lane<kUnit>(F, D, u, ld_u64(D + u) >> 32, glane(), nb, extra_base(F, u), S, r, T, mark,
                               stamp);
    }
    for (uint32_t j = blockIdx.x; j < nh; j += gridDim.x) {
      const uint32_t u = q.cur[1][j];
      const uint32_t nb = F.nbk[u];
      const uint64_t du = ld_u64(D + u) >> 32;
      const uint32_t xb = extra_base(F, u);
      for (uint32_t b = threadIdx.x; b < nb; b += kBlock)
        relax_bucket_lane<kUnit>(F, D, u, du, b, nb, xb, S, r, T, mark, stamp);
    }
    for (uint32_t it = gtid; it < ngi * kGiantLanes; it += nthreads) {
      const uint32_t u = q.cur[2][it / kGiantLanes];
      const uint32_t nb = F.nbk[u];
      const uint64_t du = ld_u64(D + u) >> 32;
      const uint32_t xb = extra_base(F, u);
      for (uint32_t b = it % kGiantLanes; b < nb; b += kGiantLanes)
        relax_bucket_lane<kUnit>(F, D, u, du, b, nb, xb, S, r, T, mark, stamp);
    }
    stage_close(S);
    return;
  }
  // Weighted: each thread walks its (vertex, bucket) work items of the four paths in turn
  // through a single relaxation call site.  Four inlined copies of the weighted relaxation
  // need 150 VGPRs (three waves per SIMD), one needs 92 (five).  Lanes in different paths
  // still relax together.
  int path = 0;       // 0 single-bucket, 1 group, 2 heavy, 3 giant, 4 done
  uint32_t i = gtid;  // item index within the path
  uint32_t b = 0;     // next bucket of the current heavy / giant vertex
  while (path < 4) {
    uint32_t u = 0, nb = 1, bk = 0;
    bool have = false;
    if (path == 0) {  // one lane per single-bucket vertex
      if (i < nl) {
        u = q.cur[0][i];
        i += nthreads;
        nb = F.nbk[u];
        have = nb == 1;
      } else {
        path = 1;
        i = gtid / kGroup;
      }
    } else if (path == 1) {  // 2 .. kHeavyBuckets buckets: a 16-lane group, a lane per bucket
      if (i < nl) {
        u = q.cur[0][i];
        i += ng;
        nb = F.nbk[u];
        bk = (uint32_t)glane();
        have = nb > 1 && bk < nb;
      } else {
        path = 2;
        i = blockIdx.x;
        b = threadIdx.x;
      }
    } else if (path == 2) {  // heavy: a block per vertex, a lane per bucket
      if (i < nh) {
        u = q.cur[1][i];
        nb = F.nbk[u];
        if (b < nb) {
          bk = b;
          b += kBlock;
          have = true;
        } else {
          i += gridDim.x;
          b = threadIdx.x;
        }
      } else {
        path = 3;
        i = gtid;
        b = gtid % kGiantLanes;
      }
    } else {  // giant: kGiantLanes lanes per vertex
      if (i < ngi * kGiantLanes) {
        u = q.cur[2][i / kGiantLanes];
        nb = F.nbk[u];
        if (b < nb) {
          bk = b;
          b += kGiantLanes;
          have = true;
        } else {
          i += nthreads;
          b = i % kGiantLanes;
        }
      } else {
        path = 4;
      }
    }
    if (!have) continue;
    const uint64_t du = ld_u64(D + u) >> 32;
    relax_bucket_lane<kUnit>(F, D, u, du, bk, nb, nb > 1 ? extra_base(F, u) : 0u, S, r, T, mark, stamp);
  }
  stage_close(S);
}

// Band step, part 1: reset the pile minimum and the size of the pile about to be filled.
__global__ void k_band_reset(uint32_t* fmin, uint32_t* next_cnt) {
  if (threadIdx.x == 0) {
    *fmin = 0xFFFFFFFFu;
    *next_cnt = 0;
  }
}

// Band step, part 2: the smallest distance on the far pile at or above the old threshold
// (an entry below it was expanded, at its current distance, in an earlier band).
__global__ void k_band_min(const uint64_t* D, const uint32_t* far, const uint32_t* far_cnt, const uint32_t* T,
                           uint32_t* fmin) {
  const uint32_t n = *far_cnt, told = *T;
  uint32_t m = 0xFFFFFFFFu;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t d = (uint32_t)(ld_u64(D + far[i]) >> 32);
    if (d >= told && d < m) m = d;
  }
  for (int o = 32; o > 0; o >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, o));
  if (lane64() == 0 && m != 0xFFFFFFFFu) atomicMin(fmin, m);
}

// Band step, part 3: the new threshold is fmin + delta; pile entries in [old T, new T) form
// the frontier of the next band, later ones move to the other pile under the new band id.
__global__ void k_band_split(const uint32_t* nbk, const uint64_t* D, const uint32_t* far, const uint32_t* far_cnt,
                             const uint32_t* T, const uint32_t* fmin, uint32_t delta, uint32_t* T_next,
                             PushQ Q, uint32_t* far_next, uint32_t* next_cnt, uint32_t* far_mark,
                             uint32_t band_next) {
  const uint32_t n = *far_cnt, told = *T, fm = *fmin;
  const uint32_t tnew = fm == 0xFFFFFFFFu ? told : (fm >= 0xFFFFFFFFu - delta ? 0xFFFFFFFFu : fm + delta);
  if (blockIdx.x == 0 && threadIdx.x == 0) *T_next = tnew;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x + threadIdx.x - lane; base < n; base += stride) {
    const uint32_t i = base + lane;
    bool near = false, keep = false;
    uint32_t v = 0, nb = 0;
    if (i < n) {
      v = far[i];
      const uint32_t d = (uint32_t)(ld_u64(D + v) >> 32);
      near = d >= told && d < tnew;
      keep = d >= tnew;
    }
    if (keep) far_mark[v] = band_next;
    wave_push(far_next, next_cnt, keep, v);
    if (near) nb = nbk[v];
    wave_push(Q.q[0], Q.c[0], near && nb <= kHeavyBuckets, v);
    wave_push(Q.q[1], Q.c[1], near && nb > kHeavyBuckets && nb <= kGiantBuckets, v);
    wave_push(Q.q[2], Q.c[2], near && nb > kGiantBuckets, v);
  }
}

__global__ void k_trav_init(uint64_t* D, uint32_t nv, uint32_t src) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x)
    D[v] = v == src ? (uint64_t)src : kTreeNone;
}

// Reset the rotating counters so that slot 0 is the current frontier, empty both far
// piles and set the first threshold to 0 (every prologue push of a weighted traversal
// waits on the pile until the first band step).
__global__ void k_queue_reset(uint32_t* cnt, uint32_t* inval_cnt) {
  if (threadIdx.x < 13) cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0 && inval_cnt) *inval_cnt = 0;
}

__global__ void k_seed_source(DView F, uint32_t src, PushQ Q, Route r, uint32_t* mark, uint32_t stamp) {
  if (threadIdx.x != 0) return;
  if (r.T) {  // weighted: the source waits on the far pile for the first band step
    r.far_mark[src] = r.band;
    r.far[0] = src;
    *r.far_cnt = 1;
    return;
  }
  mark[src] = stamp;
  const uint32_t nb = F.nbk[src];
  const int k = nb <= kHeavyBuckets ? 0 : (nb <= kGiantBuckets ? 1 : 2);
  Q.q[k][0] = src;
  *Q.c[k] = 1;
}

// Insert prologue: relax each effective inserted arc.
template <bool kUnit>
__global__ void k_relax_batch(DView F, uint64_t* D, Log lg, uint64_t n, PushQ Q, Route r, uint32_t* mark,
                              uint32_t stamp) {
  __shared__ Stage S[4];
  open_routed(S, Q, r);
  const uint32_t T = band_limit(r);
  // whole waves step together so that the wave-wide push sees every lane
  const uint64_t lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; base < n;
       base += stride) {
    const uint64_t i = base + lane;
    bool improve = false;
    uint32_t v = 0;
    uint64_t cand = kTreeNone;
    if (i < n && lg.st[i] == 1) {
      const uint32_t u = lg.s[i];
      v = lg.d[i];
      const uint64_t du = ld_u64(D + u);
      if (du != kTreeNone) {
        cand = tree_node((du >> 32) + (kUnit ? 1u : lg.w[i]), u);
        if (cand < D[v]) improve = amin64(D + v, cand) > cand;
      }
    }
    push_staged(S, F.nbk, r, T, mark, stamp, improve, v, (uint32_t)(cand >> 32));
  }
  stage_close(S);
}

// A vertex cut from the tree (by exactly one successful CAS, so it needs no frontier
// mark) is staged to [3] the invalidated list and [0..2] the light, heavy or giant queue.
__device__ inline void stage_cut(Stage (&S)[4], const uint32_t* nbk, bool hit, uint32_t y) {
  const uint32_t nb = hit ? nbk[y] : 0u;
  stage_push(S[3], hit, y);
  stage_push(S[0], hit && nb <= kHeavyBuckets, y);
  stage_push(S[1], hit && nb > kHeavyBuckets && nb <= kGiantBuckets, y);
  stage_push(S[2], hit && nb > kGiantBuckets, y);
}

// Delete prologue, step 1: a deleted arc (u, v) of the dependence tree invalidates v.
__global__ void k_invalidate(DView F, uint64_t* D, Log lg, uint64_t n, PushQ Q, uint32_t* inval,
                             uint32_t* inval_cnt) {
  // a vertex is cut by exactly one successful CAS, so it needs no frontier mark
  __shared__ Stage S[4];
  for (int k = 0; k < 3; ++k) stage_open(S[k], Q.q[k], Q.c[k]);
  stage_open(S[3], inval, inval_cnt);
  __syncthreads();
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
      const uint64_t dv = ld_u64(D + v);
      if (dv != kTreeNone && (uint32_t)dv == u) hit = cas64(D + v, dv, kTreeNone) == dv;
    }
    stage_cut(S, F.nbk, hit, v);
  }
  stage_close(S);
}

// Delete prologue, step 2: invalidate the subtree below each invalidated vertex x (its
// tree children are the out-neighbours y whose parent is x).
__device__ inline void inval_word(const DView& F, uint64_t* D, uint32_t x_parent, uint64_t w,
                                  bool data, Stage (&S)[4]) {
  const uint32_t y = (uint32_t)w;
  bool hit = false;
  if (data && valid_key(y)) {
    const uint64_t dy = ld_u64(D + y);
    if (dy != kTreeNone && (uint32_t)dy == x_parent) hit = cas64(D + y, dy, kTreeNone) == dy;
  }
  stage_cut(S, F.nbk, hit, y);
}

__global__ void __launch_bounds__(kBlock) k_propagate(DView F, uint64_t* D, Queues q, uint32_t* inval,
                                                      uint32_t* inval_cnt) {
  const uint32_t nl = q.cnt[q.icur], nh = q.cnt[3 + q.icur], ngi = q.cnt[6 + q.icur];
  if (blockIdx.x == 0 && threadIdx.x < 3) q.cnt[3 * threadIdx.x + q.iclear] = 0;
  if (nl == 0 && nh == 0 && ngi == 0) return;  // the same for the whole grid
  __shared__ Stage S[4];
  for (int k = 0; k < 3; ++k) stage_open(S[k], q.next.q[k], q.next.c[k]);
  stage_open(S[3], inval, inval_cnt);
  __syncthreads();
  // single-bucket vertices: one lane each; the child tests of a slab are issued together
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += gridDim.x * blockDim.x) {
    const uint32_t x = q.cur[0][i];
    if (F.nbk[x] != 1) continue;
    Slab sl;
    uint32_t t = x;
    while (true) {
      load_slab(F, t, sl);
      uint64_t dy[kKeysPerSlab];
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j) {
        const uint32_t y = (uint32_t)sl.w[j];
        dy[j] = valid_key(y) ? ld_u64(D + y) : kTreeNone;
      }
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j) {
        const uint32_t y = (uint32_t)sl.w[j];
        const bool child = dy[j] != kTreeNone && (uint32_t)dy[j] == x;
        dy[j] = child ? cas64(D + y, dy[j], kTreeNone) ^ dy[j] : 1ull;  // 0: this lane cut y
      }
      uint32_t cut = 0;
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j)
        if (dy[j] == 0) cut |= 1u << j;
      uint32_t heavy = 0, giant = 0;
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j) {
        const uint32_t nb = (cut >> j & 1) ? F.nbk[(uint32_t)sl.w[j]] : 1u;
        if (nb > kGiantBuckets) giant |= 1u << j;
        else if (nb > kHeavyBuckets) heavy |= 1u << j;
      }
      stage_words(S[3], cut, sl);
      stage_words(S[0], cut & ~(heavy | giant), sl);
      stage_words(S[1], heavy, sl);
      stage_words(S[2], giant, sl);
      t = (uint32_t)sl.w[15];
      if (t == kInvalid) break;
    }
  }
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  for (uint32_t i = g0; i < nl; i += ng) {
    const uint32_t x = q.cur[0][i];
    if (F.nbk[x] == 1) continue;
    for_each_slab(F, x, [&](uint64_t w, bool data) { inval_word(F, D, x, w, data, S); });
  }
  const uint32_t gib = threadIdx.x / kGroup;
  for (uint32_t j = blockIdx.x; j < nh; j += gridDim.x) {
    const uint32_t x = q.cur[1][j];
    for_each_slab_strided(F, x, gib, kGroupsPerBlock, [&](uint64_t w, bool data) {
      inval_word(F, D, x, w, data, S);
    });
  }
  for (uint32_t it = g0; it < ngi * kGiantSplit; it += ng) {
    const uint32_t x = q.cur[2][it / kGiantSplit];
    for_each_slab_strided(F, x, it % kGiantSplit, kGiantSplit, [&](uint64_t w, bool data) {
      inval_word(F, D, x, w, data, S);
    });
  }
  stage_close(S);
}

// Delete prologue, step 3: each invalidated vertex takes the best candidate offered by
// its still-valid in-neighbours (reverse view) and, if reached, joins the frontier.
// Single-bucket vertices are pulled by one lane, up to kHeavyBuckets buckets by a 16-lane
// group, larger ones by a whole block (each group offers its own best; the atomic
// minimum keeps the smallest).
template <bool kUnit>
__device__ inline uint64_t pull_word(const uint64_t* D, uint64_t x, bool data) {
  const uint32_t u = (uint32_t)x;
  if (!data || !valid_key(u)) return kTreeNone;
  const uint64_t du = ld_u64(D + u);
  if (du == kTreeNone) return kTreeNone;
  return tree_node((du >> 32) + (kUnit ? 1ull : (x >> 32)), u);
}

template <bool kUnit>
__global__ void __launch_bounds__(kBlock) k_dec_pull(DView F, DView R, uint64_t* D,
                                                     const uint32_t* inval, const uint32_t* inval_cnt,
                                                     PushQ Q, Route r, uint32_t* mark, uint32_t stamp) {
  __shared__ Stage S[4];
  open_routed(S, Q, r);
  const uint32_t n = *inval_cnt;
  const uint32_t T = band_limit(r);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t y = inval[i];
    if (R.nbk[y] != 1) continue;
    uint64_t best = kTreeNone;
    Slab sl;
    uint32_t t = y;
    while (true) {
      load_slab(R, t, sl);
      uint64_t c[kKeysPerSlab];
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j) c[j] = pull_word<kUnit>(D, sl.w[j], true);
#pragma unroll
      for (int j = 0; j < kKeysPerSlab; ++j) best = c[j] < best ? c[j] : best;
      t = (uint32_t)sl.w[15];
      if (t == kInvalid) break;
    }
    bool improve = false;
    if (best != kTreeNone) improve = amin64(D + y, best) > best;
    push_staged(S, F.nbk, r, T, mark, stamp, improve, y, (uint32_t)(best >> 32));
  }
  const uint32_t g0 = (blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint32_t ng = gridDim.x * kGroupsPerBlock;
  for (uint32_t i = g0; i < n; i += ng) {
    const uint32_t y = inval[i];
    const uint32_t nb = R.nbk[y];
    if (nb == 1 || nb > kHeavyBuckets) continue;
    uint64_t best = kTreeNone;
    for_each_slab(R, y, [&](uint64_t x, bool data) {
      const uint64_t c = pull_word<kUnit>(D, x, data);
      best = c < best ? c : best;
    });
    best = gmin_u64(best);
    bool improve = false;
    if (glane() == 0 && best != kTreeNone) improve = amin64(D + y, best) > best;
    push_staged(S, F.nbk, r, T, mark, stamp, improve, y, (uint32_t)(best >> 32));
  }
  const uint32_t gib = threadIdx.x / kGroup;
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const uint32_t y = inval[i];
    if (R.nbk[y] <= kHeavyBuckets) continue;
    uint64_t best = kTreeNone;
    for_each_slab_strided(R, y, gib, kGroupsPerBlock, [&](uint64_t x, bool data) {
      const uint64_t c = pull_word<kUnit>(D, x, data);
      best = c < best ? c : best;
    });
    best = gmin_u64(best);
    bool improve = false;
    if (glane() == 0 && best != kTreeNone) improve = amin64(D + y, best) > best;
    push_staged(S, F.nbk, r, T, mark, stamp, improve, y, (uint32_t)(best >> 32));
  }
  stage_close(S);
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
  uint32_t* far[2];     // far piles of the weighted epilogue
  uint32_t* far_mark;
  uint32_t* cnt;        // [0..8] rotating frontier sizes, [9..10] pile sizes,
                        // [11..12] band thresholds, [13] smallest pile distance
  uint32_t* inval_cnt;  // invalidated-list size
  uint32_t* stamp;      // host-side stamp counter (also numbers the bands)
  uint64_t* h_pin;      // pinned host words for size read-backs
  uint32_t delta;       // band width
};

TravCtx graph_ctx(mk_graph* g, uint64_t* D) {
  TravCtx c;
  c.D = D;
  for (int i = 0; i < 6; ++i) c.fq[i] = g->fq[i];
  c.mark = g->mark;
  c.inval = g->inval;
  c.far[0] = g->far[0];
  c.far[1] = g->far[1];
  c.far_mark = g->far_mark;
  c.cnt = g->ctr->frontier;
  c.inval_cnt = &g->ctr->inval;
  c.stamp = &g->stamp;
  c.h_pin = g->h_pin;
  c.delta = g->sssp_delta;
  return c;
}

// Host-side band state of one weighted traversal: which pile and threshold word are current.
struct Bands {
  int fb = 0, tb = 0;
  uint32_t band = 0;
};

Route route_of(const TravCtx& c, const Bands& b) {
  return Route{c.cnt + 11 + b.tb, c.far[b.fb], c.cnt + 9 + b.fb, c.far_mark, b.band};
}

// Band 0 of a weighted traversal (kUnit == false): threshold 0, so every prologue push
// lands on pile 0.  Unweighted traversals route nothing.
template <bool kUnit>
Route first_route(const TravCtx& c, Bands& b) {
  if (kUnit) return Route{nullptr, nullptr, nullptr, nullptr, 0};
  b = Bands{};
  b.band = ++*c.stamp;
  return route_of(c, b);
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

// Run frontier iterations (expand or propagate) from iteration *it until the frontier is
// empty.  Iteration `it` reads slot it%3; the frontier of iteration 0 sits in fq[0] /
// fq[2] / fq[4] and slot 0.  On return *it is the first iteration with an empty frontier
// and c.h_pin holds the counters read back last.
template <class Launch>
mk_status run_frontier(mk_graph* g, const TravCtx& c, hipStream_t stream, Launch&& launch,
                       uint64_t* it_io = nullptr) {
  uint64_t it = it_io ? *it_io : 0;
  int every = kSyncFirst;
  for (;; every = every < kSyncMax ? 2 * every : kSyncMax) {
    for (int k = 0; k < every; ++k, ++it) {
      launch(queues(c, it), ++*c.stamp);
      MK_LAUNCH(g, "frontier kernel");
    }
    const int slot = (int)(it % 3);
    MK_HIP(g, hipMemcpyAsync(c.h_pin, c.cnt, 14 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    MK_HIP(g, hipStreamSynchronize(stream));
    const uint32_t* h = reinterpret_cast<const uint32_t*>(c.h_pin);
    if (h[slot] == 0 && h[3 + slot] == 0 && h[6 + slot] == 0) break;
  }
  if (it_io) *it_io = it;
  return MK_OK;
}

constexpr uint32_t kBandBlocks = 1024;

// Frontier epilogue.  Unweighted: expand until the frontier is empty.  Weighted: band by
// band; each band step moves the next band of the far pile into the (empty) frontier of
// the current iteration, then the band is expanded until its frontier is empty.
template <bool kUnit>
mk_status run_expand(mk_graph* g, const TravCtx& c, hipStream_t stream, Bands& b) {
  const DView F = g->view[VF].d;
  if (kUnit) {
    const Route r{nullptr, nullptr, nullptr, nullptr, 0};
    return run_frontier(g, c, stream, [&](Queues q, uint32_t stamp) {
      hipLaunchKernelGGL(k_expand<kUnit>, dim3(kExpandBlocks), dim3(kBlock), 0, stream, F, c.D, q, r,
                         c.mark, stamp);
    });
  }
  uint32_t* fmin = c.cnt + 13;
  uint64_t it = 0;
  while (true) {
    const int nf = b.fb ^ 1, nt = b.tb ^ 1;
    const uint32_t band_next = ++*c.stamp;
    hipLaunchKernelGGL(k_band_reset, dim3(1), dim3(64), 0, stream, fmin, c.cnt + 9 + nf);
    hipLaunchKernelGGL(k_band_min, dim3(kBandBlocks), dim3(kBlock), 0, stream, c.D, c.far[b.fb],
                       c.cnt + 9 + b.fb, c.cnt + 11 + b.tb, fmin);
    PushQ cur;
    for (int k = 0; k < 3; ++k) {
      cur.q[k] = c.fq[2 * k + (int)(it & 1)];
      cur.c[k] = c.cnt + 3 * k + (int)(it % 3);
    }
    hipLaunchKernelGGL(k_band_split, dim3(kBandBlocks), dim3(kBlock), 0, stream, F.nbk, c.D, c.far[b.fb],
                       c.cnt + 9 + b.fb, c.cnt + 11 + b.tb, fmin, c.delta, c.cnt + 11 + nt, cur, c.far[nf],
                       c.cnt + 9 + nf, c.far_mark, band_next);
    MK_LAUNCH(g, "band step");
    b.fb = nf;
    b.tb = nt;
    b.band = band_next;
    const Route r = route_of(c, b);
    mk_status s = run_frontier(g, c, stream, [&](Queues q, uint32_t stamp) {
      hipLaunchKernelGGL(k_expand<kUnit>, dim3(kExpandBlocks), dim3(kBlock), 0, stream, F, c.D, q, r,
                         c.mark, stamp);
    }, &it);
    if (s != MK_OK) return s;
    const uint32_t* h = reinterpret_cast<const uint32_t*>(c.h_pin);
    if (h[9 + b.fb] == 0) break;  // the frontier and the pile are both empty
  }
  return MK_OK;
}

template <bool kUnit>
mk_status static_from(mk_graph* g, const TravCtx& c, uint32_t source, hipStream_t stream) {
  const DView F = g->view[VF].d;
  const uint32_t stamp0 = ++*c.stamp;
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, stream, c.cnt, c.inval_cnt);
  hipLaunchKernelGGL(k_trav_init, dim3(blocks_for(g->n)), dim3(kBlock), 0, stream, c.D, g->n, source);
  Bands b;
  const Route r0 = first_route<kUnit>(c, b);
  hipLaunchKernelGGL(k_seed_source, dim3(1), dim3(64), 0, stream, F, source, first_push(c), r0, c.mark,
                     stamp0);
  MK_LAUNCH(g, "traversal init");
  return run_expand<kUnit>(g, c, stream, b);
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
  bool full = mode == MK_RECOMPUTE || !st.valid || st.source != source || p.lost ||
              p.kinds == 3 || (p.kinds == 2 && !can_dec);
  if (!full && mode == MK_AUTO) {  // the cost model, when one is set, may prefer a recompute
    mk_status s = auto_prefers_recompute(g, kUnit ? MK_ALGO_BFS : MK_ALGO_SSSP, p, stream, &full);
    if (s != MK_OK) return s;
  }
  if (full) {
    // A graph with the reverse view and a mean out-degree of at least 8: distances first
    // (direction-optimizing BFS levels, or the distance-only SSSP), then every vertex's
    // parent from its in-arcs.  On sparser graphs (a road network) the tree traversal in
    // one pass beats distances plus parents.
    const bool by_dist = can_dec && g->m0 >= 8ull * N;
    mk_status s = !by_dist ? static_from<kUnit>(g, c, source, stream)
                  : kUnit  ? bfs_tree_by_levels(g, source, d_out, D, stream)
                           : sssp_tree_by_distances(g, source, d_out, D, stream);
    if (s != MK_OK) return s;
  } else if (!p.list.empty()) {
    const uint32_t stamp0 = ++g->stamp;
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, stream, c.cnt, c.inval_cnt);
    Bands bands;
    if (p.kinds == 1) {
      const Route r0 = first_route<kUnit>(c, bands);
      for (const BatchRec* b : p.list) {
        Log lg = g->log;
        lg.s += b->off; lg.d += b->off; lg.w += b->off; lg.st += b->off; lg.uf += b->off;
        hipLaunchKernelGGL(k_relax_batch<kUnit>, dim3(blocks_for(b->n)), dim3(kBlock), 0, stream, F, D,
                           lg, b->n, first_push(c), r0, c.mark, stamp0);
      }
    } else {  // deletions only
      for (const BatchRec* b : p.list) {
        Log lg = g->log;
        lg.s += b->off; lg.d += b->off; lg.w += b->off; lg.st += b->off; lg.uf += b->off;
        hipLaunchKernelGGL(k_invalidate, dim3(blocks_for(b->n)), dim3(kBlock), 0, stream, F, D, lg, b->n,
                           first_push(c), c.inval, c.inval_cnt);
      }
      MK_LAUNCH(g, "k_invalidate");
      mk_status s = run_frontier(g, c, stream, [&](Queues q, uint32_t stamp) {
        hipLaunchKernelGGL(k_propagate, dim3(kExpandBlocks), dim3(kBlock), 0, stream, F, D, q, c.inval,
                           c.inval_cnt);
      });
      if (s != MK_OK) return s;
      hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, stream, c.cnt, nullptr);
      const uint32_t stamp1 = ++g->stamp;
      const Route r0 = first_route<kUnit>(c, bands);
      hipLaunchKernelGGL(k_dec_pull<kUnit>, dim3(kExpandBlocks), dim3(kBlock), 0, stream, F,
                         g->view[VR].d, D, c.inval, c.inval_cnt, first_push(c), r0, c.mark, stamp1);
    }
    MK_LAUNCH(g, "traversal prologue");
    mk_status s = run_expand<kUnit>(g, c, stream, bands);
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
  // D (8 B); six queues, stamps, the invalidated list, two far piles and the band marks
  // (4 B each); counters; 256-byte alignment of each of the 13 regions
  return (size_t)n * (8 + 11 * 4) + 128 + 14 * 256;
}

}  // namespace

extern "C" {

mk_status mk_incr_bfs(mk_graph* g, uint32_t source, uint32_t* d_level, uint32_t* d_parent,
                      mk_mode mode, hipStream_t stream) {
  if (!g) return MK_ERR_INVALID_ARG;
  if (mk_status gs = graph_guard(g); gs != MK_OK) return gs;
  return traverse<true>(g, g->bfs, g->bfs_D, source, d_level, d_parent, mode, stream);
}

mk_status mk_incr_sssp(mk_graph* g, uint32_t source, uint32_t* d_dist, uint32_t* d_parent,
                       mk_mode mode, hipStream_t stream) {
  if (!g) return MK_ERR_INVALID_ARG;
  if (mk_status gs = graph_guard(g); gs != MK_OK) return gs;
  return traverse<false>(g, g->sssp, g->sssp_D, source, d_dist, d_parent, mode, stream);
}

size_t mk_traversal_workspace_bytes(const mk_graph* g) { return g ? ws_bytes_for(g->n) : 0; }

mk_status mk_traverse_from(mk_graph* g, uint32_t source, int weighted, void* d_ws, size_t ws_bytes,
                           uint32_t slot, uint32_t* d_dist, uint32_t* d_parent, hipStream_t stream) {
  if (!g || !d_ws || !d_dist || source >= g->n || slot >= kSlots) return MK_ERR_INVALID_ARG;
  if (ws_bytes < ws_bytes_for(g->n)) return MK_ERR_CAPACITY;
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
  TravCtx c;
  c.D = reinterpret_cast<uint64_t*>(take((size_t)N * 8));
  for (int i = 0; i < 6; ++i) c.fq[i] = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  c.mark = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  c.inval = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  c.far[0] = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  c.far[1] = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  c.far_mark = reinterpret_cast<uint32_t*>(take((size_t)N * 4));
  c.cnt = reinterpret_cast<uint32_t*>(take(128));
  c.inval_cnt = c.cnt + 16;
  uint32_t stamp = 0;
  c.stamp = &stamp;
  c.h_pin = g->slot_pin[slot];
  c.delta = g->sssp_delta;
  hipLaunchKernelGGL(k_fill_mark, dim3(blocks_for(N)), dim3(kBlock), 0, stream, c.mark, N);
  hipLaunchKernelGGL(k_fill_mark, dim3(blocks_for(N)), dim3(kBlock), 0, stream, c.far_mark, N);
  mk_status s = weighted ? static_from<false>(g, c, source, stream) : static_from<true>(g, c, source, stream);
  if (s != MK_OK) return s;
  hipLaunchKernelGGL(k_split, dim3(blocks_for(N)), dim3(kBlock), 0, stream, c.D, N, d_dist, d_parent);
  MK_LAUNCH(g, "k_split");
  return MK_OK;
}

}  // extern "C"
