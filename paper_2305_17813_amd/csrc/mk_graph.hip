// Graph construction, batched updates and queries, export, statistics and self-check.
//
// Section 3.1 (memory management): every vertex gets bucket_count[v] head slabs from its
// initial degree and the load factor; an exclusive scan of the bucket counts gives each
// vertex's first head slab inside one contiguous head-slab region.  Chained slabs come
// from a per-view pool behind a device bump counter (the SlabAlloc role of figure 1).
// The graph-operation discussion of the experimental section fixes the semantics of
// insert (store only if absent, at the end of the hashed chain, linking a new slab when
// the chain is full), delete (flip the found lane to TOMBSTONE, stop when found) and
// search (probe the hashed chain only).
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <cstring>

#include "mk_internal.h"

using namespace mk;

namespace mk {

mk_status hip_fail(mk_graph* g, hipError_t e, const char* what) {
  if (g) g->last_err = std::string(what) + ": " + hipGetErrorString(e);
  return MK_ERR_HIP;
}

Pending pending_for(const mk_graph* g, const AlgoState& st) {
  Pending p;
  if (st.seen_seq < g->dropped_seq) p.lost = true;
  for (const auto& b : g->batches)
    if (b.seq > st.seen_seq) {
      p.list.push_back(&b);
      p.kinds |= (b.kind == kInsertBatch) ? 1 : 2;
    }
  return p;
}

void mark_seen(mk_graph* g, AlgoState& st) { st.seen_seq = g->next_seq - 1; }

}  // namespace mk

namespace {
void poll_snapshots(mk_graph* g);
}

namespace mk {
mk_status graph_guard(mk_graph* g, bool poll) {
  if (poll && !g->overflowed.load(std::memory_order_relaxed)) poll_snapshots(g);
  return g->overflowed.load(std::memory_order_relaxed) ? MK_ERR_OUT_OF_SLABS : MK_OK;
}
}  // namespace mk

// ============================================================ device: updates
namespace {

// Insert <key, w> into u's table (one lane).  Returns 1 inserted, 0 already present,
// kPoolEmpty when no slab could be taken (the host-side pool check makes this unreachable;
// the caller raises the view's overflow bit).  Progress never depends on a load being
// fresh: every failed CAS returns the word's true value and `floor` (words of this slab
// known to be filled) only grows, so a slab is retried at most 15 times.
constexpr int kPoolEmpty = 3;

__device__ int insert_key_core(const DView& V, uint32_t u, uint32_t key, uint32_t w, uint32_t& spare) {
  Slab sl;
  int nd;
  uint32_t s = lane_head(V, u, key, sl, nd);
  const uint64_t mine = ((uint64_t)w << 32) | key;
  int floor = 0;
  while (true) {
    uint64_t* sp = slab_ptr(V, s);
    int hit, empty;
    uint64_t hitw;
    scan_slab(sl, nd, key, floor, hit, hitw, empty);
    if (hit >= 0) return 0;
    if (empty >= 0) {
      // the lowest EMPTY word of the chain: claim it, or learn who did
      const uint64_t old = cas64(sp + empty, kEmptyWord, mine);
      if (old == kEmptyWord) return 1;
      if ((uint32_t)old == key) return 0;
      floor = empty + 1;  // another key took the word: look at the rest of this slab again
      load_slab(V, s, sl);
      continue;
    }
    const uint64_t link = sl.w[15];
    if ((uint32_t)link != kInvalid) {
      s = (uint32_t)link;
      floor = 0;
      nd = kKeysPerSlab;
      load_slab(V, s, sl);
      continue;
    }
    // Full tail: put the key in word 0 of a fresh slab, then link the slab.  Pool slabs
    // were filled with EMPTY words and an INVALID link at creation, so word 0 is the only
    // word to write; writing it with a CAS from EMPTY (performed where the other CASes
    // are) and waiting for its result orders it before the link without an L2 write-back.
    // A spare kept from a lost link race already holds this key in word 0.
    if (spare == kInvalid) {
      // the bump pointer first (one counter atomic for the lanes of the wave that need a
      // slab now), reclaimed slabs once it is exhausted; both hand out EMPTY slabs
      uint64_t m = __ballot(true);
      int leader = __builtin_ctzll(m);
      uint32_t base = 0;
      if (lane64() == leader) base = atomicAdd(V.pool_ctr, (uint32_t)__popcll(m));
      const uint32_t got = __shfl(base, leader) + lanes_below(m);
      if (got < V.pool_cap) {
        spare = V.pool_base + got;
      } else {
        m = __ballot(true);
        leader = __builtin_ctzll(m);
        if (lane64() == leader) base = atomicAdd(V.pool_ctr + 2, (uint32_t)__popcll(m));
        const uint32_t idx = __shfl(base, leader) + lanes_below(m);
        if ((int32_t)(V.pool_ctr[1] - idx) <= 0) return kPoolEmpty;
        spare = V.free_ids[idx % V.pool_cap];
      }
    }
    const uint64_t prev = cas64(slab_ptr(V, spare), kEmptyWord, mine);
    if (prev != kEmptyWord && prev != mine) {
      // not a fresh slab (the free list handed out a slab in use): leave it alone and
      // report the pool as broken rather than list it as a spare
      spare = kInvalid;
      return kPoolEmpty;
    }
    // the link word keeps its meta half (the bucket count of a primary slab)
    const uint64_t old = cas64(sp + 15, link, (link & 0xFFFFFFFF00000000ull) | spare);
    if (old == link) {
      spare = kInvalid;  // linked: now part of the chain
      return 1;
    }
    s = (uint32_t)old;  // lost the race: continue in the winner's slab, keep the spare
    floor = 0;
    nd = kKeysPerSlab;
    load_slab(V, s, sl);
  }
}

// insert_key_core, then a slab that was taken but never linked (its lane lost every link
// race and placed the key elsewhere) is cleared and listed for return to the free list
// once the kernel has finished.
__device__ int insert_key(const DView& V, uint32_t u, uint32_t key, uint32_t w) {
  uint32_t spare = kInvalid;
  const int r = insert_key_core(V, u, key, w, spare);
  if (spare != kInvalid) {
    slab_ptr(V, spare)[0] = kEmptyWord;
    V.spare_ids[atomicAdd(V.pool_ctr + 3, 1u)] = spare;
  }
  return r;
}

// After the insert kernels: their unused spares join the free list (one block per view;
// the take counter, which inserts may have run past the end of the list, is clamped first).
__global__ void k_spare_merge(DView F, DView R, DView U, uint32_t views) {
  if (!(views & (1u << blockIdx.x))) return;
  const DView& V = blockIdx.x == 0 ? F : (blockIdx.x == 1 ? R : U);
  uint32_t* c = V.pool_ctr;
  const uint32_t n = c[3];
  if (n == 0) return;
  const uint32_t end = c[1];
  const uint32_t take = (int32_t)(end - c[2]) < 0 ? end : c[2];
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) V.free_ids[(end + i) % V.pool_cap] = V.spare_ids[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    c[2] = take;
    c[1] = end + n;
    c[3] = 0;
  }
}

// Pool counters of every view and the overflow bits, gathered for one asynchronous copy.
__global__ void k_pool_snapshot(const uint32_t* f, const uint32_t* r, const uint32_t* u,
                                const uint32_t* overflow, uint32_t* out) {
  const uint32_t t = threadIdx.x;
  if (t < 12) {
    const uint32_t* c = t < 4 ? f : (t < 8 ? r : u);
    out[t] = (c && (t & 3) < 3) ? c[t & 3] : 0u;
  } else if (t == 12) {
    out[t] = *overflow;
  } else if (t < 16) {
    out[t] = 0u;
  }
}

// Delete key from u's table (one lane).  Returns 1 deleted, 0 absent; *w_out gets the weight.
__device__ int delete_key(const DView& V, uint32_t u, uint32_t key, uint32_t* w_out) {
  Slab sl;
  int nd;
  uint32_t s = lane_head(V, u, key, sl, nd);
  while (true) {
    int hit, empty;
    uint64_t hitw;
    scan_slab(sl, nd, key, 0, hit, hitw, empty);
    if (hit >= 0) {
      *w_out = (uint32_t)(hitw >> 32);
      return cas64(slab_ptr(V, s) + hit, hitw, kTombWord) == hitw ? 1 : 0;
    }
    if (empty >= 0) return 0;
    s = (uint32_t)sl.w[15];
    if (s == kInvalid) return 0;
    load_slab(V, s, sl);
    nd = kKeysPerSlab;
  }
}

__device__ inline bool bad_arc(uint32_t s, uint32_t d, uint32_t nv) {
  return s >= nv || d >= nv || s == d;  // nv <= 2^30, so reserved ids are >= nv
}

// Forward view of an insert batch, one lane per arc.  Writes the status and the log.
__global__ void __launch_bounds__(kBlock) k_insert_fwd(DView F, const uint32_t* __restrict__ src,
                                                       const uint32_t* __restrict__ dst,
                                                       const uint32_t* __restrict__ w, uint64_t n,
                                                       uint32_t nv, uint8_t* status, Log log,
                                                       uint32_t* overflow) {
  const uint64_t op = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (op >= n) return;
  const uint32_t s = src[op], d = dst[op];
  const uint32_t wt = w ? w[op] : 1u;
  int st = 2;
  if (!bad_arc(s, d, nv)) st = insert_key(F, s, d, wt);
  if (st == 1) atomicAdd(F.deg + s, 1u);
  if (st == kPoolEmpty) {  // not stored: reported as not applied, the graph is flagged
    atomicOr(overflow, 1u);
    st = 2;
  }
  if (status) status[op] = (uint8_t)st;
  log.s[op] = s;
  log.d[op] = d;
  log.w[op] = wt;
  log.st[op] = (uint8_t)st;
  log.uf[op] = 0;
}

// Every view of an insert batch in one launch, four lanes per arc: the forward view (status
// and change log), the reverse view, and both directions of the undirected view.  The other
// views take the arc straight from the batch rather than waiting for the forward view's
// status: the views hold one arc set, so an arc the forward view already has is in the
// others too and its insert there is a no-op.  Copies of one arc inside a batch must carry
// one weight, since each view keeps the copy that wins its own CAS.  The canonical
// undirected direction (small id -> large id) decides which op reports the undirected edge
// as new.
__global__ void __launch_bounds__(kBlock) k_insert_all(DView F, DView R, DView U, uint32_t views,
                                                       const uint32_t* __restrict__ src,
                                                       const uint32_t* __restrict__ dst,
                                                       const uint32_t* __restrict__ w, uint64_t n,
                                                       uint32_t nv, uint8_t* status, Log log,
                                                       uint32_t* overflow) {
  const uint64_t gid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t op = gid >> 2;
  const int task = (int)(gid & 3);
  if (op >= n) return;
  if (task == 1 && !(views & MK_VIEW_REV)) return;
  if (task >= 2 && !(views & MK_VIEW_UND)) return;
  const uint32_t s = src[op], d = dst[op];
  const uint32_t wt = w ? w[op] : 1u;
  const bool bad = bad_arc(s, d, nv);
  if (task == 0) {
    int st = 2;
    if (!bad) st = insert_key(F, s, d, wt);
    if (st == 1) atomicAdd(F.deg + s, 1u);
    if (st == kPoolEmpty) {
      atomicOr(overflow, 1u);
      st = 2;
    }
    if (status) status[op] = (uint8_t)st;
    log.s[op] = s;
    log.d[op] = d;
    log.w[op] = wt;
    log.st[op] = (uint8_t)st;
    if (!(views & MK_VIEW_UND)) log.uf[op] = 0;
    return;
  }
  if (bad) {
    if (task == 2) log.uf[op] = 0;
    return;
  }
  int r;
  if (task == 1) {
    r = insert_key(R, d, s, wt);
    if (r == 1) atomicAdd(R.deg + d, 1u);
  } else {
    const uint32_t a = task == 2 ? min(s, d) : max(s, d);
    const uint32_t b = task == 2 ? max(s, d) : min(s, d);
    r = insert_key(U, a, b, 1u);
    if (r == 1) atomicAdd(U.deg + a, 1u);
    if (task == 2) log.uf[op] = r == 1;
  }
  if (r == kPoolEmpty) atomicOr(overflow, task == 1 ? 2u : 4u);
}

__global__ void __launch_bounds__(kBlock) k_delete_fwd(DView F, const uint32_t* __restrict__ src,
                                                       const uint32_t* __restrict__ dst, uint64_t n,
                                                       uint32_t nv, uint8_t* status, Log log) {
  const uint64_t op = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (op >= n) return;
  const uint32_t s = src[op], d = dst[op];
  int st = 2;
  uint32_t wt = 0;
  if (!bad_arc(s, d, nv)) st = delete_key(F, s, d, &wt);
  if (st == 1) atomicSub(F.deg + s, 1u);
  if (status) status[op] = (uint8_t)st;
  log.s[op] = s;
  log.d[op] = d;
  log.w[op] = wt;
  log.st[op] = (uint8_t)st;
  log.uf[op] = 0;
}

// The other views of a delete batch, three lanes per deleted arc: the reverse view, and
// the two directions of the undirected view, where {u,v} goes only if the reverse arc is
// absent once the whole batch has been applied to the forward view.  The three lanes of
// an arc sit in one wave (21 arcs per wave, lane 63 idle), so the forward-view probe for
// the reverse arc is made once and handed to the second undirected lane by a shuffle.
constexpr uint32_t kOpsPerWave = 21;
__global__ void __launch_bounds__(kBlock) k_delete_aux(DView F, DView R, DView U, uint32_t views,
                                                       Log log, uint64_t n) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int task = (int)(lane % 3);
  const uint64_t op = wave * kOpsPerWave + lane / 3;
  bool live = lane < 3 * kOpsPerWave && op < n;
  if (live) live = log.st[op] == 1;
  if (task == 0 && !(views & MK_VIEW_REV)) live = false;
  if (task != 0 && !(views & MK_VIEW_UND)) live = false;
  uint32_t s = 0, d = 0, w;
  if (live) {
    s = log.s[op];
    d = log.d[op];
  }
  if (live && task == 0 && delete_key(R, d, s, &w) == 1) atomicSub(R.deg + d, 1u);
  bool absent = false;
  if (live && task == 1) absent = lane_probe(F, d, s) == kEmptyWord;
  // every lane is active here: lane 3k+2 takes the answer of lane 3k+1
  const int from = (int)(lane - task) + 1;
  absent = __shfl((int)absent, from < 64 ? from : (int)lane) != 0;
  if (!live || task == 0 || !absent) return;
  const uint32_t a = task == 1 ? min(s, d) : max(s, d);
  const uint32_t b = task == 1 ? max(s, d) : min(s, d);
  const int r = delete_key(U, a, b, &w);
  if (r == 1) atomicSub(U.deg + a, 1u);
  if (task == 1) log.uf[op] = r == 1;
}

__global__ void __launch_bounds__(kBlock) k_query(DView F, const uint32_t* __restrict__ src,
                                                  const uint32_t* __restrict__ dst, uint64_t n,
                                                  uint32_t nv, uint8_t* __restrict__ found,
                                                  uint32_t* __restrict__ wout) {
  const uint64_t op = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (op >= n) return;
  const uint32_t s = src[op], d = dst[op];
  uint64_t x = kEmptyWord;
  if (!bad_arc(s, d, nv)) x = lane_probe(F, s, d);
  const bool f = x != kEmptyWord;
  found[op] = f;
  if (wout) wout[op] = f ? (uint32_t)(x >> 32) : 0u;
}

// ============================================================ device: build
__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_slabs(uint64_t* words, uint64_t n_words) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words;
       i += (uint64_t)gridDim.x * blockDim.x)
    words[i] = (i & 15) == 15 ? kNextNone : kEmptyWord;
}

__global__ void k_count_deg(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                            uint64_t m, uint32_t nv, uint32_t* cf, uint32_t* cr, uint32_t* cu) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t s = src[i], d = dst[i];
    if (bad_arc(s, d, nv)) continue;
    atomicAdd(cf + s, 1u);
    if (cr) atomicAdd(cr + d, 1u);
    if (cu) {
      atomicAdd(cu + s, 1u);
      atomicAdd(cu + d, 1u);
    }
  }
}

// bucket_count[v] = max(1, ceil(deg0(v) / (load_factor * 15))), 1 when hashing is off;
// extra[v] = bucket_count[v] - 1 head slabs beyond the primary one.
__global__ void k_plan(const uint32_t* cnt, uint32_t nv, float keys_per_bucket, uint32_t* nb,
                       uint32_t* extra) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    uint32_t b = 1;
    if (keys_per_bucket > 0.f) b = max(1u, (uint32_t)ceilf((float)cnt[v] / keys_per_bucket));
    nb[v] = b;
    extra[v] = b - 1;
  }
}

// Primary slab v: word 15 = <INVALID next, nb>; with several buckets, word 14 holds the
// index of the extra head slabs.
__global__ void k_init_primary(uint64_t* slab, const uint32_t* nb, const uint32_t* xrel, uint32_t nv) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    uint64_t* p = slab + (uint64_t)v * kGroup;
    p[15] = primary_link(nb[v], kInvalid);
    if (nb[v] > 1) p[14] = 0xFFFFFFFF00000000ull | (uint64_t)(nv + xrel[v]);
  }
}

__global__ void k_extra_total(const uint32_t* nb, const uint32_t* xrel, uint32_t nv,
                              unsigned long long* total) {
  if (threadIdx.x == 0) *total = (unsigned long long)xrel[nv - 1] + nb[nv - 1] - 1;
}

// IterationScheme2 pairs: bucket k = off[v] + i of vertex v becomes <v, i>.
__global__ void k_pairs_build(const uint32_t* nbk, const uint32_t* off, uint32_t nv, uint32_t* pv, uint32_t* pi) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    const uint32_t o = off[v], nb = nbk[v];
    for (uint32_t i = 0; i < nb; ++i) {
      pv[o + i] = v;
      pi[o + i] = i;
    }
  }
}

// ============================================================ device: export / stats / check
__global__ void __launch_bounds__(kBlock) k_export(DView F, uint32_t nv, uint32_t* os, uint32_t* od,
                                                   uint32_t* ow, unsigned long long cap,
                                                   unsigned long long* count) {
  const uint64_t g0 = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint64_t ng = (uint64_t)gridDim.x * kGroupsPerBlock;
  for (uint64_t v = g0; v < nv; v += ng) {
    for_each_slab(F, (uint32_t)v, [&](uint64_t x, bool data) {
      const uint32_t k = (uint32_t)x;
      const bool p = data && valid_key(k);
      const uint64_t m = __ballot(p);
      if (m == 0) return;
      const int leader = __builtin_ctzll(m);
      unsigned long long base = 0;
      if (lane64() == leader) base = atomicAdd(count, (unsigned long long)__popcll(m));
      base = __shfl(base, leader);
      const unsigned long long at = base + lanes_below(m);
      if (p && at < cap) {
        os[at] = (uint32_t)v;
        od[at] = k;
        if (ow) ow[at] = (uint32_t)(x >> 32);
      }
    });
  }
}

__global__ void k_sum_u32(const uint32_t* a, uint32_t n, unsigned long long* out) {
  unsigned long long acc = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    acc += a[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane64() == 0 && acc) atomicAdd(out, acc);
}

// Audit one chain (bucket b of vertex v, head slab s with nd data words).  Returns the
// violations seen by this lane and adds the live keys to *live.
__device__ uint32_t check_chain(const DView& V, uint32_t v, uint32_t nb, uint32_t b, uint32_t s, int nd,
                                uint32_t slab_end, uint32_t* live) {
  const int gl = glane();
  uint32_t errs = 0, hops = 0;
  bool seen_empty = false;
  const uint32_t head = s;
  const int head_nd = nd;
  while (s != kInvalid) {
    if (++hops > (1u << 22)) return errs + 1;  // a cycle
    const uint64_t x = slab_ptr(V, s)[gl];
    const uint32_t k = (uint32_t)x;
    const bool data = gl < nd;
    const bool isv = data && valid_key(k);
    // prefix rule: no filled lane after an EMPTY lane in chain order
    const uint32_t em = gballot(data && k == kEmptyKey);
    const uint32_t filled = gballot(data && k != kEmptyKey);
    if (gl == 0 && seen_empty && filled) errs++;
    if (em) {
      if (gl == 0 && (filled >> __builtin_ctz(em))) errs++;
      seen_empty = true;
    }
    if (data && !isv && x != kEmptyWord && x != kTombWord) errs++;
    if (isv && (nb > 1 ? bucket_of(k, nb, V.hash_a, V.hash_b) : 0u) != b) errs++;
    if (isv) {  // duplicates: count this lane's key over the whole chain
      uint32_t occ = 0, t = head, h2 = 0;
      int tnd = head_nd;
      while (t != kInvalid && ++h2 < (1u << 22)) {
        const uint64_t* tp = slab_ptr(V, t);
        for (int j = 0; j < tnd; ++j) occ += (uint32_t)tp[j] == k;
        t = (uint32_t)tp[15];
        if (t != kInvalid && (t < V.pool_base || t >= slab_end)) break;
        tnd = kKeysPerSlab;
      }
      if (occ != 1) errs++;
    }
    *live += __popc(gballot(isv));
    const uint32_t nx = gbcast(k, 15);
    if (nx != kInvalid && (nx < V.pool_base || nx >= slab_end)) return errs + (gl == 0);
    if (em && nx != kInvalid && gl == 0) errs++;  // an EMPTY lane is only in the tail
    s = nx;
    nd = kKeysPerSlab;
  }
  return errs;
}

// One group per vertex: audit every chain of the vertex's table.
__global__ void __launch_bounds__(kBlock) k_check(DView V, uint32_t nv, uint32_t n_head,
                                                  uint32_t pool_used, unsigned long long* bad) {
  const uint64_t g0 = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint64_t ng = (uint64_t)gridDim.x * kGroupsPerBlock;
  const int gl = glane();
  const uint32_t slab_end = V.pool_base + pool_used;
  for (uint64_t vv = g0; vv < nv; vv += ng) {
    const uint32_t v = (uint32_t)vv;
    const uint64_t* pp = slab_ptr(V, v);
    const uint32_t nb = (uint32_t)(pp[15] >> 32);
    uint32_t errs = 0, live = 0;
    if (nb != V.nbk[v] || nb == 0) {
      errs = 1;
    } else {
      uint32_t xb = 0;
      if (nb > 1) {
        xb = (uint32_t)pp[14];
        if ((pp[14] >> 32) != 0xFFFFFFFFu || xb < nv || xb + nb - 1 > n_head) errs = 1;
      }
      if (!errs) {
        errs += check_chain(V, v, nb, 0, v, nb > 1 ? kKeysPerSlab - 1 : kKeysPerSlab, slab_end, &live);
        for (uint32_t b = 1; b < nb; ++b)
          errs += check_chain(V, v, nb, b, xb + b - 1, kKeysPerSlab, slab_end, &live);
      }
    }
    for (int o = 8; o > 0; o >>= 1) errs += __shfl_xor(errs, o, kGroup);
    if (gl == 0) {
      if (live != V.deg[v]) errs++;
      if (errs) atomicAdd(bad, (unsigned long long)errs);
    }
  }
}

// Byte model: slabs one probe walks (op 0: until found / first EMPTY / end; op 1: to the
// end of the chain unless the key is found first).  A second head access counts as a slab.
// ------------------------------------------------------------ slab reclamation
// Take back free-list entries that inserts asked for but did not get (the take counter
// may run past the append counter).
__global__ void k_free_fix(uint32_t* ctr) {
  if (threadIdx.x == 0 && (int32_t)(ctr[1] - ctr[2]) < 0) ctr[2] = ctr[1];
}

// Rewrite every chain holding at least min_tomb tombstones with its live words packed from
// its head slab in chain order, EMPTY after them, and the chain cut after the last slab it
// still needs; the slabs after the cut are refilled with EMPTY words and appended to the
// free list.  One 16-lane group per chain (head slab h: primary slabs [0, N), extra head
// slabs after them).  Packing only moves a word to an earlier position of its own chain,
// so the write position never passes the slab being read.
__global__ void __launch_bounds__(kBlock) k_compact(DView V, uint64_t n_head, uint32_t nv, uint32_t min_tomb,
                                                    unsigned long long* freed, uint64_t* marks) {
  const uint64_t g0 = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kGroup;
  const uint64_t ng = (uint64_t)gridDim.x * kGroupsPerBlock;
  const int gl = glane();
  const uint32_t below = (1u << gl) - 1u;
  unsigned long long total = 0;
  for (uint64_t h = g0; h < n_head; h += ng) {
    const uint32_t head = (uint32_t)h;
    const uint64_t x = ld_word(slab_ptr(V, head) + gl);
    const int nd0 = (head < nv && (uint32_t)(gbcast64(x, 15) >> 32) > 1) ? kKeysPerSlab - 1 : kKeysPerSlab;
    uint32_t tomb = 0;
    {
      uint64_t y = x;
      int nd = nd0;
      while (true) {
        tomb += __popc(gballot(gl < nd && y == kTombWord));
        const uint32_t nx = gbcast((uint32_t)y, 15);
        if (nx == kInvalid) break;
        y = ld_word(slab_ptr(V, nx) + gl);
        nd = kKeysPerSlab;
      }
    }
    if (tomb < min_tomb || tomb == 0) continue;
    // words move: the chain's update mark (if the view keeps marks) restarts at the head
    if (marks && gl == 0) marks[h] = 0;
    uint32_t ws = head;  // slab being written, its capacity and fill
    int wcap = nd0, wpos = 0;
    uint64_t y = x;
    int rnd = nd0;
    while (true) {
      const uint32_t next = gbcast((uint32_t)y, 15);
      const bool live = gl < rnd && valid_key((uint32_t)y);
      const uint32_t m = gballot(live);
      const int r = __popc(m & below), cnt = __popc(m);
      const int n1 = min(cnt, wcap - wpos);
      if (live && r < n1) slab_ptr(V, ws)[wpos + r] = y;
      wpos += n1;
      if (cnt > n1) {  // spill into the next slab of the chain (not past the one being read)
        ws = (uint32_t)ld_word(slab_ptr(V, ws) + 15);
        wcap = kKeysPerSlab;
        if (live && r >= n1) slab_ptr(V, ws)[r - n1] = y;
        wpos = cnt - n1;
      }
      if (next == kInvalid) break;
      y = ld_word(slab_ptr(V, next) + gl);
      rnd = kKeysPerSlab;
    }
    // end the chain at ws and hand the rest to the free list (each lane rewrites only the
    // word it read itself; the link comes from lane 15)
    const uint64_t xw = ld_word(slab_ptr(V, ws) + gl);
    const uint64_t wl = gbcast64(xw, 15);
    const uint32_t rest = (uint32_t)wl;
    if (gl >= wpos && gl < wcap) slab_ptr(V, ws)[gl] = kEmptyWord;
    if (gl == 15) slab_ptr(V, ws)[15] = (wl & 0xFFFFFFFF00000000ull) | kInvalid;
    uint32_t k = 0;
    for (uint32_t t = rest; t != kInvalid; t = (uint32_t)ld_word(slab_ptr(V, t) + 15)) ++k;
    if (k == 0) continue;
    uint32_t pos = 0;
    if (gl == 0) pos = atomicAdd(V.pool_ctr + 1, k);
    pos = gbcast(pos, 0);
    for (uint32_t t = rest; t != kInvalid;) {
      const uint64_t xt = ld_word(slab_ptr(V, t) + gl);
      const uint32_t nx = (uint32_t)gbcast64(xt, 15);
      slab_ptr(V, t)[gl] = gl == 15 ? kNextNone : kEmptyWord;
      if (gl == 0) V.free_ids[pos % V.pool_cap] = t;
      ++pos;
      t = nx;
    }
    total += k;
  }
  if (gl == 0 && total) atomicAdd(freed, total);
}

__device__ inline uint32_t walk_cost(const DView& V, uint32_t u, uint32_t key, int op) {
  Slab sl;
  int nd;
  uint32_t extra;
  lane_head(V, u, key, sl, nd, &extra);
  uint32_t slabs = 1 + extra;
  while (true) {
    int hit, empty;
    uint64_t hitw;
    scan_slab(sl, nd, key, 0, hit, hitw, empty);
    if (hit >= 0 || empty >= 0) return slabs;
    const uint32_t s = (uint32_t)sl.w[15];
    if (s == kInvalid) return slabs;
    load_slab(V, s, sl);
    nd = kKeysPerSlab;
    ++slabs;
  }
}

__global__ void __launch_bounds__(kBlock) k_probe_cost(DView V, int op, int view,
                                                       const uint32_t* __restrict__ src,
                                                       const uint32_t* __restrict__ dst, uint64_t n,
                                                       uint32_t nv, unsigned long long* acc) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  uint32_t c = 0;
  if (i < n) {
    const uint32_t s = src[i], d = dst[i];
    if (!bad_arc(s, d, nv)) {
      if (view == 0) c = walk_cost(V, s, d, op);
      else if (view == 1) c = walk_cost(V, d, s, op);
      else c = walk_cost(V, s, d, op) + walk_cost(V, d, s, op);
    }
  }
  unsigned long long t = c;
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
  if (lane64() == 0 && t) atomicAdd(acc, t);
}

inline uint32_t grid_stride_blocks(uint64_t n, uint32_t cap = 8192) {
  uint64_t b = (n + kBlock - 1) / kBlock;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b, cap));
}

// ============================================================ host: arena layout
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

bool config_ok(const mk_config* c) {
  return c && c->n_vertices >= 1 && c->n_vertices <= (1u << 30) && c->load_factor >= 0.f &&
         c->load_factor <= 64.f && c->reserved == 0;
}

uint64_t view_arcs(int v, uint64_t m) { return v == VU ? 2 * m : m; }

uint64_t head_bound(const mk_config* c, uint64_t arcs) {
  if (c->load_factor <= 0.f) return c->n_vertices;
  const double per = (double)c->load_factor * kKeysPerSlab;
  return (uint64_t)c->n_vertices + (uint64_t)std::ceil((double)arcs / per) + 1;
}

uint64_t pool_default(const mk_config* c, uint64_t arcs) {
  if (c->pool_slabs) return c->pool_slabs;
  uint64_t headroom = std::max<uint64_t>(65536, std::min<uint64_t>(1ull << 22, arcs / 2));
  return (arcs + kKeysPerSlab - 1) / kKeysPerSlab + headroom;
}

uint64_t log_default(const mk_config* c, uint64_t m) {
  if (c->log_capacity) return c->log_capacity;
  return std::max<uint64_t>(1ull << 21, m / 8);
}

// Carve (or, with base == nullptr, just measure) every region of the arena.
bool layout(const mk_config* c, uint64_t m, char* base, mk_graph* g, size_t* total) {
  Carver cv{base};
  const uint32_t N = c->n_vertices;
  const uint32_t views = c->views | MK_VIEW_FWD;
  uint64_t hb_fwd = 0, hb_rev = 0, und_words = 0;
  for (int v = 0; v < 3; ++v) {
    const bool on = views & (1u << v);
    if (!on) continue;
    const uint64_t arcs = view_arcs(v, m);
    const uint64_t hb = head_bound(c, arcs), pc = pool_default(c, arcs);
    if (hb + pc >= 0xFFFFFFF0ull) return false;  // slab indices are u32
    if (v == VF) hb_fwd = hb;
    uint64_t* slab = cv.take<uint64_t>((hb + pc) * kGroup);
    uint32_t* nbk = cv.take<uint32_t>(N);
    uint32_t* deg = cv.take<uint32_t>(N);
    uint32_t* pctr = cv.take<uint32_t>(64);
    uint32_t* free_ids = cv.take<uint32_t>(pc);
    uint32_t* spare_ids = cv.take<uint32_t>(pc);
    uint32_t *pair_v = nullptr, *pair_i = nullptr, *pair_off = nullptr;
    if (v != VU) {  // IterationScheme2 work lists: one entry per head slab
      pair_v = cv.take<uint32_t>(hb);
      pair_i = cv.take<uint32_t>(hb);
      pair_off = cv.take<uint32_t>(N);
    }
    if (v == VR) hb_rev = hb;
    if (v == VU) und_words = (hb + pc) * kKeysPerSlab;  // bounds the live keys of the view
    if (g) {
      ViewHost& vh = g->view[v];
      vh.on = true;
      vh.nbk = nbk;
      vh.head_reserved = hb;
      vh.pool_cap = pc;
      vh.d.nbk = nbk;
      vh.d.slab = slab;
      vh.d.deg = deg;
      vh.d.pool_ctr = pctr;
      vh.d.free_ids = free_ids;
      vh.d.spare_ids = spare_ids;
      vh.d.pool_cap = (uint32_t)pc;
      vh.pair_v = pair_v;
      vh.pair_i = pair_i;
      vh.pair_off = pair_off;
    }
  }
  const uint64_t L = log_default(c, m);
  Log lg;
  lg.s = cv.take<uint32_t>(L);
  lg.d = cv.take<uint32_t>(L);
  lg.w = cv.take<uint32_t>(L);
  lg.st = cv.take<uint8_t>(L);
  lg.uf = cv.take<uint8_t>(L);
  Counters* ctr = cv.take<Counters>(1);
  uint32_t* fq[6];
  for (auto& q : fq) q = cv.take<uint32_t>(N);
  uint32_t* mark = cv.take<uint32_t>(N);
  uint32_t* inval = cv.take<uint32_t>(N);
  uint32_t* far0 = cv.take<uint32_t>(N);
  uint32_t* far1 = cv.take<uint32_t>(N);
  uint32_t* far_mark = cv.take<uint32_t>(N);
  uint64_t* bfsD = cv.take<uint64_t>(N);
  uint64_t* ssspD = cv.take<uint64_t>(N);
  uint32_t* par = cv.take<uint32_t>(N);
  float* px = cv.take<float>(N);
  float* py = cv.take<float>(N);
  float* pc = cv.take<float>(N);
  uint32_t* hv = cv.take<uint32_t>(N);
  double* hacc = cv.take<double>(N);
  double* prp = cv.take<double>(kPrParts);
  double* prpair = hb_rev ? cv.take<double>(hb_rev) : nullptr;
  // packed in-arc lists: one u32 per data word of the reverse view's slabs
  const uint64_t rev_words = hb_rev ? (hb_rev + pool_default(c, view_arcs(VR, m))) * kKeysPerSlab : 0;
  uint32_t* prlist = hb_rev ? cv.take<uint32_t>(rev_words) : nullptr;
  uint32_t* proff = hb_rev ? cv.take<uint32_t>((uint64_t)N + 1) : nullptr;
  uint32_t *prperm = nullptr, *prrank = nullptr, *prk0 = nullptr, *prk1 = nullptr, *pridx = nullptr;
  float* prcp = nullptr;
  uint64_t* prcr = nullptr;
  void* prsort = nullptr;
  size_t prsort_bytes = 0;
  if (hb_rev) {
    prperm = cv.take<uint32_t>(N);
    prrank = cv.take<uint32_t>(N);
    prk0 = cv.take<uint32_t>(N);
    prk1 = cv.take<uint32_t>(N);
    pridx = cv.take<uint32_t>(N);
    prcp = cv.take<float>(N);
    prcr = cv.take<uint64_t>(N);
    if (rocprim::radix_sort_pairs(nullptr, prsort_bytes, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                  (uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)N, 0, 6) != hipSuccess)
      return false;
    prsort = cv.take<char>(prsort_bytes + 256);
  }
  uint64_t* umark = cv.take<uint64_t>(hb_fwd);
  uint32_t* wflag = cv.take<uint32_t>(N);
  char* lvc = cv.take<char>(256);
  const uint64_t lv_cap = (uint64_t)N + hb_fwd / kGroup + 64;  // >= levels_multi_cap
  uint32_t* lvm0 = cv.take<uint32_t>(lv_cap);
  uint32_t* lvm1 = cv.take<uint32_t>(lv_cap);
  uint64_t* tk0 = nullptr;
  uint64_t* tk1 = nullptr;
  uint32_t* tclist = nullptr;
  uint64_t* tcoff = nullptr;
  size_t sort_bytes = 0, scan_bytes = 0, scan64_bytes = 0;
  if (views & MK_VIEW_UND) {
    tk0 = cv.take<uint64_t>(2 * L);
    tk1 = cv.take<uint64_t>(2 * L);
    tclist = cv.take<uint32_t>(und_words);
    tcoff = cv.take<uint64_t>(N);
    if (rocprim::exclusive_scan(nullptr, scan64_bytes, (uint32_t*)nullptr, (uint64_t*)nullptr, (uint64_t)0,
                                (size_t)N, rocprim::plus<uint64_t>()) != hipSuccess)
      return false;
    if (rocprim::radix_sort_keys(nullptr, sort_bytes, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                 (size_t)(2 * L), 0, 64) != hipSuccess)
      return false;
  }
  void* sort_tmp = cv.take<char>(sort_bytes + 256);
  // scans over the vertices, and over the sorted batch keys of the triangle update (2 L)
  if (rocprim::exclusive_scan(nullptr, scan_bytes, (uint32_t*)nullptr, (uint32_t*)nullptr, 0u,
                              std::max<size_t>(N, 2 * L), rocprim::plus<uint32_t>()) != hipSuccess)
    return false;
  scan_bytes = std::max(scan_bytes, scan64_bytes);  // and the u64 offsets of the packed lists
  void* scan_tmp = cv.take<char>(scan_bytes + 256);
  if (g) {
    g->log = lg;
    g->log_cap = L;
    g->ctr = ctr;
    for (int i = 0; i < 6; ++i) g->fq[i] = fq[i];
    g->mark = mark;
    g->inval = inval;
    g->far[0] = far0;
    g->far[1] = far1;
    g->far_mark = far_mark;
    g->bfs_D = bfsD;
    g->sssp_D = ssspD;
    g->wcc_parent = par;
    g->pr_x = px;
    g->pr_y = py;
    g->pr_c = pc;
    g->heavy_rev = hv;
    g->pr_hacc = hacc;
    g->pr_part = prp;
    g->pr_pair = prpair;
    g->pr_list = prlist;
    g->pr_off = proff;
    g->pr_perm = prperm;
    g->pr_rank = prrank;
    g->pr_skey[0] = prk0;
    g->pr_skey[1] = prk1;
    g->pr_sidx = pridx;
    g->pr_cp = prcp;
    g->pr_cr = prcr;
    g->pr_sort_tmp = prsort;
    g->pr_sort_bytes = prsort_bytes;
    g->upd_mark = umark;
    g->wcc_flag = wflag;
    g->lv_cnt = lvc;
    g->lv_multi[0] = lvm0;
    g->lv_multi[1] = lvm1;
    g->tc_keys[0] = tk0;
    g->tc_keys[1] = tk1;
    g->tc_list = tclist;
    g->tc_off = tcoff;
    g->sort_tmp = sort_tmp;
    g->sort_tmp_bytes = sort_bytes;
    g->scan_tmp = scan_tmp;
    g->scan_tmp_bytes = scan_bytes;
  }
  *total = cv.off + 256;
  return true;
}

uint64_t hash_const(uint32_t seed, uint64_t salt) {
  uint64_t z = ((uint64_t)seed << 1) + salt;  // SplitMix64 finaliser as a seed mixer
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Default band width of the weighted frontier epilogue: kBandArcs mean weights spread
// over the mean out-degree (so that a band of a sparse, long-range graph holds enough
// vertices to fill the device while few are improved again after their expansion), and
// at least kBandMin mean weights (so that a dense, low-diameter graph needs few bands).
constexpr double kBandArcs = 32.0;
constexpr double kBandMin = 8.0;
uint32_t default_band(uint64_t m, uint32_t n, double mean_w) {
  const double deg = std::max(1.0, (double)m / std::max<uint32_t>(n, 1));
  const double w = std::max(1.0, mean_w);
  const double b = std::ceil(std::max(kBandArcs * w / deg, kBandMin * w));
  return (uint32_t)std::min(b, (double)(1u << 30));
}

// Pool slabs in use from one view's counters: bump high-water mark minus the free-list
// entries not yet taken.
uint64_t used_from(const ViewHost& vh, const uint32_t* c) {
  const int32_t avail = std::max<int32_t>(0, (int32_t)(c[1] - c[2]));
  const uint64_t hw = std::min<uint64_t>(c[0], vh.pool_cap);
  return hw - std::min<uint64_t>((uint64_t)avail, hw);
}

// Exact pool figures and the overflow bits (synchronizes the stream).
mk_status refresh_pool(mk_graph* g, hipStream_t stream) {
  for (int v = 0; v < 3; ++v)
    if (g->view[v].on)
      MK_HIP(g, hipMemcpyAsync(g->h_pin + 2 * v, g->view[v].d.pool_ctr, 3 * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, stream));
  MK_HIP(g, hipMemcpyAsync(g->h_pin + 7, &g->ctr->overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
  MK_HIP(g, hipStreamSynchronize(stream));
  g->overflowed.fetch_or(*reinterpret_cast<const uint32_t*>(g->h_pin + 7));
  for (int v = 0; v < 3; ++v) {
    ViewHost& vh = g->view[v];
    if (!vh.on) continue;
    const uint32_t* c = reinterpret_cast<const uint32_t*>(g->h_pin + 2 * v);
    vh.pool_hw = std::min<uint64_t>(c[0], vh.pool_cap);
    vh.pool_used_est = used_from(vh, c);
  }
  // every snapshot still in flight is older than these figures
  for (auto& sn : g->snap) sn.pending = false;
  return MK_OK;
}

bool stream_capturing(hipStream_t stream) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Use the newest completed snapshot, if any: slabs in use then, plus the bound of every
// insert enqueued after it, bound the slabs in use now.  Never waits.
void poll_snapshots(mk_graph* g) {
  int best = -1;
  for (int i = 0; i < kSnaps; ++i) {
    PoolSnap& sn = g->snap[i];
    if (!sn.pending || hipEventQuery(sn.ev) != hipSuccess) continue;
    if (best < 0 || sn.added_at[VF] > g->snap[best].added_at[VF]) best = i;
  }
  if (best < 0) return;
  const PoolSnap& b = g->snap[best];
  g->overflowed.fetch_or(b.pin[12]);
  for (int v = 0; v < 3; ++v) {
    ViewHost& vh = g->view[v];
    if (!vh.on) continue;
    const uint64_t bound = used_from(vh, b.pin + 4 * v) + (vh.added - b.added_at[v]);
    vh.pool_used_est = std::min(vh.pool_used_est, bound);
  }
  // this one and every older completed snapshot are consumed
  for (auto& sn : g->snap)
    if (sn.pending && sn.added_at[VF] <= b.added_at[VF] && hipEventQuery(sn.ev) == hipSuccess)
      sn.pending = false;
}

// Enqueue a snapshot of the pool counters behind the work already on the stream.
void enqueue_snapshot(mk_graph* g, hipStream_t stream) {
  PoolSnap& sn = g->snap[g->snap_next];
  if (sn.pending && hipEventQuery(sn.ev) != hipSuccess) return;  // ring slot still in flight
  const auto ctr_of = [&](int v) -> const uint32_t* { return g->view[v].on ? g->view[v].d.pool_ctr : nullptr; };
  hipLaunchKernelGGL(k_pool_snapshot, dim3(1), dim3(64), 0, stream, ctr_of(VF), ctr_of(VR), ctr_of(VU),
                     &g->ctr->overflow, g->ctr->snap);
  if (hipMemcpyAsync(sn.pin, g->ctr->snap, 16 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipEventRecord(sn.ev, stream) != hipSuccess) {
    (void)hipGetLastError();
    sn.pending = false;
    return;
  }
  for (int v = 0; v < 3; ++v) sn.added_at[v] = g->view[v].added;
  sn.pending = true;
  g->snap_next = (g->snap_next + 1) % kSnaps;
}

// Slabs one insert call may take per view: one per arc (two for the undirected view).
uint64_t insert_need(int v, uint64_t n) { return v == VU ? 2 * n : n; }

bool pool_fits(const mk_graph* g, uint64_t n) {
  for (int v = 0; v < 3; ++v) {
    const ViewHost& vh = g->view[v];
    if (vh.on && vh.pool_used_est + insert_need(v, n) > vh.pool_cap) return false;
  }
  return true;
}

// Make sure every enabled view's pool can take `n` more inserts.  The host keeps an upper
// bound of the slabs in use; when it runs short, a completed snapshot tightens it, and only
// when that is not enough either is the stream synchronized for the exact figures (never
// under stream capture: the call is then refused).
mk_status ensure_pool(mk_graph* g, uint64_t n, hipStream_t stream) {
  if (pool_fits(g, n)) return MK_OK;
  poll_snapshots(g);
  if (g->overflowed.load()) return MK_ERR_OUT_OF_SLABS;
  if (pool_fits(g, n)) return MK_OK;
  if (stream_capturing(stream)) return MK_ERR_OUT_OF_SLABS;
  mk_status st = refresh_pool(g, stream);
  if (st != MK_OK) return st;
  if (g->overflowed.load()) return MK_ERR_OUT_OF_SLABS;
  return pool_fits(g, n) ? MK_OK : MK_ERR_OUT_OF_SLABS;
}

// Reserve n log entries for a new batch, dropping the oldest batches it overwrites.
uint64_t reserve_log(mk_graph* g, uint64_t n) {
  if (g->log_tail + n > g->log_cap) g->log_tail = 0;
  const uint64_t lo = g->log_tail, hi = lo + n;
  while (!g->batches.empty()) {
    const BatchRec& b = g->batches.front();
    const bool overlap = b.off < hi && lo < b.off + b.n;
    bool later_overlap = false;
    for (const auto& o : g->batches)
      if (o.off < hi && lo < o.off + o.n) later_overlap = true;
    if (!overlap && !later_overlap) break;
    g->dropped_seq = b.seq;
    g->batches.pop_front();
  }
  return lo;
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

DView dv(const mk_graph* g, int v) { return g->view[v].on ? g->view[v].d : g->view[VF].d; }

void launch_insert(mk_graph* g, const uint32_t* s, const uint32_t* d, const uint32_t* w, uint64_t n,
                   uint8_t* status, const Log& lg, hipStream_t stream) {
  if (g->view[VR].on || g->view[VU].on)
    hipLaunchKernelGGL(k_insert_all, dim3(grid_for_lanes(4 * n)), dim3(kBlock), 0, stream, dv(g, VF), dv(g, VR),
                       dv(g, VU), g->cfg.views, s, d, w, n, g->n, status, lg, &g->ctr->overflow);
  else
    hipLaunchKernelGGL(k_insert_fwd, dim3(grid_for_lanes(n)), dim3(kBlock), 0, stream, dv(g, VF), s, d, w,
                       n, g->n, status, lg, &g->ctr->overflow);
  hipLaunchKernelGGL(k_spare_merge, dim3(3), dim3(kBlock), 0, stream, dv(g, VF), dv(g, VR), dv(g, VU),
                     g->cfg.views | MK_VIEW_FWD);
}

}  // namespace

namespace mk {
mk_status ensure_pairs(mk_graph* g, int v, hipStream_t stream) {
  ViewHost& vh = g->view[v];
  if (!vh.on || !vh.pair_v) return MK_ERR_STATE;
  if (vh.pairs_ok) return MK_OK;
  size_t tb = g->scan_tmp_bytes;
  if (rocprim::exclusive_scan(g->scan_tmp, tb, vh.nbk, vh.pair_off, 0u, (size_t)g->n, rocprim::plus<uint32_t>(),
                              stream) != hipSuccess)
    return MK_ERR_HIP;
  hipLaunchKernelGGL(k_pairs_build, dim3(grid_stride_blocks(g->n)), dim3(kBlock), 0, stream, vh.nbk,
                     vh.pair_off, g->n, vh.pair_v, vh.pair_i);
  MK_LAUNCH(g, "k_pairs_build");
  vh.pairs_ok = true;
  return MK_OK;
}

}  // namespace mk

// ============================================================ C-ABI
extern "C" {

size_t mk_arena_bytes(const mk_config* cfg, uint64_t n_edges_hint) {
  if (!config_ok(cfg)) return 0;
  size_t total = 0;
  if (!layout(cfg, n_edges_hint, nullptr, nullptr, &total)) return 0;
  return total;
}

mk_status mk_graph_create(const mk_config* cfg, void* d_arena, size_t arena_bytes,
                          const uint32_t* d_src, const uint32_t* d_dst, const uint32_t* d_w,
                          uint64_t m, hipStream_t stream, mk_graph** out) {
  if (!out || !config_ok(cfg) || !d_arena || ((uintptr_t)d_arena & 255)) return MK_ERR_INVALID_ARG;
  if (m && (!d_src || !d_dst)) return MK_ERR_INVALID_ARG;
  *out = nullptr;
  size_t need = 0;
  if (!layout(cfg, m, nullptr, nullptr, &need)) return MK_ERR_INVALID_ARG;
  if (arena_bytes < need) return MK_ERR_CAPACITY;
  mk_graph* g = new mk_graph();
  g->cfg = *cfg;
  g->cfg.views |= MK_VIEW_FWD;
  g->n = cfg->n_vertices;
  g->m0 = m;
  g->arena = (char*)d_arena;
  g->arena_bytes = arena_bytes;
  layout(&g->cfg, m, g->arena, g, &g->used);
  auto fail = [&](mk_status s) {
    mk_graph_destroy(g);
    return s;
  };
  if (hipHostMalloc((void**)&g->h_pin, 64 * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess)
    return fail(MK_ERR_HIP);
  uint32_t* snap_pin = nullptr;
  if (hipHostMalloc((void**)&snap_pin, kSnaps * 16 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess)
    return fail(MK_ERR_HIP);
  for (int i = 0; i < kSnaps; ++i) {
    g->snap[i].pin = snap_pin + 16 * i;
    if (hipEventCreateWithFlags(&g->snap[i].ev, hipEventDisableTiming) != hipSuccess) return fail(MK_ERR_HIP);
  }
  const uint32_t N = g->n;
  const uint32_t nb_blocks = grid_stride_blocks(N);
  for (int v = 0; v < 3; ++v) {
    ViewHost& vh = g->view[v];
    if (!vh.on) continue;
    vh.d.hash_a = hash_const(cfg->hash_seed, 0x1000 + v) | 1ull;
    vh.d.hash_b = hash_const(cfg->hash_seed, 0x2000 + v);
    hipLaunchKernelGGL(k_fill_u32, dim3(nb_blocks), dim3(kBlock), 0, stream, vh.d.deg, N, 0u);
  }
  (void)hipMemsetAsync(g->ctr, 0, sizeof(Counters), stream);
  if (m)
    hipLaunchKernelGGL(k_count_deg, dim3(grid_stride_blocks(m)), dim3(kBlock), 0, stream, d_src,
                       d_dst, m, N, g->view[VF].d.deg, g->view[VR].on ? g->view[VR].d.deg : nullptr,
                       g->view[VU].on ? g->view[VU].d.deg : nullptr);
  const float kpb = cfg->load_factor > 0.f ? cfg->load_factor * kKeysPerSlab : 0.f;
  for (int v = 0; v < 3; ++v) {
    ViewHost& vh = g->view[v];
    if (!vh.on) continue;
    hipLaunchKernelGGL(k_plan, dim3(nb_blocks), dim3(kBlock), 0, stream, vh.d.deg, N, kpb, vh.nbk,
                       g->fq[0]);
    size_t tb = g->scan_tmp_bytes;
    if (rocprim::exclusive_scan(g->scan_tmp, tb, g->fq[0], g->fq[1 + v], 0u, (size_t)N,
                                rocprim::plus<uint32_t>(), stream) != hipSuccess)
      return fail(MK_ERR_HIP);
  }
  // extra head slabs per view: read back the scan totals to place the pools
  for (int v = 0; v < 3; ++v) {
    ViewHost& vh = g->view[v];
    if (!vh.on) continue;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, (uint32_t*)&g->ctr->u64tmp[v], 2, 0u);
    hipLaunchKernelGGL(k_extra_total, dim3(1), dim3(64), 0, stream, vh.nbk, g->fq[1 + v], N,
                       &g->ctr->u64tmp[v]);
  }
  // the initial weight sum sets the default band width of the weighted epilogue
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, (uint32_t*)&g->ctr->u64tmp[3], 2, 0u);
  if (m && d_w)
    hipLaunchKernelGGL(k_sum_u32, dim3(grid_stride_blocks(m, 1024)), dim3(kBlock), 0, stream, d_w,
                       (uint32_t)std::min<uint64_t>(m, 0xFFFFFFFFu), &g->ctr->u64tmp[3]);
  if (hipMemcpyAsync(g->h_pin, g->ctr->u64tmp, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost,
                     stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail(MK_ERR_HIP);
  g->sssp_delta = cfg->sssp_delta ? cfg->sssp_delta
                                  : default_band(m, N, m ? (d_w ? (double)g->h_pin[3] / m : 1.0) : 1.0);
  for (int v = 0; v < 3; ++v) {
    ViewHost& vh = g->view[v];
    if (!vh.on) continue;
    vh.n_head = (uint64_t)N + g->h_pin[v];
    if (vh.n_head > vh.head_reserved) return fail(MK_ERR_CAPACITY);
    vh.d.pool_base = (uint32_t)vh.n_head;
    hipLaunchKernelGGL(k_fill_slabs, dim3(grid_stride_blocks((vh.n_head + vh.pool_cap) * kGroup)),
                       dim3(kBlock), 0, stream, vh.d.slab, (vh.n_head + vh.pool_cap) * kGroup);
    hipLaunchKernelGGL(k_init_primary, dim3(nb_blocks), dim3(kBlock), 0, stream, vh.d.slab, vh.nbk,
                       g->fq[1 + v], N);
    hipLaunchKernelGGL(k_fill_u32, dim3(nb_blocks), dim3(kBlock), 0, stream, vh.d.deg, N, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, vh.d.pool_ctr, 64, 0u);
  }
  hipLaunchKernelGGL(k_fill_u32, dim3(nb_blocks), dim3(kBlock), 0, stream, g->mark, N, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(nb_blocks), dim3(kBlock), 0, stream, g->far_mark, N, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(nb_blocks), dim3(kBlock), 0, stream, g->wcc_flag, N, 0u);
  // update marks start at the chain heads (encoded 0)
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_stride_blocks(2 * g->view[VF].n_head)), dim3(kBlock), 0,
                     stream, (uint32_t*)g->upd_mark, 2 * g->view[VF].n_head, 0u);
  // bulk insert, in chunks that fit the change log (used here as scratch)
  for (uint64_t off = 0; off < m; off += g->log_cap) {
    const uint64_t k = std::min<uint64_t>(g->log_cap, m - off);
    launch_insert(g, d_src + off, d_dst + off, d_w ? d_w + off : nullptr, k, nullptr, g->log, stream);
  }
  if (hipGetLastError() != hipSuccess) return fail(MK_ERR_HIP);
  if (refresh_pool(g, stream) != MK_OK) return fail(MK_ERR_HIP);
  // the initial arcs did not fit the pool (only an explicit, too small pool_slabs can do this)
  if (g->overflowed.load()) return fail(MK_ERR_OUT_OF_SLABS);
  *out = g;
  return MK_OK;
}

mk_status mk_graph_destroy(mk_graph* g) {
  if (!g) return MK_OK;
  if (g->h_pin) (void)hipHostFree(g->h_pin);
  for (auto* p : g->slot_pin)
    if (p) (void)hipHostFree(p);
  for (auto& sn : g->snap)
    if (sn.ev) (void)hipEventDestroy(sn.ev);
  if (g->snap[0].pin) (void)hipHostFree(g->snap[0].pin);
  delete g;
  return MK_OK;
}

mk_status mk_insert_edges(mk_graph* g, const uint32_t* d_src, const uint32_t* d_dst,
                          const uint32_t* d_w, uint64_t n, uint8_t* d_status, hipStream_t stream) {
  if (!g) return MK_ERR_INVALID_ARG;
  if (n == 0) return MK_OK;
  if (!d_src || !d_dst) return MK_ERR_INVALID_ARG;
  if (n > g->log_cap) return MK_ERR_CAPACITY;
  mk_status st = graph_guard(g, true);
  if (st != MK_OK) return st;
  st = ensure_pool(g, n, stream);
  if (st != MK_OK) return st;
  const uint64_t off = reserve_log(g, n);
  launch_insert(g, d_src, d_dst, d_w, n, d_status, log_at(g, off), stream);
  MK_LAUNCH(g, "k_insert");
  for (int v = 0; v < 3; ++v)
    if (g->view[v].on) {
      g->view[v].pool_used_est += insert_need(v, n);
      g->view[v].added += insert_need(v, n);
    }
  // the bound would not admit two more batches of this size: have exact figures on the way,
  // so that they are usually there before the bound runs out
  if (!pool_fits(g, 2 * n) && !stream_capturing(stream)) enqueue_snapshot(g, stream);
  g->batches.push_back(BatchRec{kInsertBatch, off, n, g->next_seq++});
  g->log_tail = off + n;
  g->batches_applied++;
  return MK_OK;
}

mk_status mk_delete_edges(mk_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                          uint8_t* d_status, hipStream_t stream) {
  if (!g) return MK_ERR_INVALID_ARG;
  if (n == 0) return MK_OK;
  if (!d_src || !d_dst) return MK_ERR_INVALID_ARG;
  if (n > g->log_cap) return MK_ERR_CAPACITY;
  mk_status st = graph_guard(g, true);
  if (st != MK_OK) return st;
  const uint64_t off = reserve_log(g, n);
  const Log lg = log_at(g, off);
  hipLaunchKernelGGL(k_delete_fwd, dim3(grid_for_lanes(n)), dim3(kBlock), 0, stream, dv(g, VF),
                     d_src, d_dst, n, g->n, d_status, lg);
  MK_LAUNCH(g, "k_delete_fwd");
  if (g->view[VR].on || g->view[VU].on) {
    hipLaunchKernelGGL(k_delete_aux, dim3(grid_for_lanes((n + kOpsPerWave - 1) / kOpsPerWave * 64)),
                       dim3(kBlock), 0, stream, dv(g, VF),
                       dv(g, VR), dv(g, VU), g->cfg.views, lg, n);
    MK_LAUNCH(g, "k_delete_aux");
  }
  g->batches.push_back(BatchRec{kDeleteBatch, off, n, g->next_seq++});
  g->log_tail = off + n;
  g->batches_applied++;
  return MK_OK;
}

mk_status mk_query_edges(mk_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                         uint8_t* d_found, uint32_t* d_w, hipStream_t stream) {
  if (!g) return MK_ERR_INVALID_ARG;
  if (n == 0) return MK_OK;
  if (!d_src || !d_dst || !d_found) return MK_ERR_INVALID_ARG;
  mk_status st = graph_guard(g);
  if (st != MK_OK) return st;
  hipLaunchKernelGGL(k_query, dim3(grid_for_lanes(n)), dim3(kBlock), 0, stream, dv(g, VF), d_src,
                     d_dst, n, g->n, d_found, d_w);
  MK_LAUNCH(g, "k_query");
  return MK_OK;
}

mk_status mk_graph_export(mk_graph* g, uint32_t* d_src, uint32_t* d_dst, uint32_t* d_w,
                          uint64_t cap, uint64_t* h_count, hipStream_t stream) {
  if (!g || !h_count || (cap && (!d_src || !d_dst))) return MK_ERR_INVALID_ARG;
  if (mk_status gs = graph_guard(g); gs != MK_OK) return gs;
  unsigned long long* cnt = &g->ctr->u64tmp[3];
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, (uint32_t*)cnt, 2, 0u);
  hipLaunchKernelGGL(k_export, dim3(grid_for_groups(std::min<uint64_t>(g->n, 1u << 20))),
                     dim3(kBlock), 0, stream, dv(g, VF), g->n, d_src, d_dst, d_w,
                     (unsigned long long)cap, cnt);
  MK_LAUNCH(g, "k_export");
  MK_HIP(g, hipMemcpyAsync(g->h_pin, cnt, 8, hipMemcpyDeviceToHost, stream));
  MK_HIP(g, hipStreamSynchronize(stream));
  *h_count = g->h_pin[0];
  return g->h_pin[0] > cap ? MK_ERR_CAPACITY : MK_OK;
}

mk_status mk_graph_stats(mk_graph* g, mk_stats* h_out, hipStream_t stream) {
  if (!g || !h_out) return MK_ERR_INVALID_ARG;
  std::memset(h_out, 0, sizeof(*h_out));
  unsigned long long* acc = &g->ctr->u64tmp[0];
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, (uint32_t*)acc, 4, 0u);
  hipLaunchKernelGGL(k_sum_u32, dim3(grid_stride_blocks(g->n, 1024)), dim3(kBlock), 0, stream,
                     g->view[VF].d.deg, g->n, acc);
  if (g->view[VU].on)
    hipLaunchKernelGGL(k_sum_u32, dim3(grid_stride_blocks(g->n, 1024)), dim3(kBlock), 0, stream,
                       g->view[VU].d.deg, g->n, acc + 1);
  MK_LAUNCH(g, "k_sum_u32");
  MK_HIP(g, hipMemcpyAsync(g->h_pin + 8, acc, 16, hipMemcpyDeviceToHost, stream));
  mk_status st = refresh_pool(g, stream);
  if (st != MK_OK) return st;
  h_out->n_arcs = g->h_pin[8];
  h_out->n_und_edges = g->h_pin[9] / 2;
  for (int v = 0; v < 3; ++v) {
    if (!g->view[v].on) continue;
    h_out->head_slabs[v] = g->view[v].n_head;
    h_out->pool_used[v] = g->view[v].pool_used_est;
    h_out->pool_capacity[v] = g->view[v].pool_cap;
  }
  h_out->arena_bytes_used = g->used;
  h_out->batches_applied = g->batches_applied;
  return g->overflowed.load() ? MK_ERR_OUT_OF_SLABS : MK_OK;
}

mk_status mk_graph_check(mk_graph* g, uint64_t* h_bad, hipStream_t stream) {
  if (!g || !h_bad) return MK_ERR_INVALID_ARG;
  mk_status st = refresh_pool(g, stream);
  if (st != MK_OK) return st;
  unsigned long long* bad = &g->ctr->u64tmp[2];
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, (uint32_t*)bad, 2, 0u);
  for (int v = 0; v < 3; ++v) {
    if (!g->view[v].on) continue;
    hipLaunchKernelGGL(k_check, dim3(grid_for_groups(std::min<uint64_t>(g->n, 1u << 20))),
                       dim3(kBlock), 0, stream, g->view[v].d, g->n, (uint32_t)g->view[v].n_head,
                       (uint32_t)g->view[v].pool_hw, bad);
    MK_LAUNCH(g, "k_check");
  }
  MK_HIP(g, hipMemcpyAsync(g->h_pin, bad, 8, hipMemcpyDeviceToHost, stream));
  MK_HIP(g, hipStreamSynchronize(stream));
  *h_bad = g->h_pin[0];
  return g->overflowed.load() ? MK_ERR_OUT_OF_SLABS : MK_OK;
}

mk_status mk_compact(mk_graph* g, uint32_t min_tombstones, uint64_t* h_freed, hipStream_t stream) {
  if (!g || !h_freed) return MK_ERR_INVALID_ARG;
  if (mk_status gs = graph_guard(g); gs != MK_OK) return gs;
  unsigned long long* freed = &g->ctr->u64tmp[2];
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, (uint32_t*)freed, 2, 0u);
  for (int v = 0; v < 3; ++v) {
    const ViewHost& vh = g->view[v];
    if (!vh.on) continue;
    hipLaunchKernelGGL(k_free_fix, dim3(1), dim3(64), 0, stream, vh.d.pool_ctr);
    hipLaunchKernelGGL(k_compact, dim3(grid_for_groups(std::min<uint64_t>(vh.n_head, 1u << 20))),
                       dim3(kBlock), 0, stream, vh.d, vh.n_head, g->n, min_tombstones, freed,
                       v == VF ? g->upd_mark : nullptr);
    MK_LAUNCH(g, "k_compact");
  }
  MK_HIP(g, hipMemcpyAsync(g->h_pin + 10, freed, 8, hipMemcpyDeviceToHost, stream));
  mk_status st = refresh_pool(g, stream);
  if (st != MK_OK) return st;
  *h_freed = g->h_pin[10];
  return MK_OK;
}

mk_status mk_probe_cost(mk_graph* g, int op, int view, const uint32_t* d_src, const uint32_t* d_dst,
                        uint64_t n, uint64_t* h_slabs, hipStream_t stream) {
  if (!g || !h_slabs || view < 0 || view > 2 || op < 0 || op > 1) return MK_ERR_INVALID_ARG;
  if (!g->view[view].on) return MK_ERR_STATE;
  if (mk_status gs = graph_guard(g); gs != MK_OK) return gs;
  *h_slabs = 0;
  if (n == 0) return MK_OK;
  if (!d_src || !d_dst) return MK_ERR_INVALID_ARG;
  unsigned long long* acc = &g->ctr->u64tmp[1];
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, (uint32_t*)acc, 2, 0u);
  hipLaunchKernelGGL(k_probe_cost, dim3(grid_for_lanes(n)), dim3(kBlock), 0, stream, g->view[view].d,
                     op, view, d_src, d_dst, n, g->n, acc);
  MK_LAUNCH(g, "k_probe_cost");
  MK_HIP(g, hipMemcpyAsync(g->h_pin, acc, 8, hipMemcpyDeviceToHost, stream));
  MK_HIP(g, hipStreamSynchronize(stream));
  *h_slabs = g->h_pin[0];
  return MK_OK;
}

mk_status mk_set_iteration_scheme(mk_graph* g, mk_iter_scheme scheme) {
  if (!g || (scheme != MK_ITER_SCHEME1 && scheme != MK_ITER_SCHEME2 && scheme != MK_ITER_PACKED))
    return MK_ERR_INVALID_ARG;
  g->iter_scheme = scheme;
  return MK_OK;
}

const char* mk_status_string(mk_status s) {
  switch (s) {
    case MK_OK: return "ok";
    case MK_ERR_INVALID_ARG: return "invalid argument";
    case MK_ERR_OUT_OF_SLABS: return "slab pool exhausted (nothing applied)";
    case MK_ERR_CAPACITY: return "capacity exceeded";
    case MK_ERR_STATE: return "the graph lacks a view this operation needs";
    case MK_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

}  // extern "C"
