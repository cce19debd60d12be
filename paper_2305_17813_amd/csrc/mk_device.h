// Device-side building blocks of the slab-hash graph for gfx950 (CDNA4, wave64).
//
// Slab geometry (the paper's section 2 slab, redesigned for wave64): one slab is
// 128 bytes = one L2 line = 16 words of 8 bytes.  A *group* of 16 lanes (one DPP row)
// reads a slab with one coalesced dwordx2 per lane, so a wave64 runs four independent
// probes at once.  Data words hold the pair <key, weight> (key in the low half); word 15
// holds <next slab index, meta>.  Keys are unordered within a slab.
//
// Head slabs (section 3.1, redesigned so that a probe needs no directory lookup): slab v
// is the *primary* slab of vertex v and starts bucket 0.  Its word 15 carries the bucket
// count nb in the meta half.  When nb > 1, word 14 of the primary slab holds the index
// of the vertex's extra head slabs (buckets 1 .. nb-1, contiguous), so bucket 0 keeps 14
// data words and every other slab 15.  A vertex with one bucket is therefore probed with
// a single 128-byte access; any other with at most two.
//
// Sentinels (section 2 footnotes): EMPTY key 0xFFFFFFFE (the whole EMPTY word is
// 0xFFFFFFFF_FFFFFFFE, i.e. UINT64_MAX-1), TOMBSTONE word <0xFFFFFFFD, 0xFFFFFFFD>,
// INVALID slab/vertex 0xFFFFFFFF.
//
// Chain invariant that makes lock-free inserts unique: a key is only ever written into
// the lowest EMPTY word of its chain (by CAS), a word only moves EMPTY -> key ->
// TOMBSTONE, and tombstones are never reused.  The filled words of a chain therefore
// always form a prefix, so a probe may stop at the first EMPTY word.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mk {

constexpr uint32_t kEmptyKey = 0xFFFFFFFEu;
constexpr uint32_t kTombKey = 0xFFFFFFFDu;
constexpr uint32_t kInvalid = 0xFFFFFFFFu;
constexpr uint64_t kEmptyWord = 0xFFFFFFFFFFFFFFFEull;
constexpr uint64_t kTombWord = 0xFFFFFFFDFFFFFFFDull;
constexpr uint64_t kNextNone = 0xFFFFFFFFFFFFFFFFull;  // word 15 of a non-primary slab
constexpr uint64_t kTreeNone = 0xFFFFFFFFFFFFFFFFull;  // <INF, INVALID> tree node
constexpr int kGroup = 16;          // lanes per slab probe
constexpr int kKeysPerSlab = 15;    // data words per slab (14 in a multi-bucket primary slab)
constexpr int kBlock = 256;         // threads per block (4 waves, 16 groups)
constexpr int kGroupsPerBlock = kBlock / kGroup;
constexpr uint32_t kHeavyBuckets = 16;  // vertices with more buckets are walked by a block

// One view of the graph (forward, reverse or undirected), passed by value to kernels.
struct DView {
  uint64_t* slab;       // slab s occupies words [16 s, 16 s + 16); slab v is v's primary
  const uint32_t* nbk;  // bucket count per vertex (a copy of the primary slabs' meta)
  uint32_t* pool_ctr;   // [0] chained slabs handed out by the bump pointer so far,
                        // [1] slabs ever appended to the free list, [2] taken from it,
                        // [3] spares returned by the running insert kernels
  uint32_t* free_ids;   // free list: a ring of pool_cap reclaimed slab ids
  uint32_t* spare_ids;  // slabs taken but never linked by the running insert kernels
  uint32_t pool_base;   // index of the first chained (pool) slab
  uint32_t pool_cap;    // number of pool slabs
  uint32_t* deg;        // live keys per vertex
  uint64_t hash_a;      // multiply-shift hash: bucket = hi32(a*key + b) * nb >> 32
  uint64_t hash_b;
};

__device__ __host__ inline uint32_t bucket_of(uint32_t key, uint32_t nb, uint64_t a, uint64_t b) {
  uint32_t h = (uint32_t)((a * (uint64_t)key + b) >> 32);
  return (uint32_t)(((uint64_t)h * nb) >> 32);
}

__device__ __host__ inline bool valid_key(uint32_t k) { return k < kTombKey; }
__device__ __host__ inline uint64_t primary_link(uint32_t nb, uint32_t next) {
  return ((uint64_t)nb << 32) | next;
}

// ----------------------------------------------------------------- lane helpers
__device__ inline int lane64() { return (int)__lane_id(); }
__device__ inline int glane() { return (int)(__lane_id() & 15); }
__device__ inline int group_base_lane() { return (int)(__lane_id() & 48); }

// 16-bit ballot of the calling lane's group (all 16 lanes of a group run together).
__device__ inline uint32_t gballot(bool p) {
  uint64_t b = __ballot(p);
  return (uint32_t)(b >> group_base_lane()) & 0xFFFFu;
}
__device__ inline uint32_t gbcast(uint32_t v, int src) { return __shfl(v, src, kGroup); }
__device__ inline uint64_t gbcast64(uint64_t v, int src) {
  uint32_t lo = __shfl((uint32_t)v, src, kGroup);
  uint32_t hi = __shfl((uint32_t)(v >> 32), src, kGroup);
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline double gsum(double v) {
  for (int o = kGroup / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kGroup);
  return v;
}
__device__ inline uint64_t gsum_u64(uint64_t v) {
  for (int o = kGroup / 2; o > 0; o >>= 1) {
    uint32_t lo = __shfl_xor((uint32_t)v, o, kGroup);
    uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, kGroup);
    v += ((uint64_t)hi << 32) | lo;
  }
  return v;
}
__device__ inline uint64_t gmin_u64(uint64_t v) {
  for (int o = kGroup / 2; o > 0; o >>= 1) {
    uint32_t lo = __shfl_xor((uint32_t)v, o, kGroup);
    uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, kGroup);
    uint64_t w = ((uint64_t)hi << 32) | lo;
    v = w < v ? w : v;
  }
  return v;
}

// Number of set bits of `m` in lanes below the calling lane (mbcnt).
__device__ inline uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Wave-aggregated append (the paper's warp enqueue, Alg. 2, with ballot + mbcnt): every
// active lane with `p` writes `v` at a slot reserved by one atomic per wave.
__device__ inline void wave_push(uint32_t* q, uint32_t* ctr, bool p, uint32_t v) {
  uint64_t m = __ballot(p);
  if (m == 0) return;
  int leader = __builtin_ctzll(m);
  uint32_t base = 0;
  if (lane64() == leader) base = atomicAdd(ctr, (uint32_t)__popcll(m));
  base = __shfl(base, leader);
  if (p) q[base + lanes_below(m)] = v;
}

// ----------------------------------------------------------------- block-staged appends
// Appends to a queue whose counter would otherwise take one atomic per wave (sparse pushes
// from many waves serialize on that one address) go to an LDS buffer per output, with one
// LDS atomic per wave; when the kernel ends, the block reserves room for each buffer with a
// single global atomic and copies it out.  A full buffer spills further appends straight to
// its output.  Every thread of the block must reach stage_close (no early return).
constexpr uint32_t kStage = 1024;
struct Stage {
  uint32_t n, base;
  uint32_t* q;    // output queue and its counter
  uint32_t* ctr;
  uint32_t buf[kStage];
};

// Thread 0 opens the stages; the caller then synchronizes the block once.
__device__ inline void stage_open(Stage& S, uint32_t* q, uint32_t* ctr) {
  if (threadIdx.x == 0) {
    S.n = 0;
    S.q = q;
    S.ctr = ctr;
  }
}

// Reserve `cnt` (0..15) staged slots per active lane: positions [pos, pos + cnt) of the
// block's buffer, the part at or past kStage going straight to the output at
// spill + (position - max(base, kStage)), with one global atomic per wave.
struct StageSlots {
  uint32_t pos, lo, spill;
};
__device__ inline StageSlots stage_reserve(Stage& S, uint32_t cnt, bool& any) {
  uint32_t excl = 0, total = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint64_t m = __ballot((cnt >> b) & 1u);
    excl += lanes_below(m) << b;
    total += (uint32_t)__popcll(m) << b;
  }
  any = total != 0;
  if (!any) return StageSlots{0, 0, 0};
  const int leader = __builtin_ctzll(__ballot(true));
  uint32_t base = 0;
  if (lane64() == leader) base = atomicAdd(&S.n, total);
  base = __shfl(base, leader);
  const uint32_t lo = max(base, kStage);
  uint32_t spill = 0;
  if (base + total > kStage && lane64() == leader) spill = atomicAdd(S.ctr, base + total - lo);
  spill = __shfl(spill, leader);
  return StageSlots{base + excl, lo, spill};
}

__device__ inline void stage_put(Stage& S, const StageSlots& t, uint32_t pos, uint32_t v) {
  if (pos < kStage) S.buf[pos] = v;
  else S.q[t.spill + (pos - t.lo)] = v;
}

__device__ inline void stage_push(Stage& S, bool p, uint32_t v) {
  bool any;
  const StageSlots t = stage_reserve(S, p ? 1u : 0u, any);
  if (p) stage_put(S, t, t.pos, v);
}

template <int K>
__device__ inline void stage_close(Stage (&S)[K]) {
  __syncthreads();
  if (threadIdx.x < K) {
    Stage& t = S[threadIdx.x];
    const uint32_t n = min(t.n, kStage);
    t.base = n ? atomicAdd(t.ctr, n) : 0u;
  }
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    const uint32_t n = min(S[k].n, kStage);
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) S[k].q[S[k].base + i] = S[k].buf[i];
  }
}

// ----------------------------------------------------------------- memory access
// Slab words are read with relaxed atomic loads of wavefront scope: ordinary cached
// loads for the hardware, but the compiler may not merge or hoist them across the CASes
// of a retry loop.  The update protocol never relies on a load being fresh: a stale word
// only makes a CAS fail, and the CAS returns the true value.
__device__ inline uint64_t ld_word(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
// Tree nodes and union-find parents are read the same way: a value another lane changes
// during the kernel may be seen late (the L2 of each XCD caches it), which only delays
// progress (a stale distance relaxes worse candidates, a stale parent makes a CAS fail and
// return the true one).  Agent-scope loads would bypass that cache on every read.
__device__ inline uint32_t ld_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ inline uint64_t ld_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ inline uint64_t cas64(uint64_t* p, uint64_t expect, uint64_t desire) {
  return atomicCAS((unsigned long long*)p, (unsigned long long)expect, (unsigned long long)desire);
}
__device__ inline uint64_t amin64(uint64_t* p, uint64_t v) {
  return atomicMin((unsigned long long*)p, (unsigned long long)v);
}

__device__ inline uint64_t* slab_ptr(const DView& V, uint32_t s) {
  return V.slab + (uint64_t)s * kGroup;
}

// ----------------------------------------------------------------- slab iterator
// Walk every slab of vertex v (all buckets, each chain to its end), calling
// f(word, is_data) on the 16 lanes of the group for each slab.  This is the SlabIterator
// of section 3.4 (a BucketIterator per bucket, one after the other).
template <class F>
__device__ inline void walk_chain(const DView& V, uint32_t s, uint64_t x, int nd, F&& f) {
  const int gl = glane();
  while (true) {
    f(x, gl < nd);
    s = gbcast((uint32_t)x, 15);
    if (s == kInvalid) return;
    x = ld_word(slab_ptr(V, s) + gl);
    nd = kKeysPerSlab;
  }
}

template <class F>
__device__ inline void for_each_slab(const DView& V, uint32_t v, F&& f) {
  const int gl = glane();
  const uint64_t x = ld_word(slab_ptr(V, v) + gl);
  const uint32_t nb = (uint32_t)(gbcast64(x, 15) >> 32);
  const uint32_t xb = nb > 1 ? gbcast((uint32_t)x, 14) : 0u;
  walk_chain(V, v, x, nb > 1 ? kKeysPerSlab - 1 : kKeysPerSlab, f);
  for (uint32_t b = 1; b < nb; ++b) {
    const uint32_t s = xb + b - 1;
    walk_chain(V, s, ld_word(slab_ptr(V, s) + gl), kKeysPerSlab, f);
  }
}

// Walk the buckets b0, b0+stride, ... of vertex v (used when a block shares one vertex).
template <class F>
__device__ inline void for_each_slab_strided(const DView& V, uint32_t v, uint32_t b0, uint32_t stride,
                                             F&& f) {
  const int gl = glane();
  const uint64_t x = ld_word(slab_ptr(V, v) + gl);
  const uint32_t nb = (uint32_t)(gbcast64(x, 15) >> 32);
  const uint32_t xb = nb > 1 ? gbcast((uint32_t)x, 14) : 0u;
  for (uint32_t b = b0; b < nb; b += stride) {
    if (b == 0) {
      walk_chain(V, v, x, nb > 1 ? kKeysPerSlab - 1 : kKeysPerSlab, f);
    } else {
      const uint32_t s = xb + b - 1;
      walk_chain(V, s, ld_word(slab_ptr(V, s) + gl), kKeysPerSlab, f);
    }
  }
}

// Walk buckets [b0, min(b1, nb)) of vertex v (a work item of a heavy vertex).
template <class F>
__device__ inline void for_each_bucket_range(const DView& V, uint32_t v, uint32_t b0, uint32_t b1, F&& f) {
  const int gl = glane();
  const uint64_t x = ld_word(slab_ptr(V, v) + gl);
  const uint32_t nb = (uint32_t)(gbcast64(x, 15) >> 32);
  const uint32_t xb = nb > 1 ? gbcast((uint32_t)x, 14) : 0u;
  if (b1 > nb) b1 = nb;
  for (uint32_t b = b0; b < b1; ++b) {
    if (b == 0) {
      walk_chain(V, v, x, nb > 1 ? kKeysPerSlab - 1 : kKeysPerSlab, f);
    } else {
      const uint32_t s = xb + b - 1;
      walk_chain(V, s, ld_word(slab_ptr(V, s) + gl), kKeysPerSlab, f);
    }
  }
}

// ----------------------------------------------------------------- one op per lane
// Batched insert/delete/query ops are independent and latency-bound, so each lane runs
// its own op and reads the whole slab itself (8 x 16-byte loads): a wave keeps 64 probes
// in flight instead of the 4 a 16-lane group gives.
struct Slab {
  uint64_t w[16];
};

__device__ inline void load_slab(const DView& V, uint32_t s, Slab& sl) {
  const uint4* q = reinterpret_cast<const uint4*>(slab_ptr(V, s));
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint4 v = q[i];
    sl.w[2 * i] = ((uint64_t)v.y << 32) | v.x;
    sl.w[2 * i + 1] = ((uint64_t)v.w << 32) | v.z;
  }
}

// Load the first slab of the bucket of `key` in u's table; returns its index and sets
// nd (data words) and *extra (1 when a second head access was needed).
__device__ inline uint32_t lane_head(const DView& V, uint32_t u, uint32_t key, Slab& sl, int& nd,
                                     uint32_t* extra = nullptr) {
  load_slab(V, u, sl);
  const uint32_t nb = (uint32_t)(sl.w[15] >> 32);
  nd = kKeysPerSlab;
  if (extra) *extra = 0;
  if (nb <= 1) return u;
  const uint32_t b = bucket_of(key, nb, V.hash_a, V.hash_b);
  if (b == 0) {
    nd = kKeysPerSlab - 1;
    return u;
  }
  const uint32_t s = (uint32_t)sl.w[14] + b - 1;
  load_slab(V, s, sl);
  if (extra) *extra = 1;
  return s;
}

// Scan the data words [0, nd) of a slab: index and word of `key` (or -1), and the lowest
// EMPTY word at or above `floor` (or -1).
__device__ inline void scan_slab(const Slab& sl, int nd, uint32_t key, int floor, int& hit,
                                 uint64_t& hitw, int& empty) {
  hit = -1;
  empty = -1;
  hitw = kEmptyWord;
#pragma unroll
  for (int i = kKeysPerSlab - 1; i >= 0; --i) {
    if (i < nd) {
      const uint32_t k = (uint32_t)sl.w[i];
      if (k == key) {
        hit = i;
        hitw = sl.w[i];
      }
      if (k == kEmptyKey && i >= floor) empty = i;
    }
  }
}

// Lane-level SearchEdge: the data word of `key` in u's table, or kEmptyWord.
__device__ inline uint64_t lane_probe(const DView& V, uint32_t u, uint32_t key) {
  Slab sl;
  int nd;
  lane_head(V, u, key, sl, nd);
  while (true) {
    int hit, empty;
    uint64_t hitw;
    scan_slab(sl, nd, key, 0, hit, hitw, empty);
    if (hit >= 0) return hitw;
    if (empty >= 0) return kEmptyWord;
    const uint32_t s = (uint32_t)sl.w[15];
    if (s == kInvalid) return kEmptyWord;
    load_slab(V, s, sl);
    nd = kKeysPerSlab;
  }
}

// Where the lanes of a group probe many keys in one table (triangle counting): u's bucket
// count and first extra head slab, read once from u's primary slab by the whole group.
struct Table {
  uint32_t u, nb, xb;
};
__device__ inline Table group_table(const DView& V, uint32_t u) {
  const uint64_t x = ld_word(slab_ptr(V, u) + glane());
  const uint32_t nb = (uint32_t)(gbcast64(x, 15) >> 32);
  return Table{u, nb, nb > 1 ? gbcast((uint32_t)x, 14) : 0u};
}

// Single-lane membership test of `key` in a table whose head is known: one round trip per
// slab of the hashed chain (whole slabs are read with 16-byte loads).
__device__ inline bool lane_has(const DView& V, const Table& t, uint32_t key) {
  uint32_t s = t.u;
  int nd = kKeysPerSlab;
  if (t.nb > 1) {
    const uint32_t b = bucket_of(key, t.nb, V.hash_a, V.hash_b);
    if (b == 0) nd = kKeysPerSlab - 1;
    else s = t.xb + b - 1;
  }
  Slab sl;
  load_slab(V, s, sl);
  while (true) {
    int hit, empty;
    uint64_t hitw;
    scan_slab(sl, nd, key, 0, hit, hitw, empty);
    if (hit >= 0) return true;
    if (empty >= 0) return false;
    s = (uint32_t)sl.w[15];
    if (s == kInvalid) return false;
    load_slab(V, s, sl);
    nd = kKeysPerSlab;
  }
}

}  // namespace mk
