// Device-side building blocks of the slab-hash graph for gfx950 (CDNA4, wave64).
//
// Slab geometry (the paper's section 2 slab, redesigned for wave64): one slab is
// 128 bytes = one L2 line = 16 words of 8 bytes.  A *group* of 16 lanes (one DPP row)
// reads a slab with one coalesced dwordx2 per lane, so a wave64 runs four independent
// probes at once.  Word l (l < 15) holds the pair <key, weight> (key in the low half);
// word 15 holds <next slab index, unused>.  Keys are unordered within a slab.
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
constexpr uint64_t kNextNone = 0xFFFFFFFFFFFFFFFFull;
constexpr uint64_t kTreeNone = 0xFFFFFFFFFFFFFFFFull;  // <INF, INVALID> tree node
constexpr int kGroup = 16;          // lanes per slab probe
constexpr int kKeysPerSlab = 15;    // data words per slab
constexpr int kBlock = 256;         // threads per block (4 waves, 16 groups)
constexpr int kGroupsPerBlock = kBlock / kGroup;
constexpr uint32_t kHeavyBuckets = 16;  // vertices with more buckets are walked by a block

// One view of the graph (forward, reverse or undirected), passed by value to kernels.
struct DView {
  const uint2* dir;     // per vertex: x = first head slab, y = bucket count
  uint64_t* slab;       // slab s occupies words [16 s, 16 s + 16)
  uint32_t* pool_ctr;   // chained slabs handed out so far
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

// ----------------------------------------------------------------- memory access
// Mutating kernels read slab words with agent-scope atomic loads so that a wave on one
// XCD sees words written by a wave on another XCD (separate L2s); read-only kernels use
// ordinary cached loads.
template <bool kCoherent>
__device__ inline uint64_t ld_word(const uint64_t* p) {
  if constexpr (kCoherent)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}
__device__ inline uint32_t ld_u32_coherent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t ld_u64_coherent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
// Walk every slab of vertex v (all buckets, each chain to its end), calling f(word) on
// the 16 lanes of the group for each slab; lanes 0..14 hold the data words.  This is
// the SlabIterator of section 3.4 (a BucketIterator per bucket, one after the other).
template <bool kCoherent, class F>
__device__ inline void for_each_slab(const DView& V, uint32_t v, F&& f) {
  const uint2 de = V.dir[v];
  for (uint32_t b = 0; b < de.y; ++b) {
    uint32_t s = de.x + b;
    while (s != kInvalid) {
      const uint64_t x = ld_word<kCoherent>(slab_ptr(V, s) + glane());
      f(x);
      s = gbcast((uint32_t)x, 15);
    }
  }
}

// Walk the buckets b0, b0+stride, ... of vertex v (used when a block shares one vertex).
template <bool kCoherent, class F>
__device__ inline void for_each_slab_strided(const DView& V, uint2 de, uint32_t b0, uint32_t stride,
                                             F&& f) {
  for (uint32_t b = b0; b < de.y; b += stride) {
    uint32_t s = de.x + b;
    while (s != kInvalid) {
      const uint64_t x = ld_word<kCoherent>(slab_ptr(V, s) + glane());
      f(x);
      s = gbcast((uint32_t)x, 15);
    }
  }
}

// Group-cooperative membership probe (SearchEdge): walk only the hashed chain of `u`.
// Returns the data word when found, or kEmptyWord when absent.
template <bool kCoherent>
__device__ inline uint64_t probe(const DView& V, uint32_t u, uint32_t key) {
  const uint2 de = V.dir[u];
  uint32_t s = de.x + bucket_of(key, de.y, V.hash_a, V.hash_b);
  const int gl = glane();
  while (true) {
    const uint64_t x = ld_word<kCoherent>(slab_ptr(V, s) + gl);
    const uint32_t k = (uint32_t)x;
    const uint32_t hit = gballot(gl < kKeysPerSlab && k == key);
    if (hit) return gbcast64(x, __builtin_ctz(hit));
    if (gballot(gl < kKeysPerSlab && k == kEmptyKey)) return kEmptyWord;
    s = gbcast(k, 15);
    if (s == kInvalid) return kEmptyWord;
  }
}

}  // namespace mk
