// Host-side graph object shared by the library's translation units.
#pragma once
#include <atomic>
#include <deque>
#include <string>
#include <vector>

#include "meerkat_mi355x.h"
#include "mk_device.h"

namespace mk {

enum { VF = 0, VR = 1, VU = 2 };
constexpr uint32_t kSlots = 16;  // concurrent one-off traversals (distinct streams)
constexpr uint32_t kPrParts = 8192;  // FP64 partial sums of one PageRank iteration
enum BatchKind { kInsertBatch = 0, kDeleteBatch = 1 };

// One applied update batch, remembered for the incremental algorithms.  Its ops live in
// the change log at [off, off + n) with their endpoints, weight, per-op status and the
// "undirected edge changed" flag.
struct BatchRec {
  int kind;
  uint64_t off, n, seq;
};

struct Log {
  uint32_t *s = nullptr, *d = nullptr, *w = nullptr;
  uint8_t *st = nullptr, *uf = nullptr;
};

struct ViewHost {
  bool on = false;
  DView d{};
  uint32_t* nbk = nullptr;     // bucket count per vertex
  uint64_t head_reserved = 0;  // head slabs the arena reserves (upper bound)
  uint64_t n_head = 0;         // head slabs in use (N primary + extra)
  uint64_t pool_cap = 0;       // chained slabs
  uint64_t pool_used_est = 0;  // host-side upper bound of the pool slabs in use
  uint64_t pool_hw = 0;        // bump-pointer high-water mark read back last
  uint64_t added = 0;          // slabs the inserts so far may have taken (running sum of
                               // the per-call bounds; snapshots are placed against it)
  // IterationScheme2 work list (fwd and rev views): bucket k = off[v] + i of vertex v is the
  // pair <pair_v[k], pair_i[k]> = <v, i>, with off the exclusive scan of the bucket counts.
  // Bucket counts never change after creation, so the list is built once, when first used.
  uint32_t* pair_v = nullptr;
  uint32_t* pair_i = nullptr;
  uint32_t* pair_off = nullptr;
  bool pairs_ok = false;
};

struct AlgoState {
  bool valid = false;      // holds a result for the graph as of batch `seen_seq`
  uint32_t source = 0;
  uint64_t seen_seq = 0;   // every batch with seq <= seen_seq is reflected
};

struct Counters {          // device-side scalars, one 4 KiB block
  uint32_t frontier[16];   // [0..8] rotating frontier sizes (light, heavy and giant
                           // queues), [9..10] far-pile sizes, [11..12] band thresholds,
                           // [13] smallest far distance
  uint32_t inval;          // invalidated-vertex list size
  uint32_t overflow;       // bit per view (1 fwd, 2 rev, 4 und): an insert found its pool empty
  uint32_t n_heavy_wcc;    // vertices of more than 16 buckets, all-arc WCC walk
  uint32_t n_heavy_pr;     // the same for the PageRank pull (reverse view)
  uint32_t n_heavy_tc;     // the same for the static triangle count (undirected view)
  uint32_t tc_work;        // next hub work item of the triangle batch update
  uint32_t n_listed_light; // vertices listed for an incremental WCC pass: up to 16 buckets,
  uint32_t n_listed_heavy; //   and more (these two are cleared together)
  uint32_t wcc_big;        // root of the sampled largest component of a static WCC
  unsigned long long tc_s[3];  // S1, S2, S3 of the triangle batch identity
  unsigned long long tc_total; // current triangle count
  unsigned long long u64tmp[4];
  double pr_acc[8];        // PageRank sums: [2i] dangling, [2i+1] L1 change (rotating)
  uint32_t pr_state[8];    // [0] done flag, [1] iterations run, [2] stall count
  double pr_last;          // last L1 change
  double pr_best;          // smallest L1 change seen
  double feat[6];          // batch-feature sums
  uint32_t feat_max[2];    // batch-feature maxima
  uint32_t snap[16];       // pool snapshot staging: view v's bump, free-end and free-take
                           // counters at [4v, 4v+3), the overflow bits at [12]
  float mlp_x[16];         // features of an MK_AUTO decision (MK_MLP_IN used)
  float mlp_y[4];          // the cost model's outputs for them (MK_MLP_OUT used)
};

// Asynchronous pool snapshots: after an insert that leaves the host-side bound short of
// another batch, the pool counters are copied to pinned memory behind an event, so that a
// later call can tighten the bound without synchronizing the stream.
constexpr int kSnaps = 4;
struct PoolSnap {
  hipEvent_t ev = nullptr;
  uint32_t* pin = nullptr;       // 16 pinned words (layout of Counters::snap)
  uint64_t added_at[3] = {};     // ViewHost::added when the snapshot was enqueued
  bool pending = false;          // enqueued and not yet consumed
};

}  // namespace mk

struct mk_graph {
  mk_config cfg{};
  uint32_t n = 0;
  uint64_t m0 = 0;            // arcs passed at creation
  mk::ViewHost view[3];
  char* arena = nullptr;
  size_t arena_bytes = 0, used = 0;

  // change log (ring of batches)
  mk::Log log{};
  uint64_t log_cap = 0, log_tail = 0;
  std::deque<mk::BatchRec> batches;
  uint64_t next_seq = 1;      // seq of the next applied batch
  uint64_t dropped_seq = 0;   // batches with seq <= dropped_seq are no longer in the log

  // traversal scratch
  mk::Counters* ctr = nullptr;
  uint32_t* fq[6] = {};      // light, heavy and giant frontier queues (two of each)
  uint32_t* mark = nullptr;
  uint32_t* inval = nullptr;
  uint32_t* far[2] = {};      // far piles of the weighted epilogue
  uint32_t* far_mark = nullptr;
  uint32_t sssp_delta = 0;    // band width of the weighted epilogue
  uint32_t stamp = 0;
  uint32_t rot = 0;           // frontier counter rotation

  uint64_t* bfs_D = nullptr;
  uint64_t* sssp_D = nullptr;
  mk::AlgoState bfs, sssp, wcc, pr, tc;
  uint32_t* wcc_parent = nullptr;
  uint64_t* upd_mark = nullptr;   // forward-view update mark per bucket chain (head slab id)
  uint32_t* wcc_flag = nullptr;   // per vertex: listed for the running incremental WCC pass
  void* lv_cnt = nullptr;         // counters of the level-synchronous BFS (256 B)
  uint32_t* lv_multi[2] = {};     // its multi-bucket work items (vertex, chunk)
  float* pr_x = nullptr;      // current ranks
  float* pr_y = nullptr;      // next ranks
  float* pr_c = nullptr;      // contribution per vertex
  uint32_t* heavy_rev = nullptr;  // rev-view vertices split into bucket work items
  double* pr_hacc = nullptr;      // FP64 partial sums of the heavy vertices
  double* pr_part = nullptr;      // FP64 per-block partial sums of one iteration (kPrParts)
  double* pr_pair = nullptr;      // FP64 in-arc sum per reverse-view bucket (IterationScheme2)
  uint32_t* pr_list = nullptr;    // packed in-arc keys of the reverse view (MK_ITER_PACKED),
                                  // room for every data word of its slabs
  uint32_t* pr_off = nullptr;     // N + 1 segment starts in pr_list (scan of the in-degrees)
  // hot-first order of the packed iterations: perm[i] = the vertex of rank i (sources sorted
  // by out-degree class, largest first), rank = its inverse, cp = contributions in rank order
  uint32_t* pr_perm = nullptr;
  uint32_t* pr_rank = nullptr;
  uint32_t* pr_skey[2] = {};      // sort keys (out-degree classes) and their sorted copy
  uint32_t* pr_sidx = nullptr;    // 0 .. N-1, the sort's values
  float* pr_cp = nullptr;
  uint64_t* pr_cr = nullptr;     // packing iteration: <rank, contribution bits> per vertex
  void* pr_sort_tmp = nullptr;
  size_t pr_sort_bytes = 0;
  int iter_scheme = MK_ITER_PACKED;   // how all-vertex walks are scheduled
  const float* cm_params = nullptr;   // cost-model parameters for MK_AUTO (device, caller's)
  uint32_t n_heavy_rev = 0;
  bool heavy_rev_ok = false;

  uint64_t* tc_keys[2] = {nullptr, nullptr};
  // packed neighbour lists of the triangle update: the keys of the vertices whose
  // neighbourhood is walked against a hub's set, one u32 per key, at tc_off[v]
  uint32_t* tc_list = nullptr;
  uint64_t* tc_off = nullptr;
  void* sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  void* scan_tmp = nullptr;
  size_t scan_tmp_bytes = 0;

  uint64_t* h_pin = nullptr;  // pinned host words for read-backs
  mk::PoolSnap snap[mk::kSnaps];
  uint32_t snap_next = 0;     // ring position of the next snapshot
  std::atomic<uint32_t> overflowed{0};  // overflow bits seen on the host: the graph may have
                                        // lost arcs (read by concurrent read-only calls)
  uint64_t* slot_pin[mk::kSlots] = {};  // pinned words of one-off traversals, per slot
  uint64_t batches_applied = 0;
  std::string last_err;
};

namespace mk {
mk_status hip_fail(mk_graph* g, hipError_t e, const char* what);
// MK_ERR_OUT_OF_SLABS once an insert has overflowed a pool (the graph may have lost arcs).
// With `poll` (update calls only, which never overlap other calls on the graph) it first
// looks at completed pool snapshots, without waiting for the stream; read-only calls,
// which may overlap each other, only read the flag.
mk_status graph_guard(mk_graph* g, bool poll = false);
#define MK_HIP(g, call)                                  \
  do {                                                   \
    hipError_t _e = (call);                              \
    if (_e != hipSuccess) return mk::hip_fail(g, _e, #call); \
  } while (0)
#define MK_LAUNCH(g, what)                                   \
  do {                                                       \
    hipError_t _e = hipGetLastError();                       \
    if (_e != hipSuccess) return mk::hip_fail(g, _e, what);  \
  } while (0)

inline uint32_t grid_for_lanes(uint64_t lanes) { return (uint32_t)((lanes + kBlock - 1) / kBlock); }
inline uint32_t grid_for_groups(uint64_t groups) {
  return (uint32_t)((groups + kGroupsPerBlock - 1) / kGroupsPerBlock);
}

// Pending batches for an algorithm: those with seq > st.seen_seq.
struct Pending {
  bool lost = false;        // some pending batch fell out of the log
  int kinds = 0;            // bit 0: an insert batch is pending, bit 1: a delete batch
  std::vector<const BatchRec*> list;
};
Pending pending_for(const mk_graph* g, const AlgoState& st);
void mark_seen(mk_graph* g, AlgoState& st);

// One stretch of update ops for the batch features: n ops at src/dst/w (w may be null),
// deletions or insertions.
struct FeatPart {
  const uint32_t *src, *dst, *w;
  uint64_t n;
  bool del;
};
// The MK_MLP_IN features of mk_batch_features over any number of parts (synchronizes).
mk_status batch_features(mk_graph* g, int algo, const FeatPart* parts, int n_parts, float* h_out,
                         hipStream_t stream);
// The MLP forward pass (one thread per sample; mk_mlp_forward without argument checks).
void mlp_forward_launch(const float* params, const float* x, uint32_t n, float* y, hipStream_t stream);
// MK_AUTO with a cost model set: true when the model predicts a recompute of `algo` to be
// faster than applying the pending batches `p` incrementally (synchronizes).
mk_status auto_prefers_recompute(mk_graph* g, int algo, const Pending& p, hipStream_t stream, bool* out);

// IterationScheme2 work list of view v (built on first use; see ViewHost::pair_v).
mk_status ensure_pairs(mk_graph* g, int v, hipStream_t stream);

// Buffers of one level-synchronous BFS (mk_levels.hip): a 256-byte counter block, two
// frontier queues of N entries and two work-item arrays of levels_multi_cap(g) entries.
struct LevelBufs {
  void* cnt = nullptr;
  uint32_t* q[2] = {};
  uint32_t *multi_v = nullptr, *multi_c = nullptr;
};
size_t levels_multi_cap(const mk_graph* g);
mk_status levels_run(mk_graph* g, uint32_t source, bool allow_bu, const LevelBufs& b, uint32_t* level,
                     uint64_t* pin, uint32_t* h_bottom_up_steps, hipStream_t stream);
// Static BFS of the maintained state through the levels (needs MK_VIEW_REV): levels into
// `level`, then the tree nodes <level, smallest in-neighbour one level up> into D.
mk_status bfs_tree_by_levels(mk_graph* g, uint32_t source, uint32_t* level, uint64_t* D, hipStream_t stream);
// The same for SSSP: distance-only near-far relaxation into `dist`, then <dist, smallest
// in-neighbour u with dist(u) + w(u, v) = dist(v)> into D.
mk_status sssp_tree_by_distances(mk_graph* g, uint32_t source, uint32_t* dist, uint64_t* D, hipStream_t stream);
}  // namespace mk
