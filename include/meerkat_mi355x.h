/* meerkat_mi355x.h -- C-ABI of the MI355X dynamic slab-hash graph library.
 *
 * A directed graph on a fixed vertex set [0, n_vertices) is stored as one hash table per
 * vertex: the destination id picks a bucket, and each bucket is a chain of 128-byte slabs
 * (section 2 of the paper: SlabHash slabs with an EMPTY and a TOMBSTONE sentinel; section
 * 3.1: head slabs of all vertices carved from one allocation, sized from the initial
 * degree and the load factor; further slabs come from a device slab allocator).
 *
 * Conventions shared by every entry point
 *   - Device pointers (prefix d_) are caller-owned device memory, typically torch tensors.
 *     Host pointers have the prefix h_.  The library never allocates device memory: every
 *     byte it uses lives in the caller's arena passed to mk_graph_create.  It allocates a
 *     few pinned host words per graph (hipHostMalloc) for size read-backs.
 *   - Every call is ordered on the given HIP stream.  Calls that must read a size back
 *     (traversal frontier sizes, PageRank convergence, mk_graph_stats) synchronize that
 *     stream.  Delete and query calls never synchronize.  An insert call synchronizes only
 *     when the host cannot otherwise show that the slab pools hold the batch: the host keeps
 *     an upper bound of the slabs in use (one per inserted arc and view), tightened without
 *     waiting by pool snapshots that earlier inserts left behind events; only when both fall
 *     short is the stream synchronized for the exact figures.  Under stream capture an
 *     insert never synchronizes (it returns MK_ERR_OUT_OF_SLABS instead), and replays of a
 *     captured insert are not counted by the host: a caller that replays inserts must admit
 *     them against mk_graph_stats itself.
 *   - Vertex ids and weights are uint32.  Ids >= 0xFFFFFFFD are reserved sentinels
 *     (EMPTY = 0xFFFFFFFE and TOMBSTONE = 0xFFFFFFFD, as in section 2; 0xFFFFFFFF is
 *     INVALID) and are rejected.  Weights must be >= 1 for shortest paths.
 *   - Errors are returned as mk_status; nothing aborts or throws across the ABI.  On any
 *     error other than MK_ERR_HIP the graph is unchanged.  A graph is not thread-safe:
 *     use one stream per graph.
 *   - Second line of defence: an insert lane that finds its pool empty all the same (the
 *     pre-check above makes this unreachable unless pool memory was damaged) stores nothing,
 *     reports status 2 for its arc and raises a device-side overflow bit.  Once the host has
 *     seen that bit (at the next synchronizing call, or from a completed pool snapshot), the
 *     graph may have lost arcs and every later call on it returns MK_ERR_OUT_OF_SLABS.
 */
#ifndef MEERKAT_MI355X_H
#define MEERKAT_MI355X_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mk_graph mk_graph; /* opaque; host-side metadata + pointers into the arena */

typedef enum {
  MK_OK = 0,
  MK_ERR_INVALID_ARG = 1,  /* null/misaligned pointer, size out of range, bad config      */
  MK_ERR_OUT_OF_SLABS = 2, /* the slab pool could not hold the batch; nothing was applied
                              (also: the graph overflowed a pool earlier and is unusable)  */
  MK_ERR_CAPACITY = 3,     /* arena too small, or a batch larger than the change log      */
  MK_ERR_STATE = 4,        /* the operation needs a view that the graph was built without */
  MK_ERR_HIP = 5           /* a HIP runtime call failed (the message is kept per graph)   */
} mk_status;

typedef enum {
  MK_AUTO = 0,      /* incremental when the pending batches allow it, else recompute; with
                       a cost model set (mk_set_cost_model) the model decides between them  */
  MK_INCR = 1,      /* incremental if at all possible (falls back to recompute if not)    */
  MK_RECOMPUTE = 2  /* recompute from scratch on the current graph                        */
} mk_mode;

enum {
  MK_VIEW_FWD = 1, /* out-edges <dst, weight>: updates, queries, BFS, SSSP (always on)   */
  MK_VIEW_REV = 2, /* in-edges <src, weight>: PageRank pull, decremental BFS/SSSP        */
  MK_VIEW_UND = 4  /* undirected simple graph: triangle counting                         */
};

typedef struct {
  uint32_t n_vertices;   /* fixed vertex count N (1 .. 2^30)                               */
  uint32_t views;        /* MK_VIEW_* mask; MK_VIEW_FWD is implied                           */
  float load_factor;     /* keys per bucket / slab capacity at build (the paper's load
                            factor, section 3.1); 0 = one bucket per vertex (hashing off)   */
  uint32_t hash_seed;    /* seed of the bucket hash                                         */
  uint64_t pool_slabs;   /* chained slabs per view beyond the head slabs; 0 = derived from
                            the edge-count hint with room for later inserts                  */
  uint64_t log_capacity; /* update ops remembered for incremental algorithms (ring of
                            batches); 0 = max(2^20, edge hint / 8)                           */
  uint32_t sssp_delta;   /* width of one distance band of the weighted frontier epilogue
                            (vertices are expanded band by band, nearest first); 0 = derived
                            from the initial mean weight and mean out-degree                 */
  uint32_t reserved;     /* must be 0                                                        */
} mk_config;

typedef struct {
  uint64_t n_arcs;            /* live arcs in the forward view                             */
  uint64_t n_und_edges;       /* live undirected edges (0 without MK_VIEW_UND)             */
  uint64_t head_slabs[3];     /* head slabs per view (fwd, rev, und)                       */
  uint64_t pool_used[3];      /* chained slabs handed out per view                         */
  uint64_t pool_capacity[3];  /* chained-slab capacity per view                            */
  uint64_t arena_bytes_used;  /* bytes of the arena actually carved                        */
  uint64_t batches_applied;   /* update batches applied since creation                     */
} mk_stats;

/* Bytes of arena needed for `cfg` and an initial edge count `n_edges_hint` (an upper bound
 * of the arcs passed to mk_graph_create).  Returns 0 if the configuration is invalid. */
size_t mk_arena_bytes(const mk_config* cfg, uint64_t n_edges_hint);

/* Build a graph from an initial arc list (section 3.1 memory management: per-vertex
 * bucket counts from the initial degree and the load factor, one exclusive scan for the
 * head-slab offsets, then a bulk insert).
 *   d_arena/arena_bytes : caller-owned device buffer of at least mk_arena_bytes(cfg, m)
 *                         bytes, 256-byte aligned; it must outlive the graph.
 *   d_src/d_dst/d_w     : m arcs (device, uint32 each); d_w may be NULL (weight 1).
 *                         Duplicates keep one copy; invalid arcs are skipped.
 *   out                 : receives the handle.  The call synchronizes `stream` once.
 * MK_ERR_OUT_OF_SLABS if an explicit pool_slabs ran out while the initial arcs were inserted
 * (no handle).  Lanes racing to extend one chain may each hold a slab for a moment, so an
 * explicit pool should have room for one slab per initial arc that a chain cannot take. */
mk_status mk_graph_create(const mk_config* cfg, void* d_arena, size_t arena_bytes,
                          const uint32_t* d_src, const uint32_t* d_dst, const uint32_t* d_w,
                          uint64_t m, hipStream_t stream, mk_graph** out);

/* Release the host-side handle (the arena stays the caller's). NULL is accepted. */
mk_status mk_graph_destroy(mk_graph* g);

/* Batched edge insertion (the graph-operation discussion of the experimental section:
 * hash the destination to one bucket of the source, walk that chain to its end to rule
 * out a duplicate, store the arc in the first EMPTY lane, link a fresh slab from the
 * allocator when the chain is full).  Every enabled view is updated in the same call.
 *   d_src/d_dst/d_w : n arcs (device).  d_w may be NULL (weight 1).
 *   d_status        : NULL or n bytes (device): 1 inserted, 0 already present (weight
 *                     unchanged), 2 rejected (id >= N, self-loop or reserved id).  Copies
 *                     of one arc inside a batch: exactly one copy reports 1; they must carry
 *                     one weight (each view keeps the copy that wins its own race).
 * MK_ERR_OUT_OF_SLABS when the pool might not hold the batch (nothing applied);
 * MK_ERR_CAPACITY when n exceeds the change-log capacity. */
mk_status mk_insert_edges(mk_graph* g, const uint32_t* d_src, const uint32_t* d_dst,
                          const uint32_t* d_w, uint64_t n, uint8_t* d_status, hipStream_t stream);

/* Batched edge deletion (same discussion: walk the hashed chain until the arc is found and
 * turn its lane into a TOMBSTONE; stop at the first EMPTY lane).  Status bytes as for
 * insert: 1 deleted, 0 absent, 2 rejected.  An undirected edge {u,v} leaves the
 * MK_VIEW_UND view only when neither (u,v) nor (v,u) remains after the batch. */
mk_status mk_delete_edges(mk_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                          uint8_t* d_status, hipStream_t stream);

/* Batched membership query (SearchEdge: probe only the hashed chain).
 *   d_found : n bytes (device), 1 present / 0 absent (also 0 for invalid ids).
 *   d_w     : NULL or n uint32 (device): the weight when present, else 0. */
mk_status mk_query_edges(mk_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                         uint8_t* d_found, uint32_t* d_w, hipStream_t stream);

/* Breadth-first search levels from `source` kept up to date across batches (section 4.2:
 * BFS runs the SSSP kernels with unit weights).  A first call or a new source computes
 * from scratch (with MK_VIEW_REV and a mean initial out-degree of at least 8: the
 * direction-optimizing levels of mk_bfs_levels, then each vertex's parent from its
 * in-arcs; otherwise the frontier kernels); later calls apply the pending batches
 * incrementally (insert prologue: relax the inserted arcs; delete prologue: invalidate the
 * dependence subtrees of deleted tree arcs and pull from valid in-neighbours, which needs
 * MK_VIEW_REV, else a recompute) and then run the frontier epilogue to a fixed point.
 *   d_level  : N uint32 (device): hop distance, 0xFFFFFFFF if unreachable.
 *   d_parent : NULL or N uint32 (device): the smallest-id in-neighbour one level up;
 *              `source` for the source; 0xFFFFFFFF if unreachable. */
mk_status mk_incr_bfs(mk_graph* g, uint32_t source, uint32_t* d_level, uint32_t* d_parent,
                      mk_mode mode, hipStream_t stream);

/* Single-source shortest paths (section 4.2, the dynamic SSSP algorithm), maintained as
 * for BFS with the arc weights.  The <distance, parent> pair of each vertex is one 64-bit
 * word updated by atomic minimum, so among equal distances the smallest parent id wins.
 * A recompute on a graph with MK_VIEW_REV and a mean initial out-degree of at least 8 runs
 * the distances of mk_sssp_distances and then gives each vertex the smallest in-neighbour
 * u with dist(u) + w(u, v) = dist(v); the result is the same.
 *   d_dist   : N uint32 (device): distance (saturates at 0xFFFFFFFE), 0xFFFFFFFF if
 *              unreachable.
 *   d_parent : NULL or N uint32 (device), as for BFS. */
mk_status mk_incr_sssp(mk_graph* g, uint32_t source, uint32_t* d_dist, uint32_t* d_parent,
                       mk_mode mode, hipStream_t stream);

/* One-off traversal from `source` (BFS levels when weighted == 0, SSSP distances
 * otherwise; same kernels and tie-break as mk_incr_bfs / mk_incr_sssp, computed from
 * scratch) that keeps all its state in the caller's workspace, so it changes nothing in
 * the graph and may overlap other reads of the graph on other streams (the serving loop
 * runs concurrent requests this way).  Updates must not run concurrently with it.
 *   d_ws/ws_bytes : device workspace of at least mk_traversal_workspace_bytes(g) bytes.
 *   slot          : 0..15; concurrent calls must use distinct slots (each slot owns a few
 *                   pinned host words for size read-backs).
 *   d_dist, d_parent (nullable) : N uint32 (device).  Synchronizes `stream`. */
size_t mk_traversal_workspace_bytes(const mk_graph* g);
mk_status mk_traverse_from(mk_graph* g, uint32_t source, int weighted, void* d_ws, size_t ws_bytes,
                           uint32_t slot, uint32_t* d_dist, uint32_t* d_parent, hipStream_t stream);

/* Distance-only BFS levels from `source` (the "vanilla" BFS of the experimental section:
 * 32-bit levels, no parents, against the tree variant that the maintained BFS/SSSP keep).
 * Level-synchronous; each step is top-down (the frontier's out-arcs claim unreached vertices)
 * or, with MK_VIEW_REV, bottom-up (each unreached vertex scans its in-arcs and stops at the
 * first one on the current level), chosen on the device per step by direction optimization
 * (Beamer et al.) recast for slabs: bottom-up when 2 nf + mf > 6 nu + N/2, with nf and mf
 * the frontier's vertices and out-arcs and nu the unreached vertices.
 * Reads the graph only; state lives in the caller's workspace, so it may overlap other reads
 * (not updates) on other streams.
 *   flags   : 0, or MK_BFS_TOP_DOWN_ONLY to never step bottom-up (also the behaviour without
 *             MK_VIEW_REV).
 *   d_ws/ws_bytes : device workspace of at least mk_bfs_levels_workspace_bytes(g) bytes.
 *   slot    : 0..15, as for mk_traverse_from (pinned words for size read-backs).
 *   d_level : N uint32 (device): the level (0 at the source), 0xFFFFFFFF if unreachable.
 *   h_bottom_up_steps (nullable, host): number of bottom-up steps taken.
 * Synchronizes `stream` after 4, 8, 16 and 32 levels, then every 16. */
enum { MK_BFS_TOP_DOWN_ONLY = 1 };
size_t mk_bfs_levels_workspace_bytes(const mk_graph* g);
mk_status mk_bfs_levels(mk_graph* g, uint32_t source, uint32_t flags, void* d_ws, size_t ws_bytes,
                        uint32_t slot, uint32_t* d_level, uint32_t* h_bottom_up_steps, hipStream_t stream);

/* Distance-only SSSP from `source` (the vanilla SSSP of the experimental section: 32-bit
 * distances relaxed by atomic minimum, no parents).  Near-far scheduling on the device: a
 * vertex whose distance drops below the band limit joins the next frontier, any other waits
 * on a far pile that is split at (its smallest distance + the graph's band width) when the
 * frontier runs dry.  Read-only on the graph, state in the caller's workspace, as for
 * mk_bfs_levels.  Weights must be >= 1.
 *   d_dist : N uint32 (device): the distance (sums saturate at 0xFFFFFFFE), 0xFFFFFFFF if
 *            unreachable.
 * Synchronizes `stream` after 4, 8, 16 and 32 steps, then every 16. */
size_t mk_sssp_distances_workspace_bytes(const mk_graph* g);
mk_status mk_sssp_distances(mk_graph* g, uint32_t source, void* d_ws, size_t ws_bytes, uint32_t slot,
                            uint32_t* d_dist, hipStream_t stream);

/* Weakly connected components (section 4.4: union-find with full path compression).
 * Inserted arcs are united incrementally; any pending deletion forces a recompute.
 *   d_label : N uint32 (device): the smallest vertex id of the component. */
mk_status mk_incr_wcc(mk_graph* g, uint32_t* d_label, mk_mode mode, hipStream_t stream);

/* How incremental WCC finds the arcs to unite (the incremental-WCC schemes that section 6.4
 * compares in its table of speedups over the naive scheme).  Every scheme gives the same
 * labels; they differ only in the slabs they read. */
typedef enum {
  MK_WCC_LOG = 0,    /* the arcs the pending insert batches logged as applied (no slab is
                        read; the default of mk_incr_wcc)                                   */
  MK_WCC_NAIVE = 1,  /* every arc of the graph: all slab lists of all vertices             */
  MK_WCC_SLAB = 2,   /* SlabIterator: all slabs of each vertex that gained out-arcs        */
  MK_WCC_UPDATE = 3  /* UpdateIterator (section 3.4): of those vertices, only the words past
                        each chain's update mark; the pass then moves the marks to the
                        chains' ends (the paper's UpdateSlabPointers)                        */
} mk_wcc_scheme;

/* mk_incr_wcc with an explicit scheme.  Update marks are kept for the forward view, one
 * per bucket chain: <slab, lane> of the first word not yet united.  They start at each
 * chain's head, move only in MK_WCC_UPDATE passes (and in recomputes run with that
 * scheme, which set every mark to its chain's end), and mk_compact resets the marks of
 * the chains it rewrites to their heads.  A lagging mark only makes the pass read more.
 * With hashing off (load_factor 0) every vertex has a single chain: the paper's
 * "UpdateIterator + single bucket" variant.  MK_ERR_INVALID_ARG for an unknown scheme. */
mk_status mk_incr_wcc_scheme(mk_graph* g, uint32_t* d_label, mk_mode mode, mk_wcc_scheme scheme,
                             hipStream_t stream);

/* How all-vertex walks are scheduled (section 3.4, IterationScheme1 and IterationScheme2).
 * SCHEME1 gives each vertex to one worker: a lane for a single-bucket vertex, a 16-lane
 * group for up to 16 buckets, work items of a few buckets for larger ones.
 * SCHEME2 gives each bucket chain <v, i> to a 16-lane group in a grid-stride loop over the
 * list of all <vertex, bucket> pairs (built once from one exclusive scan of the bucket
 * counts, which never change after creation); a per-vertex pass then adds the buckets'
 * partial results in bucket order.
 * PACKED (the default; not in the paper) is SCHEME1 for WCC.  For PageRank its first
 * iteration of a call walks the slabs as SCHEME1 does and also packs every vertex's in-arc
 * keys into one array (segments at the exclusive scan of the in-degrees, room for every
 * data word of the reverse view in the arena); the call's later iterations read those 4-byte
 * keys instead of 128-byte slabs.
 * The scheme applies to the PageRank pull over the reverse view and to the union over every
 * arc of a static (or naive incremental) WCC.  Results are the same under every scheme
 * (PageRank within its tolerance).  MK_ERR_INVALID_ARG for an unknown scheme. */
typedef enum { MK_ITER_SCHEME1 = 1, MK_ITER_SCHEME2 = 2, MK_ITER_PACKED = 3 } mk_iter_scheme;
mk_status mk_set_iteration_scheme(mk_graph* g, mk_iter_scheme scheme);

/* PageRank (section 4.1): PR'(v) = (1-d)/N + d * (sum over in-arcs u->v of PR(u)/out(u)
 * + sum over zero-out-degree z of PR(z)/N), iterated from 1/N (first call, RECOMPUTE) or
 * from the previous vector (incremental and decremental batches) until the L1 change of
 * one iteration is <= tol_l1, stops decreasing for three iterations, or max_iter is hit.
 * Needs MK_VIEW_REV.  Ranks are stored in FP32; sums and the L1 change use FP64.
 *   d_rank  : N float (device).   d_iters : NULL or 1 uint32 (device): iterations run. */
mk_status mk_incr_pagerank(mk_graph* g, float damping, double tol_l1, uint32_t max_iter,
                           float* d_rank, uint32_t* d_iters, mk_mode mode, hipStream_t stream);

/* Triangles of the undirected simple graph under the arc set (section 4.3).  After
 * insertions T += (S1 - S2 + S3/3)/2 and after deletions T -= (S1 + S2 + S3/3)/2 with
 * S1 = Count(G, G, B), S2 = Count(G, U, B), S3 = Count(U, U, B) over both directions of
 * the effective batch B, G the graph after the batch and U the graph of the batch alone;
 * a recompute counts every edge once from its lower-(degree, id) end.  Needs MK_VIEW_UND.
 *   d_count : 1 uint64 (device). */
mk_status mk_count_triangles(mk_graph* g, uint64_t* d_count, mk_mode mode, hipStream_t stream);

/* Slab iterator export: write every live arc (order unspecified) to d_src/d_dst/d_w
 * (device, capacity `cap` each; d_w may be NULL) and the count to *h_count.  Synchronizes.
 * MK_ERR_CAPACITY if cap is too small (*h_count still receives the count). */
mk_status mk_graph_export(mk_graph* g, uint32_t* d_src, uint32_t* d_dst, uint32_t* d_w,
                          uint64_t cap, uint64_t* h_count, hipStream_t stream);

/* Slab reclamation (the paper never reuses a slab: a deleted arc leaves a TOMBSTONE that
 * later inserts skip, so chains only grow under delete churn).  Every chain holding at least
 * `min_tombstones` tombstones (0 is taken as 1) is rewritten with its live arcs packed from
 * its head slab, EMPTY lanes after them, and the chain cut after the last slab it still
 * needs; the slabs after the cut return to the view's free list, which inserts draw from
 * once the bump pointer has handed out the whole pool.  The arc set, degrees and all
 * incremental algorithm state are unchanged; the forward view's update marks of the
 * rewritten chains go back to their heads (see mk_incr_wcc_scheme).  Must not overlap any other call on the same graph (reads included).
 *   h_freed : host; receives the number of slabs returned to the free lists. */
mk_status mk_compact(mk_graph* g, uint32_t min_tombstones, uint64_t* h_freed, hipStream_t stream);

/* Byte model of the batched operations (no change is made): the number of slabs that
 * `op` (0 = query/delete, which stop at the arc or the first EMPTY lane; 1 = insert, which
 * walks the hashed chain to its end) would read for each of the n arcs in `view` (0 fwd
 * keyed by src, 1 rev keyed by dst, 2 und in both directions), summed into *h_slabs.  The
 * benchmark turns it into algorithmic bytes.  Synchronizes.
 * MK_ERR_STATE if the view is not enabled. */
mk_status mk_probe_cost(mk_graph* g, int op, int view, const uint32_t* d_src, const uint32_t* d_dst,
                        uint64_t n, uint64_t* h_slabs, hipStream_t stream);

/* Occupancy and capacity figures (synchronizes).  Fills *h_out and returns
 * MK_ERR_OUT_OF_SLABS if the graph has overflowed a pool. */
mk_status mk_graph_stats(mk_graph* g, mk_stats* h_out, hipStream_t stream);

/* Structural self-check of every chain of every view: no duplicate keys in a vertex's
 * table, no EMPTY lane before a filled one inside a chain, next links in range, the key's
 * bucket matches its hash, degree counters match the live lanes.  *h_bad receives the
 * number of violations (0 when sound).  Synchronizes. */
mk_status mk_graph_check(mk_graph* g, uint64_t* h_bad, hipStream_t stream);

/* ---------------------------------------------------------------- cost model
 * A small MLP (MK_MLP_IN -> 64 -> 64 -> MK_MLP_OUT, ReLU, FP32) that predicts, from the
 * features of a pending batch, log(ms) of the incremental path, log(ms) of a recompute,
 * and log2 of the initial slab-count scale.  It picks MK_INCR or MK_RECOMPUTE per
 * algorithm and batch; the plain always-incremental rule is the fallback.  This is not
 * in the paper: its own measurements show incremental BFS/SSSP losing to recompute on
 * road networks (dynamic-vs-static speedups below 1 in the BFS and SSSP figures).
 * Parameters: MK_MLP_PARAMS floats, W1[64][12], b1[64], W2[64][64], b2[64], W3[3][64],
 * b3[3], row-major (output x input). */
#define MK_MLP_IN 12
#define MK_MLP_HIDDEN 64
#define MK_MLP_OUT 3
#define MK_MLP_PARAMS 5187

enum { MK_ALGO_BFS = 0, MK_ALGO_SSSP = 1, MK_ALGO_WCC = 2, MK_ALGO_PAGERANK = 3, MK_ALGO_TC = 4 };

/* Features of a batch about to be applied, for algorithm `algo` (MK_ALGO_*), into
 * h_out[MK_MLP_IN] (host): log2(1+ops), insert and delete fractions, log2 N, log2(1+arcs),
 * mean and max log2(1+out-degree) of the touched sources, mean log2(1+in-degree) of the
 * touched destinations, the affected fraction (BFS/SSSP: inserted arcs that would relax
 * plus deleted tree arcs; WCC: inserted arcs joining two components plus deletions;
 * PageRank: mean 1/(1+out-degree) of the sources; triangles: mean log2(1+smaller
 * undirected degree)), log2(1+deepest finite distance of the algorithm's tree), log2(1+
 * pending batches) and algo/4; every log2 figure is divided by 32 so that the features lie
 * roughly in [0, 1].  Either part may be empty (n = 0, pointers NULL).
 * Synchronizes. */
mk_status mk_batch_features(mk_graph* g, int algo, const uint32_t* d_ins_src, const uint32_t* d_ins_dst,
                            const uint32_t* d_ins_w, uint64_t n_ins, const uint32_t* d_del_src,
                            const uint32_t* d_del_dst, uint64_t n_del, float* h_out, hipStream_t stream);

/* Hand the cost model to the graph.  d_params: MK_MLP_PARAMS floats on the device (the
 * caller's; they are read at every MK_AUTO decision, so they must stay valid until cleared
 * or the graph is destroyed), or NULL to clear.  With a model set, an algorithm called with
 * MK_AUTO on pending batches that it could apply incrementally computes the features of
 * those batches (as mk_batch_features, over the change log, with every pending batch taken
 * as applied) and runs the MLP forward kernel: it recomputes when the predicted recompute
 * time is below the predicted incremental time.  That decision synchronizes the stream.
 * Without a model MK_AUTO applies the batches incrementally whenever it can. */
mk_status mk_set_cost_model(mk_graph* g, const float* d_params);

/* Bytes of device workspace mk_mlp_grad needs for a minibatch of n samples. */
size_t mk_mlp_workspace_bytes(uint32_t n);

/* Forward pass: d_x [n][MK_MLP_IN] -> d_y [n][MK_MLP_OUT] (device, FP32). */
mk_status mk_mlp_forward(const float* d_params, const float* d_x, uint32_t n, float* d_y,
                         hipStream_t stream);

/* Gradient of the masked mean squared error L = sum m (y - t)^2 / sum m over a minibatch
 * (d_t and d_mask are [n][MK_MLP_OUT]; a mask entry of 0 leaves that output unsupervised).
 * Writes d_grad [MK_MLP_PARAMS] (overwritten, not accumulated) and *d_loss (device double).
 * d_ws: device workspace of ws_bytes >= mk_mlp_workspace_bytes(n).  Deterministic. */
mk_status mk_mlp_grad(const float* d_params, const float* d_x, const float* d_t, const float* d_mask,
                      uint32_t n, float* d_grad, void* d_ws, size_t ws_bytes, double* d_loss,
                      hipStream_t stream);

/* mk_mlp_grad without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * workspace is a file-scope device array of mk_mlp_workspace_bytes(MK_MLP_GRAD_STATIC_MAX)
 * bytes (about 16 MiB), one copy per GPU, held by each GPU the library runs on until the
 * process ends; its address is looked up on the first call on a device.  Runs on the
 * current device (the pointers and the stream must belong to it) and allocates nothing.
 * Every call on one GPU shares that array and it keeps the last call's contents: calls that
 * overlap on one GPU (on other streams or from other threads) race and must be ordered by
 * the caller.
 *   n : 1 .. MK_MLP_GRAD_STATIC_MAX, else MK_ERR_CAPACITY (nothing launched).
 * Other arguments, results and determinism as for mk_mlp_grad. */
#define MK_MLP_GRAD_STATIC_MAX 16384
mk_status mk_mlp_grad_static(const float* d_params, const float* d_x, const float* d_t, const float* d_mask,
                             uint32_t n, float* d_grad, double* d_loss, hipStream_t stream);

/* One Adam step (Kingma and Ba, with bias correction; `step` counts from 1) on n_params
 * parameters with first and second moment buffers d_m, d_v (device, FP32). */
mk_status mk_mlp_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t n_params,
                      float lr, float beta1, float beta2, float eps, uint32_t step, hipStream_t stream);

/* Human-readable name of a status; the last HIP error text for MK_ERR_HIP. */
const char* mk_status_string(mk_status s);

#ifdef __cplusplus
}
#endif
#endif /* MEERKAT_MI355X_H */
