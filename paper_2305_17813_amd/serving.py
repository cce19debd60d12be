"""Continuous-batching serving loop over one resident graph.

Requests (edge-insert batches, edge-delete batches, edge-query batches, and BFS / SSSP /
PageRank requests) arrive over time.  Each admitted request gets a sequence number; a read
returns the answer on the graph after every update with a smaller sequence number.  The
loop keeps the graph resident in HBM and:

* merges consecutive update requests of one kind whose arcs do not overlap into one batch
  (each request's statuses are then exactly those it would get alone), admitted against
  the slab-pool headroom; when an insert might not fit, the slabs that deletes left behind
  are reclaimed first (compaction, while no read is in flight), and only then is the
  insert rejected (nothing applied);
* runs the reads between two updates concurrently, one per slot, each slot with its own
  HIP stream (default priority) and its own traversal workspace, so their kernels overlap
  on the device while new requests keep being admitted;
* replays pre-captured HIP graphs for query batches (one per slot and power-of-two size
  class; a short batch is padded with an out-of-range id, which a query reports absent);
* answers a BFS or SSSP from any other source with distances only (the direction-optimizing
  levels, or the distance-only SSSP), in the slot's workspace;
* brings the maintained algorithms (PageRank, and BFS/SSSP from the tracked source) up to
  date incrementally or by recompute, as the learned cost model decides, or always
  incrementally without it;
* reports p50 / p99 latency (arrival to completion) and sustained update and query rates.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional

import numpy as np
import torch

from . import inputs as I
from . import native

UPDATE_KINDS = ("insert", "delete")
READ_KINDS = ("query", "bfs", "sssp", "pagerank")
ALGO_ID = {"bfs": 0, "sssp": 1, "pagerank": 3}


@dataclass
class Request:
    rid: int
    kind: str
    arrival: float
    src: Optional[torch.Tensor] = None
    dst: Optional[torch.Tensor] = None
    w: Optional[torch.Tensor] = None
    source: int = 0
    seq: int = -1
    t_done: float = math.nan
    result: Any = None
    rejected: bool = False
    mode: int = native.AUTO

    @property
    def size(self) -> int:
        return 0 if self.src is None else int(self.src.numel())


def _lognormal(rng, median, sigma, lo, hi):
    return int(min(hi, max(lo, round(math.exp(rng.normal(math.log(median), sigma))))))


def make_requests(g: I.EdgeList, wl: I.Workload, n: int, rate: float, seed: int, tracked: int,
                  mix=(0.4, 0.4, 0.2), upd_median=10_000, upd_clip=(100, 2_000_000),
                  q_median=100_000, q_clip=(100, 2_000_000), sigma=1.0, device="cuda") -> List[Request]:
    """A seeded Poisson request stream: updates / query batches / BFS-SSSP-PageRank at `mix`,
    update sizes log-normal with median `upd_median` (inserts and deletes alike), query
    batches log-normal with median `q_median`, analytic sources half the tracked vertex and
    half uniform.  Payloads follow the workload's evolving arc set in arrival order."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        u = rng.random()
        if u < mix[0]:
            size = _lognormal(rng, upd_median, sigma, *upd_clip)
            if rng.random() < 0.5:
                s, d, w = wl.insert_batch(size)
                r = Request(rid, "insert", t, s, d, w)
            else:
                s, d = wl.delete_batch(size)
                r = Request(rid, "delete", t, s, d)
        elif u < mix[0] + mix[1]:
            size = _lognormal(rng, q_median, sigma, *q_clip)
            s, d = wl.query_batch(size)
            r = Request(rid, "query", t, s, d)
        else:
            kind = ("bfs", "sssp", "pagerank")[int(rng.integers(0, 3))]
            src = tracked if rng.random() < 0.5 else int(rng.integers(0, g.n))
            r = Request(rid, kind, t, source=src)
        for name in ("src", "dst", "w"):
            x = getattr(r, name)
            if x is not None:
                setattr(r, name, native.as_u32(x, device))
        out.append(r)
    return out


class QueryGraphs:
    """Per slot and power-of-two size class: fixed buffers and a captured HIP graph of one
    mk_query_edges launch over them."""

    def __init__(self, G: native.Graph, streams, min_log2=10, max_log2=21):
        self.G = G
        self.classes: Dict[tuple, tuple] = {}
        self.min_log2, self.max_log2 = min_log2, max_log2
        for slot, st in enumerate(streams):
            for k in range(min_log2, max_log2 + 1):
                n = 1 << k
                src = torch.full((n,), G.n, dtype=torch.int32, device=G.device)
                dst = torch.zeros(n, dtype=torch.int32, device=G.device)
                found = torch.empty(n, dtype=torch.uint8, device=G.device)
                wout = torch.empty(n, dtype=torch.int32, device=G.device)
                graph = torch.cuda.CUDAGraph()
                with torch.cuda.stream(st):
                    G.query_edges(src, dst, stream=st, out=(found, wout))  # warm-up outside capture
                    st.synchronize()
                    with torch.cuda.graph(graph, stream=st):
                        G.query_edges(src, dst, stream=st, out=(found, wout))
                st.synchronize()
                self.classes[(slot, k)] = (graph, src, dst, found, wout)

    def run(self, slot: int, s: torch.Tensor, d: torch.Tensor, stream):
        n = s.numel()
        k = max(self.min_log2, (n - 1).bit_length())
        if k > self.max_log2:
            return self.G.query_edges(s, d, stream=stream)
        graph, src, dst, found, wout = self.classes[(slot, k)]
        src[:n].copy_(s)
        src[n:].fill_(self.G.n)
        dst[:n].copy_(d)
        graph.replay()
        return found[:n].clone(), wout[:n].clone()


@dataclass
class ServeStats:
    latencies: Dict[str, List[float]] = field(default_factory=dict)
    update_ops: int = 0
    query_ops: int = 0
    wall_s: float = 0.0
    merged_batches: int = 0
    rejected: int = 0
    modes: Dict[str, Dict[int, int]] = field(default_factory=dict)

    def summary(self) -> dict:
        allv = [x for v in self.latencies.values() for x in v]
        pct = lambda v, q: float(np.percentile(v, q)) * 1e3 if v else None
        return {
            "requests": len(allv), "wall_s": self.wall_s,
            "p50_ms": pct(allv, 50), "p99_ms": pct(allv, 99),
            "per_kind": {k: {"n": len(v), "p50_ms": pct(v, 50), "p99_ms": pct(v, 99)}
                         for k, v in self.latencies.items()},
            "updates_per_s": self.update_ops / self.wall_s if self.wall_s else None,
            "queries_per_s": self.query_ops / self.wall_s if self.wall_s else None,
            "merged_update_batches": self.merged_batches, "rejected_updates": self.rejected,
            "maintained_modes": self.modes,
        }


class Server:
    def __init__(self, G: native.Graph, tracked_source: int, n_slots: int = 4, cost_model=None,
                 capture_queries: bool = True, max_merge: int = 4_000_000, keep_results: bool = False):
        self.G = G
        self.tracked = tracked_source
        self.n_slots = n_slots
        self.cm = cost_model
        self.max_merge = max_merge
        self.keep = keep_results
        self.streams = [torch.cuda.Stream(G.device) for _ in range(n_slots)]
        ws_bytes = max(G.lib.mk_bfs_levels_workspace_bytes(G.h), G.lib.mk_sssp_distances_workspace_bytes(G.h))
        self.ws = [torch.empty(ws_bytes, dtype=torch.uint8, device=G.device) for _ in range(n_slots)]
        self.qg = QueryGraphs(G, self.streams) if capture_queries else None
        self.pool = ThreadPoolExecutor(max_workers=n_slots)
        self.maint = threading.Lock()
        self.free_slots = deque(range(n_slots))
        self.slot_cv = threading.Condition()
        self.pending: Dict[str, tuple] = {}
        st = G.stats()
        self.compactions = 0
        self.headroom_est = None
        self._refresh_headroom(st)
        self._warm_up()

    def _warm_up(self):
        """First use of the host-side helpers (the merge check, the cost model) outside the
        measured run, so that one-time loading does not land on the first requests."""
        z = torch.zeros(4, dtype=torch.int32, device=self.G.device)
        self._disjoint([Request(-1, "insert", 0.0, z, z + 1)])
        if self.cm is not None:
            self.cm.choose(np.zeros((1, 12), np.float32))
        torch.cuda.synchronize()

    # ---------------------------------------------------------------- admission
    def _refresh_headroom(self, st=None):
        st = st or self.G.stats()
        per = []
        for v, mult in ((0, 1), (1, 1), (2, 2)):
            if st["pool_capacity"][v]:
                per.append((st["pool_capacity"][v] - st["pool_used"][v]) // mult)
        self.headroom_est = min(per) if per else 0

    def _admit_insert(self, n: int) -> bool:
        if n <= self.headroom_est:
            self.headroom_est -= n
            return True
        self._refresh_headroom()
        if n > self.headroom_est:
            # reclaim the slabs that deletes left behind (no read is in flight here), then retry
            self.compactions += 1
            self.G.compact()
            self._refresh_headroom()
        if n <= self.headroom_est:
            self.headroom_est -= n
            return True
        return False

    # ---------------------------------------------------------------- requests
    def _mode(self, algo: str) -> int:
        """The cost model's choice from the features of the latest update batch applied
        since `algo` last ran, computed here rather than on the update path; AUTO without a
        model or without a pending batch."""
        pend = self.pending.get(algo)
        if self.cm is None or pend is None:
            return native.AUTO
        kind, s, d, w = pend
        feats = self.G.batch_features(ALGO_ID[algo], (s, d, w) if kind == "insert" else None,
                                      (s, d) if kind == "delete" else None)
        return int(self.cm.choose(feats[None, :])[0])

    def _maintained(self, r: Request, stream):
        with self.maint:
            algo = r.kind
            mode = self._mode(algo)
            if algo == "pagerank":
                res = self.G.pagerank(mode=mode, stream=stream)
            elif algo == "bfs":
                res = self.G.bfs(r.source, mode, stream=stream)
            else:
                res = self.G.sssp(r.source, mode, stream=stream)
            stream.synchronize()
            self.pending.pop(algo, None)
            r.mode = mode
        return res

    def _read(self, r: Request, slot: int, t0: float):
        stream = self.streams[slot]
        try:
            with torch.cuda.stream(stream):
                if r.kind == "query":
                    res = (self.qg.run(slot, r.src, r.dst, stream) if self.qg is not None
                           else self.G.query_edges(r.src, r.dst, stream=stream))
                elif r.kind == "pagerank" or r.source == self.tracked:
                    res = self._maintained(r, stream)
                elif r.kind == "bfs":  # distances only: the direction-optimizing levels
                    res = (self.G.bfs_levels(r.source, False, self.ws[slot], slot, stream)[0], None)
                else:  # distances only: the distance-only SSSP
                    res = (self.G.sssp_distances(r.source, self.ws[slot], slot, stream), None)
                stream.synchronize()
            r.t_done = time.perf_counter() - t0
            r.result = res if self.keep else None
        finally:
            with self.slot_cv:
                self.free_slots.append(slot)
                self.slot_cv.notify()

    def _take_slot(self) -> int:
        with self.slot_cv:
            while not self.free_slots:
                self.slot_cv.wait()
            return self.free_slots.popleft()

    def _apply_updates(self, group: List[Request], t0: float, stats: ServeStats):
        kind = group[0].kind
        s = torch.cat([r.src for r in group]) if len(group) > 1 else group[0].src
        d = torch.cat([r.dst for r in group]) if len(group) > 1 else group[0].dst
        w = None
        if kind == "insert":
            w = torch.cat([r.w for r in group]) if len(group) > 1 else group[0].w
            if not self._admit_insert(s.numel()):
                for r in group:
                    r.rejected = True
                    r.t_done = time.perf_counter() - t0
                stats.rejected += len(group)
                return
        if self.cm is not None:  # the latest batch, remembered until each algorithm next runs
            for algo in ALGO_ID:
                self.pending[algo] = (kind, s, d, w)
        main = self.G.stream
        if kind == "insert":
            st = self.G.insert_edges(s, d, w, stream=main)
        else:
            st = self.G.delete_edges(s, d, stream=main)
        main.synchronize()
        now = time.perf_counter() - t0
        off = 0
        for r in group:
            n = r.size
            r.result = st[off:off + n] if self.keep else None
            off += n
            r.t_done = now
        stats.update_ops += s.numel()
        stats.merged_batches += 1

    def _disjoint(self, group: List[Request]) -> bool:
        keys = torch.cat([I.key_of(native.u32_to_i64(r.src), native.u32_to_i64(r.dst)) for r in group])
        return torch.unique(keys).numel() == keys.numel()

    def run(self, requests: List[Request], realtime: bool = True) -> ServeStats:
        stats = ServeStats()
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = time.perf_counter()
        inflight = []
        i = 0
        seq = 0
        while i < len(reqs):
            r = reqs[i]
            now = time.perf_counter() - t0
            if realtime and r.arrival > now:
                time.sleep(min(r.arrival - now, 0.0005))
                continue
            if r.kind in UPDATE_KINDS:
                for f in inflight:  # reads admitted before this update see the old graph
                    f.result()
                inflight.clear()
                group = [r]
                total = r.size
                j = i + 1
                now = time.perf_counter() - t0
                while (j < len(reqs) and reqs[j].kind == r.kind and reqs[j].arrival <= now
                       and total + reqs[j].size <= self.max_merge):
                    group.append(reqs[j])
                    total += reqs[j].size
                    j += 1
                if len(group) > 1 and not self._disjoint(group):
                    group = group[:1]
                    j = i + 1
                for g in group:
                    g.seq = seq
                    seq += 1
                self._apply_updates(group, t0, stats)
                i += len(group)
            else:
                r.seq = seq
                seq += 1
                slot = self._take_slot()
                inflight.append(self.pool.submit(self._read, r, slot, t0))
                if r.kind == "query":
                    stats.query_ops += r.size
                i += 1
        for f in inflight:
            f.result()
        stats.wall_s = time.perf_counter() - t0
        for r in reqs:  # burst mode: every request is taken as arrived at the start
            stats.latencies.setdefault(r.kind, []).append(r.t_done - (r.arrival if realtime else 0.0))
            if r.kind in ("pagerank", "bfs", "sssp") and (r.kind == "pagerank" or r.source == self.tracked):
                stats.modes.setdefault(r.kind, {}).setdefault(int(r.mode), 0)
                stats.modes[r.kind][int(r.mode)] += 1
        return stats

    def close(self):
        self.pool.shutdown(wait=True)


def run_alone(G: native.Graph, requests: List[Request], tracked: int):
    """The same requests one at a time, in sequence order, on the graph's stream: the
    reference each result of the mixed run must equal."""
    out = {}
    for r in sorted(requests, key=lambda r: r.seq):
        if r.kind == "insert":
            out[r.rid] = None if r.rejected else G.insert_edges(r.src, r.dst, r.w)
        elif r.kind == "delete":
            out[r.rid] = G.delete_edges(r.src, r.dst)
        elif r.kind == "query":
            out[r.rid] = G.query_edges(r.src, r.dst)
        elif r.kind == "pagerank":
            out[r.rid] = G.pagerank()
        elif r.kind == "bfs":
            out[r.rid] = G.bfs(r.source)
        else:
            out[r.rid] = G.sssp(r.source)
        torch.cuda.synchronize()
    return out
