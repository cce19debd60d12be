"""Learned incremental-versus-recompute cost model.

An MLP (12 -> 64 -> 64 -> 3, ReLU, FP32) reads the features of a pending batch
(`Graph.batch_features`, computed by a HIP kernel) and predicts log(ms) of the incremental
path, log(ms) of a recompute and log2 of the initial slab-count scale.  Its forward pass,
gradient and Adam step are the library's HIP kernels (`mk_mlp_forward`, `mk_mlp_grad`,
`mk_mlp_adam`); this module marshals tensors, draws minibatches and keeps the records.

The training records come from the method itself: `generate_records` applies seeded
batches (sizes log-uniform, delete fraction uniform) to a graph and times, with HIP
events, each algorithm's incremental update (after the insert part and after the delete
part) and a recompute on the same graph state.  The fallback policy and the baseline of
the regret is the plain rule of the paper: always incremental.

The third output is trained by `slab_scale_records`: a graph is built at every slab scale
(a multiplier of the head-slab count, i.e. load factor 0.7 / scale) and timed on the same
work; the record carries log2 of the fastest scale, with its two timing targets masked.
`CostModel.slab_scale` turns the prediction into the nearest measured scale and
`load_factor_for` into the load factor to build the graph with (the default scale 1 is the
fallback).
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import native
from .native import _check, _ptr, load

N_IN, N_HID, N_OUT, N_PARAMS = 12, 64, 3, 5187
ALGOS = ["bfs", "sssp", "wcc", "pagerank", "tc"]
BASE_LOAD_FACTOR = 0.7
SLAB_SCALES = (0.5, 1.0, 2.0)  # head-slab count multipliers tried by slab_scale_records
RECOMPUTE_MARGIN = 1.25  # predicted incremental / recompute time ratio a recompute needs
SCALE_GAIN = 0.9  # a slab scale other than 1 is the label only when it takes < 90 % of the time


def load_factor_for(scale: float) -> float:
    """Load factor that builds `scale` times the head slabs of the default."""
    return BASE_LOAD_FACTOR / scale


class MLP:
    """Parameters, Adam moments and the training loop around the HIP kernels."""

    def __init__(self, device="cuda", seed: int = 0):
        self.lib = load()
        self.device = torch.device(device)
        g = torch.Generator().manual_seed(seed)
        parts = []
        for fan_out, fan_in, scale in [(N_HID, N_IN, math.sqrt(2.0 / N_IN)),
                                       (N_HID, N_HID, math.sqrt(2.0 / N_HID)),
                                       (N_OUT, N_HID, math.sqrt(1.0 / N_HID))]:
            parts.append(torch.randn(fan_out * fan_in, generator=g) * scale)
            parts.append(torch.zeros(fan_out))
        self.params = torch.cat(parts).float().to(self.device).contiguous()
        assert self.params.numel() == N_PARAMS
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(2, dtype=torch.float64, device=self.device)
        self.step = 0
        self.ws = None

    def _s(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        X = X.to(self.device, torch.float32).contiguous()
        Y = torch.empty(X.shape[0], N_OUT, dtype=torch.float32, device=self.device)
        _check(self.lib.mk_mlp_forward(_ptr(self.params), _ptr(X), X.shape[0], _ptr(Y), self._s()),
               "mk_mlp_forward")
        return Y

    def gradient(self, X, T, M):
        """Gradient of the masked MSE into self.grad; returns the loss (device tensor)."""
        n = X.shape[0]
        need = self.lib.mk_mlp_workspace_bytes(n)
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        _check(self.lib.mk_mlp_grad(_ptr(self.params), _ptr(X), _ptr(T), _ptr(M), n, _ptr(self.grad),
                                    _ptr(self.ws), self.ws.numel(), _ptr(self.loss), self._s()),
               "mk_mlp_grad")
        return self.loss[0]

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        _check(self.lib.mk_mlp_adam(_ptr(self.params), _ptr(self.grad), _ptr(self.m), _ptr(self.v),
                                    N_PARAMS, lr, b1, b2, eps, self.step, self._s()), "mk_mlp_adam")

    def train(self, X, T, M, epochs=200, batch=256, lr=3e-3, seed=0) -> List[float]:
        X = X.to(self.device, torch.float32).contiguous()
        T = T.to(self.device, torch.float32).contiguous()
        M = M.to(self.device, torch.float32).contiguous()
        n = X.shape[0]
        g = torch.Generator().manual_seed(seed)
        hist = []
        for ep in range(epochs):
            order = torch.randperm(n, generator=g).to(self.device)
            tot = 0.0
            for i in range(0, n, batch):
                idx = order[i:i + batch]
                loss = self.gradient(X[idx].contiguous(), T[idx].contiguous(), M[idx].contiguous())
                self.adam(lr=lr)
                tot += float(loss) * idx.numel()
            hist.append(tot / n)
        return hist


@dataclass
class Records:
    X: List[np.ndarray] = field(default_factory=list)   # features
    t_incr: List[float] = field(default_factory=list)   # ms, incremental (insert part + delete part)
    t_rec: List[float] = field(default_factory=list)    # ms, recompute on the same state
    algo: List[int] = field(default_factory=list)
    state: List[int] = field(default_factory=list)      # graph-state id (split key)
    slab_scale: List[float] = field(default_factory=list)  # log2 best slab scale, nan if unknown
    scale_ms: dict = field(default_factory=dict)  # record index -> ms per SLAB_SCALES entry

    def arrays(self):
        """Features, targets (log ms incremental, log ms recompute, log2 slab scale) and their
        masks (a timing record has no slab scale; a slab-scale record has no timings)."""
        X = np.stack(self.X).astype(np.float32)
        ti = np.asarray(self.t_incr, np.float64)
        tr = np.asarray(self.t_rec, np.float64)
        sc = np.asarray(self.slab_scale, np.float64)
        with np.errstate(invalid="ignore"):
            T = np.stack([np.nan_to_num(np.log(ti)), np.nan_to_num(np.log(tr)), np.nan_to_num(sc)], 1)
        M = np.stack([np.isfinite(ti), np.isfinite(tr), np.isfinite(sc)], 1).astype(np.float32)
        return X, T.astype(np.float32), M, ti, tr, np.asarray(self.algo), np.asarray(self.state)


def _time_call(fn, stream):
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b)


def run_algo(G, algo: str, mode: int, source: int):
    if algo == "bfs":
        return G.bfs(source, mode)
    if algo == "sssp":
        return G.sssp(source, mode)
    if algo == "wcc":
        return G.wcc(mode)
    if algo == "pagerank":
        return G.pagerank(mode=mode)
    return G.triangles(mode)


def generate_records(G, wl, source: int, n_batches: int, bmin: int, bmax: int, seed: int,
                     rec: Optional[Records] = None, state_base: int = 0, algos=ALGOS,
                     slab_scale: float = float("nan"), recompute_every: int = 1,
                     max_part: Optional[int] = None) -> Records:
    """Apply `n_batches` seeded mixed batches to G (and its workload `wl`): a size log-uniform
    in [bmin, bmax] and a delete fraction uniform in [0, 1] split each batch into an insert
    part and a delete part, applied in turn.  After each part, per algorithm, one record: the
    features of the part as MK_AUTO computes them (the part applied and pending for the
    algorithm), the time of the incremental update, and the time of a recompute on the same
    graph state.  The recompute time depends on the graph, not on the part, so it is measured
    every `recompute_every` parts per algorithm and reused in between.  A part larger than
    `max_part` is applied in slices of at most that size (one pending batch each).  An insert
    the slab pool refuses is retried once after compaction."""
    rec = rec or Records()
    rng = np.random.default_rng(seed)
    stream = G.stream
    for a in algos:  # every algorithm starts from a valid state
        run_algo(G, a, native.RECOMPUTE, source)
    t_rec_last = {}
    n_parts = 0

    def apply(kind, arrays):
        if kind == "insert":
            try:
                G.insert_edges(*arrays, status=False)
            except native.MkError as e:
                if e.status != 2:
                    raise
                G.compact()
                G.insert_edges(*arrays, status=False)
        else:
            G.delete_edges(*arrays, status=False)

    for b in range(n_batches):
        size = int(round(math.exp(rng.uniform(math.log(bmin), math.log(bmax)))))
        fdel = float(rng.uniform(0.0, 1.0))
        n_del = int(round(size * fdel))
        n_ins = size - n_del
        parts = []
        if n_ins:
            parts.append(("insert", wl.insert_batch(n_ins)))
        if n_del:
            parts.append(("delete", wl.delete_batch(n_del)))
        for kind, arrays in parts:
            k = arrays[0].numel()
            step = max_part or k
            for lo in range(0, k, step):
                apply(kind, tuple(x[lo:lo + step] for x in arrays))
            feats = {a: G.batch_features(ALGOS.index(a), arrays if kind == "insert" else None,
                                         arrays if kind == "delete" else None) for a in algos}
            for a in algos:
                t_i = _time_call(lambda: run_algo(G, a, native.INCR, source), stream)
                if a not in t_rec_last or n_parts % recompute_every == 0:
                    t_rec_last[a] = _time_call(lambda: run_algo(G, a, native.RECOMPUTE, source), stream)
                rec.X.append(feats[a])
                rec.t_incr.append(max(t_i, 1e-3))
                rec.t_rec.append(max(t_rec_last[a], 1e-3))
                rec.algo.append(ALGOS.index(a))
                rec.state.append(state_base + b)
                rec.slab_scale.append(slab_scale)
            n_parts += 1
    return rec


def slab_scale_records(graphs, seed: int, rec: Optional[Records] = None, state_base: int = 0,
                       device="cuda") -> Records:
    """Supervision of the slab-scale output.  Each graph (an `inputs.EdgeList`) is built, with
    the forward and reverse views, at every scale of SLAB_SCALES and timed on the same work:
    one insert batch and one delete batch of m/16 arcs, as many queries, a static BFS and a
    static PageRank from the vertex of largest out-degree.  The record holds the insert
    batch's features (taken on the default-scale graph) and log2 of the fastest scale, or 0
    (the default) when no scale beats the default by SCALE_GAIN."""
    from . import inputs as I
    rec = rec or Records()
    for k, g in enumerate(graphs):
        wl = I.Workload(g, seed + k)
        b = max(64, g.m // 16)
        ins, dels, qs = wl.insert_batch(b), wl.delete_batch(b), wl.query_batch(b)
        src = I.max_out_degree_vertex(g)
        feats, ms = None, []
        for sc in SLAB_SCALES:
            G = native.Graph(g.n, g.src, g.dst, g.w, views=native.VIEW_FWD | native.VIEW_REV,
                             load_factor=load_factor_for(sc), device=device)
            if sc == 1.0:
                feats = G.batch_features(0, ins, None)
            st = G.stream
            t = _time_call(lambda: G.insert_edges(*ins, status=False), st)
            t += _time_call(lambda: G.delete_edges(*dels, status=False), st)
            t += _time_call(lambda: G.query_edges(*qs), st)
            t += _time_call(lambda: G.bfs(src, native.RECOMPUTE), st)
            t += _time_call(lambda: G.pagerank(mode=native.RECOMPUTE), st)
            ms.append(t)
            del G
        rec.scale_ms[len(rec.X)] = tuple(ms)
        rec.X.append(feats)
        rec.t_incr.append(float("nan"))
        rec.t_rec.append(float("nan"))
        rec.algo.append(-1)
        rec.state.append(state_base + k)
        # the default scale keeps the label unless another is clearly faster (timing noise
        # alone must not teach the model to move away from it)
        best = int(np.argmin(ms))
        if ms[best] > SCALE_GAIN * ms[SLAB_SCALES.index(1.0)]:
            best = SLAB_SCALES.index(1.0)
        rec.slab_scale.append(math.log2(SLAB_SCALES[best]))
    return rec


class CostModel:
    """Trained MLP + the decision rule (recompute iff predicted incremental time exceeds the
    predicted recompute time by RECOMPUTE_MARGIN; near ties keep the incremental path)."""

    def __init__(self, mlp: MLP):
        self.mlp = mlp

    def predict(self, X: np.ndarray) -> np.ndarray:
        return self.mlp.forward(torch.as_tensor(np.atleast_2d(X))).cpu().numpy()

    def choose(self, X: np.ndarray) -> np.ndarray:
        """MK_INCR (1) or MK_RECOMPUTE (2) per feature row: a recompute only when it is
        predicted at least RECOMPUTE_MARGIN faster (the rule MK_AUTO applies in the library)."""
        y = self.predict(X)
        return np.where(y[:, 1] < y[:, 0] - math.log(RECOMPUTE_MARGIN), native.RECOMPUTE, native.INCR)

    def mode_for(self, G, algo: str, ins=None, dels=None) -> int:
        return int(self.choose(G.batch_features(ALGOS.index(algo), ins, dels)[None, :])[0])

    def slab_scale(self, X: np.ndarray) -> np.ndarray:
        """The measured scale (SLAB_SCALES) nearest in log2 to the prediction, per row."""
        y = self.predict(X)[:, 2]
        lg = np.log2(np.asarray(SLAB_SCALES))
        return np.asarray(SLAB_SCALES)[np.argmin(np.abs(y[:, None] - lg[None, :]), 1)]


def regret(t_incr, t_rec, choice):
    """Total time of the choices, of the best choices, and of always-incremental."""
    chosen = np.where(choice == native.INCR, t_incr, t_rec)
    best = np.minimum(t_incr, t_rec)
    return {"policy_ms": float(chosen.sum()), "best_ms": float(best.sum()),
            "always_incremental_ms": float(t_incr.sum()), "always_recompute_ms": float(t_rec.sum()),
            "policy_regret_ms": float(chosen.sum() - best.sum()),
            "heuristic_regret_ms": float(t_incr.sum() - best.sum())}


def scale_regret(cm: CostModel, rec: Records, idx) -> dict:
    """Total ms of the predicted slab scales, of the best ones and of the default scale 1,
    over the slab-scale records `idx`."""
    idx = [i for i in idx if i in rec.scale_ms]
    if not idx:
        return {}
    ms = np.asarray([rec.scale_ms[i] for i in idx])
    pick = cm.slab_scale(np.stack([rec.X[i] for i in idx]))
    col = np.asarray([SLAB_SCALES.index(float(p)) for p in pick])
    return {"policy_ms": float(ms[np.arange(len(idx)), col].sum()), "best_ms": float(ms.min(1).sum()),
            "default_ms": float(ms[:, SLAB_SCALES.index(1.0)].sum())}


def fit(rec: Records, holdout_frac=0.2, epochs=300, seed=0, device="cuda"):
    """Train on the older graph states, evaluate regret on the newest ones (the slab-scale
    records, if any, are judged by `scale_regret`)."""
    X, T, M, ti, tr, algo, state = rec.arrays()
    cut = np.quantile(state, 1 - holdout_frac)
    tr_idx = state < cut
    te_idx = ~tr_idx
    mlp = MLP(device, seed)
    hist = mlp.train(torch.from_numpy(X[tr_idx]), torch.from_numpy(T[tr_idx]), torch.from_numpy(M[tr_idx]),
                     epochs=epochs, seed=seed)
    cm = CostModel(mlp)
    timed = te_idx & np.isfinite(ti) & np.isfinite(tr)
    choice = cm.choose(X[timed])
    return cm, hist, regret(ti[timed], tr[timed], choice)
