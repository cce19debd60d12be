"""Seeded synthetic workload generators shared by the HIP path and the CPU oracle.

This module builds *inputs only*: edge lists, update batches and query batches shaped
like the paper's workloads (social power-law graphs, a uniform random graph and a road
network; the experimental setup section and its input-graph table).  It holds none of
the method's arithmetic: no hashing into buckets, no slab layout, no traversal.

Every random draw comes from one counter-based generator, the SplitMix64 output
function (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014) applied to ``seed + (i + 1) * 0x9E3779B97F4A7C15``.  It is written with
int64 torch operations whose wrap-around is the two's-complement one on every device,
so the same call returns bit-identical tensors on the CPU and on the GPU.

Keys: an arc (src, dst) is encoded as ``src << 32 | dst`` in an int64 tensor (ids are
below 2**31 in every workload here, so keys are non-negative and sort like pairs).
Weights are a function of the arc (of the unordered pair for undirected graphs), so a
re-inserted arc carries the weight it had before and duplicate draws cannot disagree.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import torch

_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK64 = (1 << 64) - 1


def _s64(v: int) -> int:
    """Reinterpret an unsigned 64-bit constant as the signed value torch stores."""
    v &= _MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of the uint64 bit pattern held in an int64 tensor."""
    return torch.bitwise_and(torch.bitwise_right_shift(x, k), (1 << (64 - k)) - 1)


def mix64(x: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output function on int64 bit patterns (wrap-around arithmetic)."""
    z = x
    z = torch.bitwise_xor(z, _srl(z, 30)) * _s64(_M1)
    z = torch.bitwise_xor(z, _srl(z, 27)) * _s64(_M2)
    return torch.bitwise_xor(z, _srl(z, 31))


def mix64_py(x: int) -> int:
    """Pure-Python SplitMix64 output function (used to pin the tensor version)."""
    z = x & _MASK64
    z = ((z ^ (z >> 30)) * _M1) & _MASK64
    z = ((z ^ (z >> 27)) * _M2) & _MASK64
    return z ^ (z >> 31)


def draws(seed: int, stream: int, start: int, n: int, device="cpu") -> torch.Tensor:
    """``n`` 64-bit draws (as int64) of stream ``stream``, counters start..start+n-1."""
    base = _s64(mix64_py(seed * 0x100000001B3 + stream * 0x2545F4914F6CDD1D + 0x5EED))
    ctr = torch.arange(start + 1, start + n + 1, dtype=torch.int64, device=device)
    return mix64(ctr * _s64(_GOLDEN) + base)


def below(r: torch.Tensor, bound: int) -> torch.Tensor:
    """Map 64-bit draws to integers in [0, bound) by multiply-shift of the top 32 bits."""
    assert 0 < bound <= (1 << 31)
    return _srl(_srl(r, 32) * bound, 32)


def key_of(src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
    return torch.bitwise_or(torch.bitwise_left_shift(src.to(torch.int64), 32), dst.to(torch.int64))


def split_key(key: torch.Tensor):
    return _srl(key, 32), torch.bitwise_and(key, 0xFFFFFFFF)


def arc_weight(src: torch.Tensor, dst: torch.Tensor, wmax: int, seed: int,
               undirected: bool = False) -> torch.Tensor:
    """Weight in [1, wmax] drawn once per arc (per unordered pair when undirected)."""
    s = src.to(torch.int64)
    d = dst.to(torch.int64)
    if undirected:
        s, d = torch.minimum(s, d), torch.maximum(s, d)
    salt = _s64(mix64_py(seed ^ 0x77E16475))
    return 1 + below(mix64(key_of(s, d) + salt), wmax)


def first_unique(keys: torch.Tensor) -> torch.Tensor:
    """Distinct values of ``keys`` in order of first occurrence."""
    if keys.numel() == 0:
        return keys
    uniq, inv = torch.unique(keys, sorted=True, return_inverse=True)
    pos = torch.arange(keys.numel(), device=keys.device)
    first = torch.full((uniq.numel(),), keys.numel(), dtype=torch.int64, device=keys.device)
    first.scatter_reduce_(0, inv, pos, reduce="amin")
    return uniq[torch.argsort(first)]


def shuffled(x: torch.Tensor, seed: int, stream: int) -> torch.Tensor:
    """Seeded permutation of a 1-D tensor (argsort of one draw per element)."""
    r = draws(seed, stream, 0, x.numel(), x.device)
    return x[torch.argsort(r, stable=True)]


def is_member(sorted_keys: torch.Tensor, q: torch.Tensor) -> torch.Tensor:
    """Membership of ``q`` in an ascending key tensor."""
    if sorted_keys.numel() == 0:
        return torch.zeros(q.shape, dtype=torch.bool, device=q.device)
    pos = torch.searchsorted(sorted_keys, q).clamp_(max=sorted_keys.numel() - 1)
    return sorted_keys[pos] == q


@dataclasses.dataclass
class EdgeList:
    """A directed arc list on ``n`` vertices (u32 ids and u32 weights as int64 tensors)."""
    n: int
    src: torch.Tensor
    dst: torch.Tensor
    w: torch.Tensor
    undirected: bool = False
    wmax: int = 100
    wseed: int = 0

    @property
    def m(self) -> int:
        return int(self.src.numel())

    def keys(self) -> torch.Tensor:
        return key_of(self.src, self.dst)

    def u32(self):
        """(src, dst, w) as int32 tensors holding the u32 bit patterns (all < 2**31)."""
        return (self.src.to(torch.int32), self.dst.to(torch.int32), self.w.to(torch.int32))


def _fresh_pairs(n: int, count: int, seed: int, stream: int, device, exclude_sorted=None,
                 undirected=False) -> torch.Tensor:
    """``count`` distinct uniform pairs (no self-loops, none in ``exclude_sorted``), as keys.

    For undirected draws the key is (min, max) and the exclusion set holds (min, max) keys.
    """
    out = torch.empty(0, dtype=torch.int64, device=device)
    start = 0
    need = count
    while need > 0:
        k = int(need * 1.25) + 64
        r1 = draws(seed, stream, start, k, device)
        r2 = draws(seed, stream + 1, start, k, device)
        start += k
        s = below(r1, n)
        d = below(r2, n)
        ok = s != d
        s, d = s[ok], d[ok]
        if undirected:
            s, d = torch.minimum(s, d), torch.maximum(s, d)
        cand = key_of(s, d)
        if exclude_sorted is not None:
            cand = cand[~is_member(exclude_sorted, cand)]
        if out.numel():
            cand = cand[~torch.isin(cand, out)]
        cand = first_unique(cand)[:need]
        out = torch.cat([out, cand])
        need = count - out.numel()
    return out


def er_graph(n: int, m: int, seed: int, wmax: int = 100, device="cpu") -> EdgeList:
    """Erdos-Renyi-style digraph: ``m`` distinct uniform arcs, no self-loops."""
    keys = _fresh_pairs(n, m, seed, 10, device)
    s, d = split_key(keys)
    return EdgeList(n, s, d, arc_weight(s, d, wmax, seed), False, wmax, seed)


def rmat_graph(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19,
               wmax: int = 100, device="cpu", shuffle: bool = True) -> EdgeList:
    """R-MAT digraph (Chakrabarti, Zhan and Faloutsos, SDM 2004) on 2**scale vertices.

    ``2**scale * edge_factor`` arcs are drawn; each picks one quadrant per level with
    probabilities (a, b, c, 1-a-b-c); vertex ids are then relabelled by a seeded
    permutation (as the Graph500 generator does), self-loops are dropped and duplicate
    arcs merged.  The surviving arcs are returned in a seeded random order.
    """
    n = 1 << scale
    m0 = n * edge_factor
    ta = int(a * 2**32)
    tab = int((a + b) * 2**32)
    tabc = int((a + b + c) * 2**32)
    src = torch.zeros(m0, dtype=torch.int64, device=device)
    dst = torch.zeros(m0, dtype=torch.int64, device=device)
    for lv in range(0, scale, 2):
        r = draws(seed, 100 + lv, 0, m0, device)
        for half in range(2):
            level = lv + half
            if level >= scale:
                break
            u = _srl(r, 32) if half == 0 else torch.bitwise_and(r, 0xFFFFFFFF)
            sbit = (u >= tab).to(torch.int64)
            dbit = (((u >= ta) & (u < tab)) | (u >= tabc)).to(torch.int64)
            src = torch.bitwise_or(src, torch.bitwise_left_shift(sbit, level))
            dst = torch.bitwise_or(dst, torch.bitwise_left_shift(dbit, level))
        del r
    perm = torch.argsort(draws(seed, 90, 0, n, device), stable=True)
    src = perm[src]
    dst = perm[dst]
    keep = src != dst
    keys = torch.unique(key_of(src[keep], dst[keep]), sorted=True)
    del src, dst, keep
    if shuffle:
        keys = shuffled(keys, seed, 91)
    s, d = split_key(keys)
    return EdgeList(n, s, d, arc_weight(s, d, wmax, seed), False, wmax, seed)


def grid_graph(side: int, seed: int, remove_frac=0.10, shortcut_frac=0.01, wmax=1000,
               device="cpu") -> EdgeList:
    """Road-network-like undirected graph, returned as both arcs of every edge.

    A ``side`` x ``side`` 4-neighbour grid (id = row * side + col); exactly
    ``round(remove_frac * E)`` of its E edges are removed at random, then
    ``round(shortcut_frac * kept)`` distinct uniform long-range shortcut edges are added.
    Both arcs of an edge carry the same weight in [1, wmax].
    """
    n = side * side
    r = torch.arange(side, device=device, dtype=torch.int64)
    rr, cc = torch.meshgrid(r, r, indexing="ij")
    vid = rr * side + cc
    h = torch.stack([vid[:, :-1].reshape(-1), vid[:, 1:].reshape(-1)], 1)
    v = torch.stack([vid[:-1, :].reshape(-1), vid[1:, :].reshape(-1)], 1)
    e = torch.cat([h, v])
    n_edges = e.shape[0]
    n_remove = int(round(remove_frac * n_edges))
    order = torch.argsort(draws(seed, 200, 0, n_edges, device), stable=True)
    e = e[order[n_remove:]]
    ukeys = key_of(torch.minimum(e[:, 0], e[:, 1]), torch.maximum(e[:, 0], e[:, 1]))
    ukeys_sorted = torch.sort(ukeys).values
    n_short = int(round(shortcut_frac * ukeys.numel()))
    sc = _fresh_pairs(n, n_short, seed, 210, device, exclude_sorted=ukeys_sorted, undirected=True)
    ukeys = torch.cat([ukeys, sc])
    us, ud = split_key(ukeys)
    src = torch.cat([us, ud])
    dst = torch.cat([ud, us])
    keys = shuffled(key_of(src, dst), seed, 220)
    s, d = split_key(keys)
    return EdgeList(n, s, d, arc_weight(s, d, wmax, seed, undirected=True), True, wmax, seed)


class Workload:
    """Evolving arc set of a graph, producing seeded insert/delete/query batches.

    Inserts are new arcs with uniform endpoints (for undirected graphs: new unordered
    pairs, returned as both arcs); deletes are drawn uniformly from the arcs present at
    that moment (undirected: present unordered pairs, both arcs); queries are half drawn
    from the present arcs and half absent uniform pairs.  The set is advanced as if each
    batch were applied, which is what the graph under test is expected to do.
    """

    def __init__(self, g: EdgeList, seed: int):
        self.g = g
        self.seed = seed
        self.step = 0
        k = g.keys()
        if g.undirected:
            s, d = split_key(k)
            k = key_of(s[s < d], d[s < d])
        self.keys = torch.sort(k).values  # arcs, or (min,max) pairs when undirected

    def _arcs(self, keys: torch.Tensor):
        s, d = split_key(keys)
        if self.g.undirected:
            s, d = torch.cat([s, d]), torch.cat([d, s])
        w = arc_weight(s, d, self.g.wmax, self.g.wseed, self.g.undirected)
        return s, d, w

    def insert_batch(self, count: int):
        """``count`` new arcs (undirected: ``count`` new edges = 2*count arcs)."""
        self.step += 1
        new = _fresh_pairs(self.g.n, count, self.seed, 1000 + 10 * self.step, self.keys.device,
                           exclude_sorted=self.keys, undirected=self.g.undirected)
        self.keys = torch.sort(torch.cat([self.keys, new])).values
        return self._arcs(new)

    def delete_batch(self, count: int):
        """``count`` arcs (undirected: edges) drawn without replacement from the present set."""
        self.step += 1
        count = min(count, self.keys.numel())
        idx = torch.argsort(draws(self.seed, 1000 + 10 * self.step, 0, self.keys.numel(),
                                  self.keys.device), stable=True)[:count]
        gone = self.keys[idx]
        keep = torch.ones(self.keys.numel(), dtype=torch.bool, device=self.keys.device)
        keep[idx] = False
        self.keys = self.keys[keep]
        s, d, _ = self._arcs(gone)
        return s, d

    def query_batch(self, count: int, present_frac: float = 0.5):
        """``count`` arc queries: ``round(count*present_frac)`` present arcs, the rest absent."""
        self.step += 1
        n_in = int(round(count * present_frac))
        dev = self.keys.device
        r = draws(self.seed, 1000 + 10 * self.step, 0, n_in, dev)
        pick = self.keys[below(r, self.keys.numel())] if self.keys.numel() else self.keys[:0]
        ps, pd = split_key(pick)
        if self.g.undirected:  # either orientation of a present edge is a present arc
            flip = torch.bitwise_and(_srl(r, 7), 1) == 1
            ps, pd = torch.where(flip, pd, ps), torch.where(flip, ps, pd)
        absent = _fresh_pairs(self.g.n, count - n_in, self.seed, 1000 + 10 * self.step + 3, dev,
                              exclude_sorted=self.keys, undirected=self.g.undirected)
        as_, ad = split_key(absent)
        s = torch.cat([ps, as_])
        d = torch.cat([pd, ad])
        order = torch.argsort(draws(self.seed, 1000 + 10 * self.step + 5, 0, s.numel(), dev),
                              stable=True)
        return s[order], d[order]

    def present_arcs(self) -> torch.Tensor:
        """All present arcs as keys (undirected: both orientations), ascending."""
        if not self.g.undirected:
            return self.keys
        s, d = split_key(self.keys)
        return torch.sort(torch.cat([key_of(s, d), key_of(d, s)])).values


def max_out_degree_vertex(g: EdgeList) -> int:
    """Vertex of largest out-degree (smallest id on ties): the traversal source used for
    the power-law workloads, where vertex 0 may be isolated after relabelling."""
    deg = torch.bincount(g.src, minlength=g.n)
    mx = deg.max()
    return int(torch.nonzero(deg == mx)[0, 0])


# Named workload shapes (the five configurations the measurements are quoted on).
def er_4k(seed=0x4D45524B, device="cpu") -> EdgeList:
    return er_graph(4096, 32768, seed, 100, device)


def rmat_s(scale: int, seed=0x4D45524B + 1, device="cpu") -> EdgeList:
    return rmat_graph(scale, 16, seed, wmax=100, device=device)


def grid_side(side: int, seed=0x4D45524B + 2, device="cpu") -> EdgeList:
    return grid_graph(side, seed, device=device)
