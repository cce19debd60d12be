"""Full-size GPU parity: the stated workload sizes, in the launch configuration bench.py times.

R-MAT scale 22 (4,194,304 vertices, 65.2M arcs, all three views, load factor 0.7) with insert
and delete batches of 1M, 100K and 10K arcs and 1M queries; and the 4096 x 4096 road-like grid
(16.8M vertices, 61M arcs) with batches of 100K, 10K and 1K edges.  The oracle computes every
output in full (each algorithm finishes in seconds at these sizes), so the comparison is
element by element after every batch.  The triangle count is compared after every batch too:
the oracle counts the graph once in full, then adds the triangles that touch the undirected
edges a batch created, or subtracts those touching the edges it removed (counted on the graph
before the batch).
"""
import time

import numpy as np
import pytest
import torch

from paper_2305_17813_amd import inputs as I
from paper_2305_17813_amd import native
from parity import PR_L1_TOL, say, u32

pytestmark = [pytest.mark.gpu, pytest.mark.fullsize]


def _pair(g, source, log_capacity):
    import oracle
    t = time.time()
    G = native.Graph(g.n, g.src, g.dst, g.w, views=7, load_factor=0.7, log_capacity=log_capacity)
    torch.cuda.synchronize()
    say(f"  HIP graph built in {time.time()-t:.1f}s")
    t = time.time()
    O = oracle.OracleGraph(g.n, u32(g.src), u32(g.dst), u32(g.w))
    say(f"  oracle loaded in {time.time()-t:.1f}s")
    return G, O


def _cmp_traversals(G, O, src, with_pr=True, state=None):
    t = time.time()
    lv, pa = G.bfs(src)
    lo, po = O.bfs(src)
    assert np.array_equal(u32(lv), lo) and np.array_equal(u32(pa), po), "BFS differs"
    lvd, bu = G.bfs_levels(src)
    assert np.array_equal(u32(lvd), lo), "distance-only BFS levels differ"
    di, pa = G.sssp(src)
    do, po = O.sssp(src)
    assert np.array_equal(u32(di), do), f"SSSP distances differ at {np.nonzero(u32(di) != do)[0][:8]}"
    assert np.array_equal(u32(pa), po), "SSSP parents differ"
    lab = G.wcc()
    lo_w = O.wcc()
    assert np.array_equal(u32(lab), lo_w), "WCC differs"
    if state is not None and "wcc_graph" in state:  # the UpdateIterator scheme, kept in step
        assert np.array_equal(u32(state["wcc_graph"].wcc(scheme=native.WCC_UPDATE)), lo_w), \
            "WCC (UpdateIterator scheme) differs"
    say(f"  BFS/SSSP/WCC equal, distance-only BFS took {bu} bottom-up steps ({time.time()-t:.1f}s)")
    if with_pr:
        t = time.time()
        r, it = G.pagerank()
        warm = None if state is None else state.get("pr")
        ro, oit = O.pagerank(tol=1e-11, max_iter=2000, warm=warm)
        if state is not None:
            state["pr"] = ro
        l1 = float(np.abs(r.double().cpu().numpy() - ro).sum())
        say(f"  PageRank L1 {l1:.2e} ({int(it.item())} GPU iterations, {oit} oracle, {time.time()-t:.1f}s)")
        assert l1 <= PR_L1_TOL


def _keys(s, d):
    return (s.astype(np.uint64) << np.uint64(32)) | d.astype(np.uint64)


def _insert_step(G, O, s, d, w, tri=None, state=None):
    """Insert a batch on both sides; statuses must agree.  With `tri` (the count before the
    batch) the GPU count after it must equal tri + the triangles touching the new undirected
    edges; returns the new count."""
    s_, d_, w_ = u32(s), u32(d), u32(w)
    rev_before = O.query(d_, s_)[0] if tri is not None else None
    st = u32(G.insert_edges(s, d, w))
    assert np.array_equal(st, O.insert(s_, d_, w_).astype(np.uint32)), "insert statuses differ"
    if state is not None and "wcc_graph" in state:
        state["wcc_graph"].insert_edges(s, d, w, status=False)
    if tri is None:
        return None
    t = time.time()
    new = (st == 1) & (rev_before == 0)  # {s, d} was no undirected edge before the batch
    tri += O.triangles_touching(s_[new], d_[new])
    tg = int(G.triangles().item())
    say(f"  triangles after the insert batch {tg} vs {tri} ({time.time()-t:.1f}s)")
    assert tg == tri
    return tri


def _delete_step(G, O, s, d, tri=None, state=None):
    """Delete a batch on both sides; statuses must agree.  With `tri`, the GPU count after it
    must equal tri - the triangles (of the graph before the batch) touching the undirected
    edges the batch removes: {s, d} goes when (s, d) is present and deleted, and (d, s) is
    absent before the batch or deleted by it too."""
    s_, d_ = u32(s), u32(d)
    removed = None
    if tri is not None:
        t = time.time()
        present = O.query(s_, d_)[0] == 1
        rev_present = O.query(d_, s_)[0] == 1
        rev_deleted = np.isin(_keys(d_, s_), _keys(s_, d_))
        gone = present & (~rev_present | rev_deleted)
        removed = O.triangles_touching(s_[gone], d_[gone])
        say(f"  triangles the delete batch removes: {removed} ({time.time()-t:.1f}s)")
    st = u32(G.delete_edges(s, d))
    assert np.array_equal(st, O.delete(s_, d_).astype(np.uint32)), "delete statuses differ"
    if state is not None and "wcc_graph" in state:
        state["wcc_graph"].delete_edges(s, d, status=False)
    if tri is None:
        return None
    tri -= removed
    tg = int(G.triangles().item())
    say(f"  triangles after the delete batch {tg} vs {tri}")
    assert tg == tri
    return tri


def test_rmat_scale22_batches_of_1m_100k_10k():
    say("case: R-MAT scale 22, batches of 1M, 100K and 10K arcs (bench configuration)")
    g = I.rmat_graph(22, 16, 0x4D45524B + 1, device="cuda")
    src = I.max_out_degree_vertex(g)
    G, O = _pair(g, src, log_capacity=1 << 22)
    state = {"wcc_graph": native.Graph(g.n, g.src, g.dst, g.w, views=native.VIEW_FWD, load_factor=0.7,
                                       log_capacity=1 << 22)}
    t = time.time()
    tri = O.triangles()
    tg = int(G.triangles().item())
    say(f"  static triangles {tg} vs {tri} ({time.time()-t:.1f}s)")
    assert tg == tri
    _cmp_traversals(G, O, src, state=state)
    wl = I.Workload(g, 0x4D45524B + 8)
    for B in (1_000_000, 100_000, 10_000):
        say(f"  batch of {B} arcs")
        tri = _insert_step(G, O, *wl.insert_batch(B), tri=tri, state=state)
        _cmp_traversals(G, O, src, state=state)
        tri = _delete_step(G, O, *wl.delete_batch(B), tri=tri, state=state)
        _cmp_traversals(G, O, src, state=state)
    qs, qd = wl.query_batch(1 << 20)
    f, qw = G.query_edges(qs, qd)
    fo, wo = O.query(u32(qs), u32(qd))
    assert np.array_equal(u32(f), fo.astype(np.uint32)) and np.array_equal(u32(qw), wo)
    say("  queries equal")
    assert G.check() == 0


def test_road_grid_4096_batches_of_100k_10k_1k():
    say("case: 4096 x 4096 road-like grid, batches of 100K, 10K and 1K edges")
    g = I.grid_graph(4096, 0x4D45524B + 2, device="cuda")
    G, O = _pair(g, 0, log_capacity=1 << 21)
    _cmp_traversals(G, O, 0, with_pr=False)
    wl = I.Workload(g, 0x4D45524B + 9)
    for B in (100_000, 10_000, 1_000):
        say(f"  batch of {B} edges ({2 * B} arcs)")
        _insert_step(G, O, *wl.insert_batch(B))
        _cmp_traversals(G, O, 0, with_pr=False)
        _delete_step(G, O, *wl.delete_batch(B))
        _cmp_traversals(G, O, 0, with_pr=False)
    assert G.check() == 0
