"""Full-size GPU parity: the stated workload sizes, in the launch configuration bench.py times.

R-MAT scale 22 (4,194,304 vertices, 65.2M arcs, all three views, load factor 0.7) with 1M-arc
insert and delete batches and 1M queries; and the 4096 x 4096 road-like grid (16.8M vertices,
61M arcs) with 100K-edge batches.  The oracle computes every output in full (it finishes each
algorithm in seconds at these sizes), so the comparison is element by element.
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


def _cmp_traversals(G, O, src, with_pr=True, with_tc=True, state=None):
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
    if state is not None:  # the UpdateIterator scheme on a graph of its own, kept in step
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
    if with_tc:
        t = time.time()
        tg = int(G.triangles().item())
        to = O.triangles()
        say(f"  triangles {tg} vs {to} ({time.time()-t:.1f}s)")
        assert tg == to


def test_rmat_scale22_batches_of_1m():
    say("case: R-MAT scale 22, 1M-arc batches (bench configuration)")
    g = I.rmat_graph(22, 16, 0x4D45524B + 1, device="cuda")
    src = I.max_out_degree_vertex(g)
    G, O = _pair(g, src, log_capacity=1 << 22)
    state = {"wcc_graph": native.Graph(g.n, g.src, g.dst, g.w, views=native.VIEW_FWD, load_factor=0.7,
                                       log_capacity=1 << 22)}
    # the oracle's triangle count takes ~2 minutes here: the GPU count is compared once, at
    # the end, where it has gone through the static count and both incremental updates
    G.triangles()
    _cmp_traversals(G, O, src, state=state, with_tc=False)
    wl = I.Workload(g, 0x4D45524B + 8)
    B = 1_000_000
    s, d, w = wl.insert_batch(B)
    st = u32(G.insert_edges(s, d, w))
    assert np.array_equal(st, O.insert(u32(s), u32(d), u32(w)).astype(np.uint32))
    state["wcc_graph"].insert_edges(s, d, w, status=False)
    say("  insert statuses equal")
    G.triangles()
    _cmp_traversals(G, O, src, state=state, with_tc=False)
    s, d = wl.delete_batch(B)
    st = u32(G.delete_edges(s, d))
    assert np.array_equal(st, O.delete(u32(s), u32(d)).astype(np.uint32))
    state["wcc_graph"].delete_edges(s, d, status=False)
    say("  delete statuses equal")
    _cmp_traversals(G, O, src, state=state)
    qs, qd = wl.query_batch(1 << 20)
    f, qw = G.query_edges(qs, qd)
    fo, wo = O.query(u32(qs), u32(qd))
    assert np.array_equal(u32(f), fo.astype(np.uint32)) and np.array_equal(u32(qw), wo)
    say("  queries equal")
    assert G.check() == 0


def test_road_grid_4096_batches_of_100k():
    say("case: 4096 x 4096 road-like grid, 100K-edge batches")
    g = I.grid_graph(4096, 0x4D45524B + 2, device="cuda")
    G, O = _pair(g, 0, log_capacity=1 << 21)
    _cmp_traversals(G, O, 0, with_pr=False, with_tc=False)
    wl = I.Workload(g, 0x4D45524B + 9)
    s, d, w = wl.insert_batch(100_000)
    st = u32(G.insert_edges(s, d, w))
    assert np.array_equal(st, O.insert(u32(s), u32(d), u32(w)).astype(np.uint32))
    _cmp_traversals(G, O, 0, with_pr=False, with_tc=False)
    s, d = wl.delete_batch(100_000)
    st = u32(G.delete_edges(s, d))
    assert np.array_equal(st, O.delete(u32(s), u32(d)).astype(np.uint32))
    _cmp_traversals(G, O, 0, with_pr=False, with_tc=False)
    assert G.check() == 0
