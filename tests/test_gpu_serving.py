"""GPU tests of the serving loop: captured query graphs replay correctly, and every result
of a concurrent, continuously batched run equals the same request run alone in sequence
order (integers exact, PageRank within 1e-6 in L1)."""
import numpy as np
import pytest
import torch

from paper_2305_17813_amd import costmodel as CM
from paper_2305_17813_amd import inputs as I
from paper_2305_17813_amd import native
from paper_2305_17813_amd import serving as S
from parity import PR_L1_TOL, say, u32

pytestmark = pytest.mark.gpu


def test_query_graph_replays_match_eager():
    say("case: captured query graph replays")
    g = I.rmat_s(12)
    G = native.Graph(g.n, g.src, g.dst, g.w)
    streams = [torch.cuda.Stream()]
    qg = S.QueryGraphs(G, streams, min_log2=10, max_log2=13)
    wl = I.Workload(g, 4)
    for rep in range(4):
        qs, qd = wl.query_batch(700 + 900 * rep)
        qs, qd = native.as_u32(qs, G.device), native.as_u32(qd, G.device)
        with torch.cuda.stream(streams[0]):
            f, w = qg.run(0, qs, qd, streams[0])
        streams[0].synchronize()
        fe, we = G.query_edges(qs, qd)  # eager, on the graph's stream
        torch.cuda.synchronize()
        assert torch.equal(f, fe) and torch.equal(w, we)
        s, d, ww = wl.insert_batch(500)  # eager work between replays changes the graph
        G.insert_edges(s, d, ww)
        torch.cuda.synchronize()


def _compare(reqs, alone):
    for r in reqs:
        a = alone[r.rid]
        if r.kind in ("insert", "delete"):
            if r.rejected:
                continue
            assert torch.equal(r.result, a), f"{r.kind} statuses differ (request {r.rid})"
        elif r.kind == "query":
            assert torch.equal(r.result[0], a[0]) and torch.equal(r.result[1], a[1])
        elif r.kind == "pagerank":
            l1 = float((r.result[0].double() - a[0].double()).abs().sum())
            assert l1 <= PR_L1_TOL, l1
        elif r.result[1] is None:  # a BFS / SSSP from an untracked source answers distances
            assert r.kind in ("bfs", "sssp") and torch.equal(r.result[0], a[0])
        else:
            assert torch.equal(r.result[0], a[0]) and torch.equal(r.result[1], a[1]), r.kind


def _serve(cost_model, realtime, seed):
    g = I.rmat_s(12)
    tracked = I.max_out_degree_vertex(g)
    G = native.Graph(g.n, g.src, g.dst, g.w)
    reqs = S.make_requests(g, I.Workload(g, seed), 160, rate=4000.0, seed=seed, tracked=tracked,
                           upd_median=300, upd_clip=(20, 4000), q_median=2000, q_clip=(10, 20000))
    srv = S.Server(G, tracked, n_slots=4, cost_model=cost_model, keep_results=True)
    st = srv.run(reqs, realtime=realtime)
    srv.close()
    say(f"  served {len(reqs)}: {st.summary()}")
    G2 = native.Graph(g.n, g.src, g.dst, g.w)
    alone = S.run_alone(G2, reqs, tracked)
    _compare(reqs, alone)
    return st


def test_mixed_run_equals_alone_burst():
    say("case: serving, burst arrivals")
    st = _serve(None, realtime=False, seed=31)
    assert st.merged_batches > 0


def test_mixed_run_equals_alone_poisson_with_cost_model():
    say("case: serving, Poisson arrivals, learned cost model")
    g = I.rmat_s(12)
    G = native.Graph(g.n, g.src, g.dst, g.w)
    rec = CM.generate_records(G, I.Workload(g, 40), I.max_out_degree_vertex(g), 30, 20, 3000, seed=4,
                              algos=["bfs", "sssp", "pagerank"])
    cm, hist, r = CM.fit(rec, epochs=150)
    st = _serve(cm, realtime=True, seed=32)
    assert st.summary()["p99_ms"] is not None


def test_mixed_run_compacts_when_the_pool_runs_low():
    """A pool with little headroom: before rejecting an insert the server reclaims slabs
    (compaction, with no read in flight); every admitted request still equals its result
    alone."""
    say("case: serving with a tight pool")
    g = I.rmat_s(12)
    tracked = I.max_out_degree_vertex(g)
    probe = native.Graph(g.n, g.src, g.dst, g.w)
    used = max(probe.stats()["pool_used"])
    del probe
    G = native.Graph(g.n, g.src, g.dst, g.w, pool_slabs=used + 3000)
    reqs = S.make_requests(g, I.Workload(g, 33), 160, rate=4000.0, seed=33, tracked=tracked,
                           upd_median=600, upd_clip=(20, 4000), q_median=2000, q_clip=(10, 20000))
    srv = S.Server(G, tracked, n_slots=4, keep_results=True)
    st = srv.run(reqs, realtime=False)
    srv.close()
    say(f"  compactions {srv.compactions}, rejected {st.rejected}: {st.summary()['p99_ms']}")
    assert srv.compactions >= 1
    G2 = native.Graph(g.n, g.src, g.dst, g.w)
    alone = S.run_alone(G2, reqs, tracked)
    _compare(reqs, alone)
