"""GPU tests of the serving loop: captured query graphs replay correctly, and every result
of a concurrent, continuously batched run equals the oracle's answer on the graph after all
earlier-sequenced updates, and the same request run alone in sequence order (integers
exact, PageRank within 1e-6 in L1)."""
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


def _compare_with_oracle(g, reqs, tracked):
    """Replay the admitted requests in sequence order on the oracle: every update is applied
    to it, and every read must equal the oracle's answer on the graph after all updates
    with smaller sequence numbers (statuses, found flags, weights, levels, distances and
    parents exact; PageRank within 1e-6 in L1 of the oracle's fixed point)."""
    import oracle
    O = oracle.OracleGraph(g.n, u32(g.src), u32(g.dst), u32(g.w))
    counts = {}
    for r in sorted(reqs, key=lambda r: r.seq):
        counts[r.kind] = counts.get(r.kind, 0) + 1
        if r.kind == "insert":
            if r.rejected:
                continue
            so = O.insert(u32(r.src), u32(r.dst), u32(r.w)).astype(np.uint32)
            assert np.array_equal(u32(r.result), so), f"insert statuses differ (request {r.rid})"
        elif r.kind == "delete":
            so = O.delete(u32(r.src), u32(r.dst)).astype(np.uint32)
            assert np.array_equal(u32(r.result), so), f"delete statuses differ (request {r.rid})"
        elif r.kind == "query":
            fo, wo = O.query(u32(r.src), u32(r.dst))
            assert np.array_equal(u32(r.result[0]), fo.astype(np.uint32)), f"query {r.rid}"
            assert np.array_equal(u32(r.result[1]), wo), f"query weights {r.rid}"
        elif r.kind == "pagerank":
            ro, _ = O.pagerank()
            l1 = float(np.abs(r.result[0].double().cpu().numpy() - ro).sum())
            assert l1 <= PR_L1_TOL, (r.rid, l1)
        else:
            do, po = O.bfs(r.source) if r.kind == "bfs" else O.sssp(r.source)
            assert np.array_equal(u32(r.result[0]), do), f"{r.kind} {r.rid} from {r.source}"
            if r.result[1] is not None:
                assert np.array_equal(u32(r.result[1]), po), f"{r.kind} parents {r.rid}"
    say(f"  every served result equals the oracle's: {counts}")


def _serve(cost_model, realtime, seed, scale=12, n_req=160):
    g = I.rmat_s(scale)
    tracked = I.max_out_degree_vertex(g)
    G = native.Graph(g.n, g.src, g.dst, g.w)
    reqs = S.make_requests(g, I.Workload(g, seed), n_req, rate=4000.0, seed=seed, tracked=tracked,
                           upd_median=300, upd_clip=(20, 4000), q_median=2000, q_clip=(10, 20000))
    srv = S.Server(G, tracked, n_slots=4, cost_model=cost_model, keep_results=True)
    st = srv.run(reqs, realtime=realtime)
    srv.close()
    say(f"  served {len(reqs)}: {st.summary()}")
    _compare_with_oracle(g, reqs, tracked)
    G2 = native.Graph(g.n, g.src, g.dst, g.w)
    alone = S.run_alone(G2, reqs, tracked)
    _compare(reqs, alone)
    return st


def test_mixed_run_equals_alone_burst():
    say("case: serving, burst arrivals")
    st = _serve(None, realtime=False, seed=31)
    assert st.merged_batches > 0


def test_served_results_equal_the_oracle_at_scale_16():
    """A larger resident graph (R-MAT scale 16, 65K vertices, 1M arcs) with the same stream
    shape: every served result against the oracle, and against the same request alone."""
    say("case: serving, burst arrivals, R-MAT scale 16")
    st = _serve(None, realtime=False, seed=34, scale=16, n_req=120)
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
    _compare_with_oracle(g, reqs, tracked)
    G2 = native.Graph(g.n, g.src, g.dst, g.w)
    alone = S.run_alone(G2, reqs, tracked)
    _compare(reqs, alone)
