"""Host logic of the serving loop (no GPU): the seeded request stream, the disjointness test
that decides whether update requests merge, and the latency summary."""
import numpy as np
import torch

from paper_2305_17813_amd import inputs as I
from paper_2305_17813_amd import serving as S


def _stream(n=400, seed=5):
    g = I.er_graph(2048, 16384, 3)
    return g, S.make_requests(g, I.Workload(g, seed), n, rate=1000.0, seed=seed, tracked=7,
                              upd_median=50, upd_clip=(10, 400), q_median=100, q_clip=(10, 800),
                              device="cpu")


def test_request_stream_mix_sizes_and_arrivals():
    g, reqs = _stream()
    kinds = [r.kind for r in reqs]
    n = len(reqs)
    upd = sum(k in ("insert", "delete") for k in kinds) / n
    qry = sum(k == "query" for k in kinds) / n
    assert abs(upd - 0.4) < 0.08 and abs(qry - 0.4) < 0.08
    arr = np.array([r.arrival for r in reqs])
    assert (np.diff(arr) >= 0).all() and arr[-1] > 0
    for r in reqs:
        if r.kind in ("insert", "delete"):
            assert 10 <= r.size <= 400 and r.src.dtype == torch.int32
            assert (r.w is not None) == (r.kind == "insert")
        elif r.kind == "query":
            assert 10 <= r.size <= 800
        else:
            assert 0 <= r.source < g.n and r.size == 0
    tracked = [r for r in reqs if r.kind in ("bfs", "sssp", "pagerank")]
    assert 0.25 < np.mean([r.source == 7 for r in tracked]) < 0.75


def test_request_stream_is_seeded():
    _, a = _stream(seed=9)
    _, b = _stream(seed=9)
    assert [r.kind for r in a] == [r.kind for r in b]
    assert all(torch.equal(x.src, y.src) for x, y in zip(a, b) if x.src is not None)


def test_disjoint_decides_merging():
    mk = lambda s, d: S.Request(0, "insert", 0.0, torch.tensor(s, dtype=torch.int32),
                                torch.tensor(d, dtype=torch.int32))
    assert S.Server._disjoint(None, [mk([1, 2], [3, 4]), mk([1, 5], [4, 3])])
    assert not S.Server._disjoint(None, [mk([1, 2], [3, 4]), mk([2], [4])])
    assert not S.Server._disjoint(None, [mk([1, 1], [3, 3])])  # a duplicate inside one request
    big = -1  # the bit pattern of id 0xFFFFFFFF stays distinct from small ids
    assert S.Server._disjoint(None, [mk([big], [0]), mk([0], [big])])


def test_summary_percentiles_and_rates():
    st = S.ServeStats()
    st.latencies = {"query": [0.001] * 99 + [0.1], "insert": [0.002]}
    st.update_ops, st.query_ops, st.wall_s = 300, 5000, 2.0
    s = st.summary()
    assert s["requests"] == 101 and s["updates_per_s"] == 150.0 and s["queries_per_s"] == 2500.0
    assert abs(s["per_kind"]["query"]["p50_ms"] - 1.0) < 1e-9
    assert s["per_kind"]["insert"]["p99_ms"] == 2.0
