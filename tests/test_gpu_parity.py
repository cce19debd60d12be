"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, element by element.

Integers (statuses, membership, weights, BFS levels, SSSP distances, parents, component
labels, triangle counts) must be bit-exact; PageRank must be within 1e-6 in L1.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2305_17813_amd import inputs as I
from paper_2305_17813_amd import native
from parity import PR_L1_TOL, Pair, say, u32

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _lib():
    native.load()


def make_pair(g: I.EdgeList, source=0, **kw):
    return Pair(g.n, g.src, g.dst, g.w, source=source, **kw)


def test_er_4096_end_to_end():
    """ER digraph 4,096 / 32,768: insert 1,024, delete 1,024, 4,096 queries; BFS and SSSP
    from vertex 0 (and WCC, PageRank, triangles) after each batch."""
    say("case: ER 4096 end to end")
    g = I.er_4k()
    p = make_pair(g, source=0)
    p.check_structure()
    p.check_all()
    wl = I.Workload(g, 11)
    s, d, w = wl.insert_batch(1024)
    st = p.insert(s, d, w)
    assert int((st == 1).sum()) == 1024
    p.check_all()
    s, d = wl.delete_batch(1024)
    st = p.delete(s, d)
    assert int((st == 1).sum()) == 1024
    p.check_all()
    qs, qd = wl.query_batch(4096)
    p.query(qs, qd)
    p.check_structure()


@pytest.mark.parametrize("scale", [10, 12])
def test_rmat_batches(scale):
    say(f"case: rmat scale {scale}")
    g = I.rmat_s(scale)
    src = I.max_out_degree_vertex(g)
    p = make_pair(g, source=src)
    p.check_all()
    wl = I.Workload(g, 5)
    for b in [100, 1000, 3000]:
        s, d, w = wl.insert_batch(b)
        p.insert(s, d, w)
        p.check_all()
        s, d = wl.delete_batch(b)
        p.delete(s, d)
        p.check_all()
    qs, qd = wl.query_batch(20000)
    p.query(qs, qd)
    p.check_structure()


def test_grid_road_like():
    say("case: grid 64x64")
    g = I.grid_side(64)
    p = make_pair(g, source=0)
    p.check_all()
    wl = I.Workload(g, 8)
    for b in [10, 100, 400]:
        s, d, w = wl.insert_batch(b)
        p.insert(s, d, w)
        p.check_all()
        s, d = wl.delete_batch(b)
        p.delete(s, d)
        p.check_all()
    p.check_structure()


def test_one_source_long_chains_and_reinsert():
    """Every op on one source (one chain of hundreds of slabs): contention on one tail,
    slab linking races, tombstones, delete then re-insert."""
    say("case: one source long chain")
    n = 6000
    p = Pair(n, [1], [2], [5], source=0)
    rng = np.random.default_rng(3)
    dst = rng.permutation(np.arange(1, n))[:5000]
    p.insert(np.zeros(5000, np.int64), dst, rng.integers(1, 100, 5000))
    p.check_structure()
    p.check_all(algos=("bfs", "sssp", "wcc", "tc"))
    p.delete(np.zeros(2500, np.int64), dst[::2])
    p.check_structure()
    p.insert(np.zeros(5000, np.int64), dst, np.full(5000, 7))  # half present, half re-inserted
    p.check_structure()
    p.query(np.zeros(n, np.int64), np.arange(n))
    p.check_all(algos=("bfs", "sssp", "wcc", "tc"))


def test_in_batch_duplicates_exactly_one_applies():
    say("case: in-batch duplicates")
    g = I.er_graph(512, 2000, 77)
    p = make_pair(g)
    rng = np.random.default_rng(4)
    s = rng.integers(0, 512, 3000)
    d = rng.integers(0, 512, 3000)
    s = np.concatenate([s, s, s, s])
    d = np.concatenate([d, d, d, d])
    w = np.full(s.size, 9)
    p.insert(s, d, w, exact_status=False)
    p.check_structure()
    p.delete(s, d, exact_status=False)
    p.check_structure()
    p.check_all()


def test_rejections_and_queries_of_invalid_ids():
    say("case: rejections")
    p = Pair(100, [0, 1], [1, 2], [3, 4])
    s = [0, 5, 100, 0xFFFFFFFD, 7, 3]
    d = [0, 101, 3, 4, 0xFFFFFFFE, 4]
    st = p.insert(s, d, [1] * 6)
    assert list(st) == [2, 2, 2, 2, 2, 1]
    p.query(s, d)
    st = p.delete(s, d)
    assert list(st) == [2, 2, 2, 2, 2, 1]


def test_out_of_slabs_is_clean():
    """A tiny pool makes the pre-check refuse the batch; nothing is applied."""
    say("case: out of slabs")
    g = I.er_graph(256, 1000, 5)
    p = make_pair(g, pool_slabs=64)
    s = np.zeros(600, np.int64)
    d = np.arange(1, 601) % 256
    with pytest.raises(native.MkError) as e:
        p.g.insert_edges(s, d, np.ones(600))
    assert e.value.status == 2
    p.check_structure()  # still equal to the oracle, which saw nothing


def test_initial_arcs_that_overflow_an_explicit_pool_are_refused():
    """With hashing off every vertex has one chain; a star of 199 arcs needs 13 chained
    slabs, more than an explicit pool of 2 holds.  The insert lanes that find the pool empty
    raise the overflow bit, and creation returns MK_ERR_OUT_OF_SLABS instead of a graph that
    silently lost arcs.  A pool with a slab per arc (lanes racing on the tail may each take
    one before the losers return theirs) builds the same star exactly."""
    say("case: initial arcs overflow an explicit pool")
    n = 200
    src = np.zeros(n - 1, np.int64)
    dst = np.arange(1, n)
    with pytest.raises(native.MkError) as e:
        native.Graph(n, src, dst, np.ones(n - 1), views=native.VIEW_FWD, load_factor=0.0, pool_slabs=2)
    assert e.value.status == 2
    p = Pair(n, src, dst, np.ones(n - 1), views=native.VIEW_FWD, load_factor=0.0, pool_slabs=256)
    p.check_structure()


def test_steady_state_inserts_do_not_wait_for_the_stream():
    """Inserts whose host-side slab bound runs short use the pool snapshots that earlier
    inserts left behind events instead of synchronizing: with a long kernel queued ahead
    of each insert, the stream is still busy when the insert call returns.  The graph then
    still equals the oracle."""
    say("case: inserts without stream synchronization")
    g = I.rmat_s(14)
    probe = native.Graph(g.n, g.src, g.dst, g.w)
    used = max(probe.stats()["pool_used"])
    del probe
    p = make_pair(g, pool_slabs=used + 200_000)
    wl = I.Workload(g, 12)
    batches = [tuple(native.as_u32(x, DEV) for x in wl.insert_batch(20_000)) for _ in range(30)]
    stream = p.g.stream
    waited = 0
    for s, d, w in batches:
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            torch.cuda._sleep(20_000_000)  # about 10 ms of spinning ahead of the insert
        st = p.g.insert_edges(s, d, w)
        waited += int(stream.query())
        so = p.o.insert(u32(s), u32(d), u32(w))
        assert np.array_equal(u32(st), so.astype(np.uint32))
    torch.cuda.synchronize()
    say(f"  inserts that found the stream drained: {waited} of {len(batches)}")
    assert waited <= 1
    p.check_structure()
    p.check_all()


def test_hashing_off_single_bucket():
    say("case: hashing off")
    g = I.rmat_s(10)
    p = make_pair(g, source=I.max_out_degree_vertex(g), load_factor=0.0)
    wl = I.Workload(g, 1)
    s, d, w = wl.insert_batch(500)
    p.insert(s, d, w)
    p.check_all()
    s, d = wl.delete_batch(500)
    p.delete(s, d)
    p.check_all()
    p.check_structure()


def test_several_pending_batches_then_one_call():
    say("case: several pending batches")
    g = I.rmat_s(11)
    p = make_pair(g, source=I.max_out_degree_vertex(g))
    p.check_all()
    wl = I.Workload(g, 2)
    for _ in range(3):  # same kind: combined incremental update
        s, d, w = wl.insert_batch(300)
        p.insert(s, d, w)
    p.check_all()
    for _ in range(3):
        s, d = wl.delete_batch(300)
        p.delete(s, d)
    p.check_all()
    s, d, w = wl.insert_batch(300)  # mixed kinds: recompute
    p.insert(s, d, w)
    s, d = wl.delete_batch(300)
    p.delete(s, d)
    p.check_all()


def test_recompute_and_incremental_agree_and_are_deterministic():
    say("case: modes and determinism")
    g = I.rmat_s(11)
    src = I.max_out_degree_vertex(g)
    outs = []
    for rep in range(2):
        p = make_pair(g, source=src)
        p.g.sssp(src)
        wl = I.Workload(g, 4)
        s, d, w = wl.insert_batch(700)
        p.insert(s, d, w)
        a = [u32(x) for x in p.g.sssp(src, native.INCR)]
        b = [u32(x) for x in p.g.sssp(src, native.RECOMPUTE)]
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
        outs.append(a + [u32(p.g.wcc()), u32(p.g.bfs(src)[0])])
    assert all(np.array_equal(x, y) for x, y in zip(outs[0], outs[1]))


def test_generators_identical_on_gpu_and_cpu():
    say("case: generator device equality")
    a = I.rmat_graph(10, 8, 123, device="cpu")
    b = I.rmat_graph(10, 8, 123, device=DEV)
    assert torch.equal(a.src, b.src.cpu()) and torch.equal(a.dst, b.dst.cpu())
    assert torch.equal(a.w, b.w.cpu())


def test_contended_inserts_on_few_tails():
    """2^18 inserts (a quarter of them copies of others) aimed at 256 single-bucket source
    vertices: thousands of lanes race on the same chain tails and slab links; every arc
    lands exactly once, and a third are then deleted."""
    say("case: contended inserts")
    n = 1 << 17
    rng = np.random.default_rng(11)
    k = 1 << 18
    src = rng.integers(0, 256, k)
    dst = rng.integers(256, n, k)
    dup = rng.integers(0, k, k // 4)
    src[: k // 4], dst[: k // 4] = src[dup], dst[dup]
    p = Pair(n, [0], [1], [1], pool_slabs=1 << 20)  # the pre-check assumes a slab per insert
    p.insert(src, dst, np.full(src.size, 3), exact_status=False)
    p.check_structure()
    p.delete(src[::3], dst[::3], exact_status=False)
    p.check_structure()


def test_pagerank_reports_max_iter():
    say("case: PageRank iteration cap")
    g = I.rmat_s(10)
    G = native.Graph(g.n, g.src, g.dst, g.w)
    r, it = G.pagerank(tol=0.0, max_iter=3, mode=native.RECOMPUTE)
    assert int(it.item()) == 3


def test_export_and_recreate_round_trip():
    """Checkpoint by export: a graph re-created from the export answers like the oracle."""
    say("case: export round trip")
    g = I.rmat_s(11)
    p = make_pair(g, source=I.max_out_degree_vertex(g))
    wl = I.Workload(g, 12)
    s, d, w = wl.insert_batch(2000)
    p.insert(s, d, w)
    s, d = wl.delete_batch(2000)
    p.delete(s, d)
    es, ed, ew = p.g.export()
    q = Pair(g.n, es, ed, ew, source=p.source)
    q.o = p.o  # the oracle already holds the same arc set
    q.check_structure()
    q.check_all()


@pytest.mark.parametrize("delta", [1, 37, 1 << 30])
def test_band_width_leaves_sssp_unchanged(delta):
    """The weighted epilogue's band width only changes the expansion order: distances and
    parents equal the oracle's for a width of 1 (one distance per band), a middling one
    and one wider than every distance (a single band), through inserts and deletes."""
    say(f"case: band width {delta}")
    for g, src in ((I.grid_side(64), 0), (I.rmat_s(11), None)):
        src = I.max_out_degree_vertex(g) if src is None else src
        p = make_pair(g, source=src, sssp_delta=delta)
        p.check_all(algos=("sssp", "bfs"))
        wl = I.Workload(g, 9)
        for b in (50, 600):
            s, d, w = wl.insert_batch(b)
            p.insert(s, d, w)
            p.check_all(algos=("sssp",))
            s, d = wl.delete_batch(b)
            p.delete(s, d)
            p.check_all(algos=("sssp",))
        dist, par = p.g.traverse_from(src, True, p.g.traversal_workspace())
        od, op = p.o.sssp(src)
        assert np.array_equal(u32(dist), np.asarray(od, np.uint32))
        assert np.array_equal(u32(par), np.asarray(op, np.uint32))


def test_compaction_keeps_the_graph_and_frees_slabs():
    """Delete churn leaves tombstones; compaction packs the chains and frees slabs, and the
    arc set, queries and every incremental algorithm still equal the oracle afterwards."""
    say("case: compaction after churn")
    g = I.rmat_s(11)
    p = make_pair(g, source=I.max_out_degree_vertex(g))
    wl = I.Workload(g, 21)
    for _ in range(3):
        s, d, w = wl.insert_batch(3000)
        p.insert(s, d, w)
        s, d = wl.delete_batch(3000)
        p.delete(s, d)
    p.check_all()  # the incremental state is now current
    used = sum(p.g.stats()["pool_used"])
    freed = p.g.compact()
    assert freed > 0 and sum(p.g.stats()["pool_used"]) == used - freed
    p.check_structure()
    qs, qd = wl.query_batch(5000)
    p.query(qs, qd)
    assert p.g.compact() == 0  # nothing left to reclaim
    for b in (2000, 500):
        s, d, w = wl.insert_batch(b)
        p.insert(s, d, w)
        p.check_structure()
        p.check_all()
        s, d = wl.delete_batch(b)
        p.delete(s, d)
        p.check_all()


def test_compaction_of_one_long_chain_and_reuse():
    """Hashing off: one source's chain of 200 slabs; after two thirds are deleted the chain
    shrinks to the slabs its live arcs need and re-inserts draw from the free list."""
    say("case: compaction of a long chain")
    n = 4000
    p = Pair(n, [1], [2], [5], source=0, load_factor=0.0)
    rng = np.random.default_rng(8)
    dst = rng.permutation(np.arange(1, n))[:3000]
    p.insert(np.zeros(3000, np.int64), dst, rng.integers(1, 100, 3000))
    p.delete(np.zeros(2000, np.int64), dst[:2000])
    freed = p.g.compact()
    assert freed >= 100, freed
    p.check_structure()
    p.query(np.zeros(n, np.int64), np.arange(n))
    p.insert(np.zeros(2000, np.int64), dst[:2000], np.full(2000, 4))
    p.check_structure()
    p.check_all(algos=("bfs", "sssp", "wcc", "tc"))


def test_compaction_lets_a_full_pool_take_more_inserts():
    """A pool sized for a few batches runs out under insert/delete churn on one source;
    after compaction the refused batch fits."""
    say("case: compaction of a full pool")
    n = 20000
    p = Pair(n, [1], [2], [5], source=0, views=native.VIEW_FWD | native.VIEW_REV, pool_slabs=600,
             load_factor=0.0)
    refused = None
    for r in range(40):
        dst = 1 + r * 300 + np.arange(300)
        try:
            p.g.insert_edges(np.zeros(300, np.int64), dst, np.full(300, 2))
        except native.MkError as e:
            assert e.status == 2
            refused = dst
            break
        p.o.insert(np.zeros(300, np.uint32), dst.astype(np.uint32), np.full(300, 2, np.uint32))
        p.delete(np.zeros(300, np.int64), dst)
    assert refused is not None, "the pool never filled"
    p.check_structure()
    say(f"  refused at round {r}: {p.g.stats()}")
    freed = p.g.compact()
    say(f"  freed {freed}: {p.g.stats()}")
    assert freed > 0
    p.insert(np.zeros(300, np.int64), refused, np.full(300, 2))
    p.check_structure()
    p.check_all(algos=("bfs", "sssp", "wcc"))


def test_degenerate_graphs_and_empty_batches():
    """One vertex; many vertices and no arc; an isolated source; empty batches (every
    algorithm unchanged); a complete digraph, whose triangle count is C(n, 3); a directed
    cycle, whose PageRank is uniform and whose BFS levels are distances along the cycle."""
    say("case: degenerate graphs")
    p = Pair(1, [], [], [], source=0)
    p.check_all()
    p = Pair(64, [], [], [], source=5)
    p.check_all()
    r, _ = p.g.pagerank()
    assert np.allclose(r.cpu().numpy(), 1 / 64, atol=1e-7)
    e = np.zeros(0, np.int64)
    p.insert(e, e, e)
    p.delete(e, e)
    f, w = p.g.query_edges(e, e)
    assert f.numel() == 0
    p.check_all()
    # complete digraph on 40 vertices
    n = 40
    s, d = np.nonzero(~np.eye(n, dtype=bool))
    p = Pair(n, s, d, (s * 7 + d) % 100 + 1, source=3)
    p.check_all()
    assert int(p.g.triangles().item()) == n * (n - 1) * (n - 2) // 6
    # directed cycle of 100
    n = 100
    s = np.arange(n)
    p = Pair(n, s, (s + 1) % n, np.ones(n), source=0)
    p.check_all()
    lv, _ = p.g.bfs(0)
    assert np.array_equal(u32(lv), np.arange(n, dtype=np.uint32))
    r, _ = p.g.pagerank()
    assert np.abs(r.double().cpu().numpy() - 1 / n).sum() <= PR_L1_TOL
    # a source without out-arcs on R-MAT: everything else unreachable
    g = I.rmat_s(10)
    deg = np.bincount(u32(g.src), minlength=g.n)
    p = make_pair(g, source=int(np.nonzero(deg == 0)[0][0]))
    p.check_all(algos=("bfs", "sssp"))


@pytest.mark.parametrize("b", [1, 63, 65, 255, 257, 4097])
def test_ragged_batch_sizes(b):
    """Batch sizes around the wave (64), block (256) and the 21-arc packing of the delete
    kernel's view lanes."""
    say(f"case: ragged batch {b}")
    g = I.rmat_s(10)
    p = make_pair(g, source=I.max_out_degree_vertex(g))
    wl = I.Workload(g, 100 + b)
    s, d, w = wl.insert_batch(b)
    p.insert(s, d, w)
    s, d = wl.delete_batch(b)
    p.delete(s, d)
    qs, qd = wl.query_batch(b)
    p.query(qs, qd)
    p.check_structure()
    p.check_all(algos=("bfs", "sssp", "wcc", "tc"))


@pytest.mark.parametrize("lf", [0.7, 0.0])
@pytest.mark.parametrize("scheme", [native.WCC_LOG, native.WCC_NAIVE, native.WCC_SLAB, native.WCC_UPDATE])
def test_wcc_schemes_agree(scheme, lf):
    """Every incremental-WCC scheme gives the oracle's labels (hashing on, and off: the
    single-bucket variant).  A graph of many small components plus a hub with 600 out-arcs
    (a heavy vertex when hashing is on) takes insert batches that merge components (hub
    arcs, in-batch duplicates, arcs already present), two pending batches at once, a delete
    batch (a recompute), and a compaction between a pass and the next one, which moves the
    words of chains that hold both tombstones and not-yet-united arcs."""
    say(f"case: WCC scheme {scheme}, load factor {lf}")
    rng = np.random.default_rng(40 + scheme)
    n, hub = 6000, 7
    src = np.concatenate([rng.integers(0, n, 2000), np.full(600, hub)])
    dst = np.concatenate([rng.integers(0, n, 2000), rng.choice(n, 600, replace=False)])
    keep = src != dst
    src, dst = src[keep], dst[keep]
    p = Pair(n, src, dst, rng.integers(1, 100, len(src)), views=native.VIEW_FWD, load_factor=lf)

    def check():
        lab = p.g.wcc(scheme=scheme)
        assert np.array_equal(u32(lab), p.o.wcc())

    def batch(b):
        s, d = rng.integers(0, n, b), rng.integers(0, n, b)
        s[: b // 3] = hub
        if b > 4:
            s[-2:], d[-2:] = s[:2], d[:2]  # duplicates inside the batch
        # the weight is a function of the arc, so whichever copy of a duplicate applies,
        # the stored weight is the same
        p.insert(s, d, (s * 31 + d * 17) % 99 + 1, exact_status=False)

    check()
    for b in (1, 300, 2000):
        batch(b)
        check()
    batch(500)
    batch(500)
    check()
    os_, od, _ = p.o.export()
    pick = rng.choice(len(os_), 400, replace=False)
    pick = np.concatenate([pick, np.nonzero(os_ == hub)[0][:100]])
    pick = np.unique(pick)
    p.delete(os_[pick], od[pick])
    check()
    batch(300)
    assert p.g.compact() >= 0
    check()
    batch(200)
    check()
    p.check_structure()
    with pytest.raises(RuntimeError):
        p.g.wcc(scheme=4)


@pytest.mark.parametrize("lf", [0.7, 0.0])
def test_sampled_static_wcc_with_all_views(lf):
    """The static WCC of a graph with the undirected view (first unions from each primary
    slab, the most frequent sampled root taken as the largest component, whose vertices then
    skip their arcs) gives the oracle's labels: two equally large components, a low id reached
    only through an in-arc, a low id that joins a large component through a vertex outside it,
    small components and many isolated vertices; again after a delete batch that cuts one
    large component in two at its only bridge, and after one that isolates the low ids."""
    say(f"case: sampled static WCC, load factor {lf}")
    rng = np.random.default_rng(91)
    n = 20_000

    def blob(lo, hi, m):
        a, b = rng.integers(lo, hi, m), rng.integers(lo, hi, m)
        return a[a != b], b[a != b]

    a1s, a1d = blob(10_000, 12_500, 12_000)
    a2s, a2d = blob(12_500, 15_000, 12_000)
    bs, bd = blob(15_000, 20_000, 24_000)
    src = np.concatenate([a1s, a2s, bs, [12_000, 12_600, 2, 100, 101, 500]])
    dst = np.concatenate([a1d, a2d, bd, [12_600, 3, 15_500, 101, 102, 2]])
    # 12000 -> 12600 is the only bridge between the halves of A; 3 has only an in-arc (from
    # 12600); 2 joins B and 500 hangs off 2; 100-101-102 is a small chain
    key = np.unique(src.astype(np.int64) * n + dst)
    src, dst = key // n, key % n
    p = Pair(n, src, dst, rng.integers(1, 100, src.size), views=7, load_factor=lf)
    p.check_all(algos=("wcc",))
    p.delete(np.array([12_000]), np.array([12_600]))
    p.check_all(algos=("wcc",))
    p.delete(np.array([12_600, 2]), np.array([3, 15_500]))
    p.check_all(algos=("wcc",))
    p.insert(np.array([3, 12_000]), np.array([15_000, 12_600]), np.array([1, 1]))
    p.check_all(algos=("wcc",))
    p.check_wcc(native.RECOMPUTE)


@pytest.mark.parametrize("top_down_only", [False, True])
def test_bfs_levels_distance_only(top_down_only):
    """The distance-only, direction-optimizing BFS gives the oracle's levels: R-MAT from the
    hub (bottom-up steps taken unless disabled) and from a low-degree vertex, after an insert
    and a delete batch, on the road-like grid, on a graph without the reverse view (top-down
    only), from a source without out-arcs, and on one vertex."""
    say(f"case: BFS levels, top-down only = {top_down_only}")

    def cmp(pair, src, expect_bu=None):
        lv, bu = pair.g.bfs_levels(src, top_down_only)
        lo, _ = pair.o.bfs(src)
        assert np.array_equal(u32(lv), lo), f"levels differ at {np.nonzero(u32(lv) != lo)[0][:10]}"
        if top_down_only:
            assert bu == 0
        elif expect_bu is not None:
            assert (bu > 0) == expect_bu, bu
        return bu

    g = I.rmat_s(12)
    hub = I.max_out_degree_vertex(g)
    p = make_pair(g, source=hub)
    cmp(p, hub, expect_bu=True)
    deg = np.bincount(u32(g.src), minlength=g.n)
    low = int(np.nonzero(deg == 1)[0][0])
    cmp(p, low)
    wl = I.Workload(g, 31)
    s, d, w = wl.insert_batch(3000)
    p.insert(s, d, w)
    cmp(p, hub)
    s, d = wl.delete_batch(3000)
    p.delete(s, d)
    cmp(p, hub)
    cmp(p, low)
    cmp(p, int(np.nonzero(deg == 0)[0][0]))
    gg = I.grid_graph(64, 0x4D45524B + 2)
    cmp(make_pair(gg), 0)
    q = make_pair(g, source=hub, views=native.VIEW_FWD)
    cmp(q, hub, expect_bu=False)
    cmp(Pair(1, [], [], [], source=0), 0, expect_bu=False)


@pytest.mark.parametrize("delta", [0, 1, 1 << 30])
def test_sssp_distances_distance_only(delta):
    """The distance-only SSSP gives the oracle's distances for any band width (0: the default):
    R-MAT from the hub and from a low-degree vertex, after an insert and a delete batch, the
    road-like grid (weights up to 1,000), a chain whose distances reach 0xFFFFFFFE (the
    largest finite one), a source without out-arcs, and one vertex."""
    say(f"case: SSSP distances, band width {delta}")

    def cmp(pair, src):
        di = pair.g.sssp_distances(src)
        do, _ = pair.o.sssp(src)
        assert np.array_equal(u32(di), do), f"distances differ at {np.nonzero(u32(di) != do)[0][:10]}"

    g = I.rmat_s(12)
    hub = I.max_out_degree_vertex(g)
    p = make_pair(g, source=hub, sssp_delta=delta)
    cmp(p, hub)
    deg = np.bincount(u32(g.src), minlength=g.n)
    low = int(np.nonzero(deg == 1)[0][0])
    cmp(p, low)
    wl = I.Workload(g, 41)
    s, d, w = wl.insert_batch(3000)
    p.insert(s, d, w)
    cmp(p, hub)
    s, d = wl.delete_batch(3000)
    p.delete(s, d)
    cmp(p, hub)
    cmp(p, int(np.nonzero(deg == 0)[0][0]))
    gg = I.grid_graph(64, 0x4D45524B + 2)
    cmp(make_pair(gg, sssp_delta=delta), 0)
    big = 0x7FFFFFFF
    cmp(Pair(4, [0, 1, 0], [1, 2, 3], [big, big, 0xFFFFFFF0], sssp_delta=delta), 0)
    cmp(Pair(1, [], [], [], sssp_delta=delta), 0)


def test_distance_only_entry_points_reject_bad_arguments():
    """Host-side checks of the distance-only traversals: a source out of range, a slot out of
    range, a workspace one byte short and an unknown flag are refused with their statuses."""
    say("case: distance-only entry points, bad arguments")
    g = I.rmat_s(10)
    G = native.Graph(g.n, g.src, g.dst, g.w)
    lib = G.lib
    n_lv, n_ds = lib.mk_bfs_levels_workspace_bytes(G.h), lib.mk_sssp_distances_workspace_bytes(G.h)
    ws = torch.empty(max(n_lv, n_ds), dtype=torch.uint8, device=G.device)
    out = torch.empty(g.n, dtype=torch.int32, device=G.device)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    s = ctypes.c_void_p(G.stream.cuda_stream)
    bu = ctypes.c_uint32()
    assert lib.mk_bfs_levels(G.h, g.n, 0, p(ws), n_lv, 0, p(out), ctypes.byref(bu), s) == 1
    assert lib.mk_bfs_levels(G.h, 0, 0, p(ws), n_lv, 16, p(out), ctypes.byref(bu), s) == 1
    assert lib.mk_bfs_levels(G.h, 0, 2, p(ws), n_lv, 0, p(out), ctypes.byref(bu), s) == 1
    assert lib.mk_bfs_levels(G.h, 0, 0, p(ws), n_lv - 1, 0, p(out), ctypes.byref(bu), s) == 3
    assert lib.mk_sssp_distances(G.h, g.n, p(ws), n_ds, 0, p(out), s) == 1
    assert lib.mk_sssp_distances(G.h, 0, p(ws), n_ds, 16, p(out), s) == 1
    assert lib.mk_sssp_distances(G.h, 0, p(ws), n_ds - 1, 0, p(out), s) == 3
    lab = torch.empty(g.n, dtype=torch.int32, device=G.device)
    assert lib.mk_incr_wcc_scheme(G.h, p(lab), 0, 4, s) == 1
    # the same calls with good arguments still work afterwards
    lv, _ = G.bfs_levels(0, ws=ws)
    di = G.sssp_distances(0, ws=ws)
    torch.cuda.synchronize()
    assert int(lv[0].item()) == 0 and int(di[0].item()) == 0


@pytest.mark.parametrize("lf", [0.7, 0.0])
def test_iteration_scheme2_agrees_with_the_oracle(lf):
    """IterationScheme2 (a 16-lane group per <vertex, bucket> chain, grid-stride over the pair
    list) for the PageRank pull and the static WCC: labels exact and PageRank within 1e-6 in
    L1, from scratch and warm after insert and delete batches, with hashing on and off (one
    bucket per vertex); switching back to IterationScheme1 gives the same results."""
    say(f"case: IterationScheme2, load factor {lf}")
    g = I.rmat_s(12)
    p = make_pair(g, source=I.max_out_degree_vertex(g), load_factor=lf)
    p.g.set_iteration_scheme(native.ITER_SCHEME2)
    p.check_wcc(native.RECOMPUTE)
    p.check_pr(native.RECOMPUTE)
    wl = I.Workload(g, 77)
    p.insert(*wl.insert_batch(2000))
    p.check_pr()
    p.check_wcc(native.RECOMPUTE)
    p.delete(*wl.delete_batch(2000))
    p.check_pr()
    p.check_wcc()  # a delete forces the recompute, here through scheme 2
    lab2 = p.g.wcc(native.RECOMPUTE)
    p.g.set_iteration_scheme(native.ITER_SCHEME1)
    assert torch.equal(p.g.wcc(native.RECOMPUTE), lab2)
    p.check_pr(native.RECOMPUTE)
    with pytest.raises(native.MkError):
        p.g.set_iteration_scheme(4)


@pytest.mark.parametrize("lf", [0.7, 0.0])
def test_packed_pagerank_iterations_agree_with_the_oracle(lf):
    """The packed PageRank iterations (the first one of a call walks the slabs and packs the
    in-arc keys, the others read the packed lists): within 1e-6 in L1 of the oracle from
    scratch and warm after insert and delete batches, hashing on and off, with vertices of
    one bucket, of 2..16 buckets and heavier ones; scheme 1 gives the same ranks within the
    tolerance."""
    say(f"case: packed PageRank, load factor {lf}")
    g = I.rmat_s(12)
    p = make_pair(g, source=I.max_out_degree_vertex(g), load_factor=lf)
    p.g.set_iteration_scheme(native.ITER_PACKED)
    p.check_pr(native.RECOMPUTE)
    wl = I.Workload(g, 78)
    for b in (3000, 300):
        p.insert(*wl.insert_batch(b))
        p.check_pr()
        p.delete(*wl.delete_batch(b))
        p.check_pr()
    r_packed, _ = p.g.pagerank(mode=native.RECOMPUTE)
    p.g.set_iteration_scheme(native.ITER_SCHEME1)
    r_s1, _ = p.g.pagerank(mode=native.RECOMPUTE)
    assert float((r_packed.double() - r_s1.double()).abs().sum()) <= 2 * PR_L1_TOL


def test_cost_model_on_the_graph_decides_auto_mode():
    """mk_set_cost_model: with parameters whose network always predicts a recompute faster
    (all weights zero, output biases log-incremental 1 > log-recompute 0), MK_AUTO recomputes
    (PageRank starts cold: as many iterations as an explicit recompute); with the biases
    swapped it applies the batch incrementally (a warm start, far fewer iterations).  Every
    result still equals the oracle's."""
    say("case: cost model set on the graph")
    g = I.rmat_s(12)
    p = make_pair(g, source=I.max_out_degree_vertex(g))
    p.check_all()
    wl = I.Workload(g, 91)
    prefer_rec = torch.zeros(5187)
    prefer_rec[5184:5187] = torch.tensor([1.0, 0.0, 0.0])
    prefer_inc = torch.zeros(5187)
    prefer_inc[5184:5187] = torch.tensor([0.0, 1.0, 0.0])
    iters = {}
    for name, params in (("recompute", prefer_rec), ("incremental", prefer_inc)):
        p.g.set_cost_model(params)
        p.insert(*wl.insert_batch(300))
        _, it = p.g.pagerank()
        iters[name] = int(it.item())
        p.check_pr()
        p.check_all(algos=("bfs", "sssp", "wcc", "tc"))
        p.delete(*wl.delete_batch(300))
        p.check_all()
    _, it_cold = p.g.pagerank(mode=native.RECOMPUTE)
    it_cold = int(it_cold.item())
    say(f"  PageRank iterations: chosen recompute {iters['recompute']}, chosen incremental "
        f"{iters['incremental']}, explicit recompute {it_cold}")
    assert abs(iters["recompute"] - it_cold) <= 1
    assert iters["incremental"] < it_cold - 2
    p.g.set_cost_model(None)
    assert p.g.lib.mk_set_cost_model(p.g.h, ctypes.c_void_p(2)) == 1  # misaligned: refused


def test_triangle_updates_around_hubs():
    """Triangle counts after batches whose edges touch hubs of 1,500, 3,000, 24,000 and 49,999
    neighbours: the batch-identity sum S1 of those edges runs through LDS hash sets of the hub
    neighbourhoods: the small-hub class (one 32 KiB set) for the first, the large class in 1,
    3 and 5 hash passes for the others, also for a batch of two edges of the 3,000-neighbour
    hub, one to the largest hub (a hub by its degree and that partner's); every count equals
    the oracle's."""
    say("case: triangle updates around hubs")
    n = 50_000
    rng = np.random.default_rng(17)
    others = np.arange(1, n)
    hub_s = np.concatenate([np.zeros(n - 1, np.int64), np.ones(24_000, np.int64), np.full(3_000, 2),
                            np.full(1_500, 3)])
    hub_d = np.concatenate([others, rng.permutation(np.arange(2, n))[:24_000],
                            rng.permutation(np.arange(3, n))[:3_000], rng.permutation(np.arange(4, n))[:1_500]])
    flip = rng.random(hub_s.size) < 0.5  # both arc directions occur
    s = np.where(flip, hub_d, hub_s)
    d = np.where(flip, hub_s, hub_d)
    bs = rng.integers(4, n, 150_000)
    bd = rng.integers(4, n, 150_000)
    keep = bs != bd
    s = np.concatenate([s, bs[keep]])
    d = np.concatenate([d, bd[keep]])
    key = np.unique(s.astype(np.int64) * n + d)
    s, d = key // n, key % n
    p = Pair(n, s, d, rng.integers(1, 100, s.size), source=0)
    p.check_tc()
    arcs = np.stack([s, d], 1)
    for b in (4_000, 20_000):
        pick = arcs[rng.choice(len(arcs), b, replace=False)]  # hub-biased: most arcs touch a hub
        p.delete(pick[:, 0], pick[:, 1])
        p.check_tc()
        ins_s = np.concatenate([np.zeros(b // 2, np.int64), rng.integers(4, n, b // 2)])
        ins_d = rng.integers(1, n, b)
        ik = np.unique(ins_s[ins_s != ins_d] * n + ins_d[ins_s != ins_d])  # no in-batch duplicates
        p.insert(ik // n, ik % n, np.full(ik.size, 3))
        p.check_tc()
        p.insert(pick[:, 0], pick[:, 1], np.full(b, 5))  # the deleted arcs come back
        p.check_tc()
    # two batch edges of the 3,000-neighbour hub, one of them to the 49,999-neighbour hub: a
    # hub by its degree and that large partner, with fewer than 4 batch edges
    e02 = arcs[((arcs[:, 0] == 0) & (arcs[:, 1] == 2)) | ((arcs[:, 0] == 2) & (arcs[:, 1] == 0))][:1]
    e2x = arcs[((arcs[:, 0] == 2) & (arcs[:, 1] > 3)) | ((arcs[:, 1] == 2) & (arcs[:, 0] > 3))][:1]
    two = np.concatenate([e02, e2x])
    assert len(two) == 2
    p.delete(two[:, 0], two[:, 1])
    p.check_tc()
    p.insert(two[:, 0], two[:, 1], np.full(2, 7))
    p.check_tc()
