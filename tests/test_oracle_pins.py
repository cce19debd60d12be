"""Pins of the CPU oracle against closed forms, brute force and independent methods.

None of these re-types the oracle's own code: the expected values come from textbook
closed forms (triangles of K_n, wheels, cycles; PageRank of a directed cycle; BFS on
a path), from library routines (scipy connected components, numpy linear solves and
matrix powers) or from brute force written differently (Bellman-Ford relaxation,
dict-based set semantics).
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

INF = 0xFFFFFFFF


def mk(orc, n, arcs, w=None):
    arcs = np.asarray(arcs, dtype=np.uint32).reshape(-1, 2)
    ww = None if w is None else np.asarray(w, np.uint32)
    return orc.OracleGraph(n, arcs[:, 0], arcs[:, 1], ww)


def undirected(pairs):
    out = []
    for a, b in pairs:
        out += [(a, b), (b, a)]
    return out


def rand_digraph(rng, n, m, wmax=9):
    arcs = set()
    while len(arcs) < m:
        a, b = rng.integers(0, n, 2)
        if a != b:
            arcs.add((int(a), int(b)))
    arcs = sorted(arcs)
    w = rng.integers(1, wmax + 1, len(arcs))
    return arcs, w


# ---------------------------------------------------------------- set semantics
def test_ops_match_dict_model(orc):
    rng = np.random.default_rng(1)
    n = 20
    g = mk(orc, n, np.zeros((0, 2)))
    model = {}
    for rnd in range(30):
        b = int(rng.integers(1, 40))
        s = rng.integers(0, n + 2, b)
        d = rng.integers(0, n + 2, b)
        w = rng.integers(1, 100, b)
        if rnd % 3 == 0:
            st = g.delete(s, d)
            for i in range(b):
                key = (int(s[i]), int(d[i]))
                if s[i] >= n or d[i] >= n or s[i] == d[i]:
                    exp = 2
                elif key in model:
                    del model[key]
                    exp = 1
                else:
                    exp = 0
                assert st[i] == exp
        else:
            st = g.insert(s, d, w)
            for i in range(b):
                key = (int(s[i]), int(d[i]))
                if s[i] >= n or d[i] >= n or s[i] == d[i]:
                    exp = 2
                elif key in model:
                    exp = 0  # present: no-op, first weight kept
                else:
                    model[key] = int(w[i])
                    exp = 1
                assert st[i] == exp
        qs = rng.integers(0, n, 50)
        qd = rng.integers(0, n, 50)
        f, qw = g.query(qs, qd)
        for i in range(50):
            key = (int(qs[i]), int(qd[i]))
            assert f[i] == (key in model)
            assert qw[i] == model.get(key, 0)
    s, d, w = g.export()
    assert sorted(model.items()) == [((int(a), int(b)), int(c)) for a, b, c in zip(s, d, w)]


def test_reserved_ids_rejected(orc):
    g = mk(orc, 8, [(0, 1)])
    st = g.insert([0xFFFFFFFD, 1, 2, 3], [1, 0xFFFFFFFE, 2, 9], [1, 1, 1, 1])
    assert list(st) == [2, 2, 2, 2]


# ---------------------------------------------------------------- BFS
def test_bfs_path_levels_equal_position(orc):
    n = 50
    g = mk(orc, n, [(i, i + 1) for i in range(n - 1)])
    lv, pa = g.bfs(0)
    assert list(lv) == list(range(n))
    assert list(pa) == [0] + list(range(n - 1))
    lv, pa = g.bfs(10)  # vertices before the source are unreachable
    assert list(lv[:10]) == [INF] * 10 and list(lv[10:]) == list(range(n - 10))
    assert list(pa[:10]) == [INF] * 10


def bellman_ford(n, arcs, w, src):
    """Repeated relaxation until no change (64-bit), no heap."""
    dist = [math.inf] * n
    dist[src] = 0
    changed = True
    while changed:
        changed = False
        for (a, b), c in zip(arcs, w):
            if dist[a] + c < dist[b]:
                dist[b] = dist[a] + c
                changed = True
    return dist


def check_tree(n, arcs, w, src, dist_exp, dist, parent):
    for v in range(n):
        if dist_exp[v] == math.inf:
            assert dist[v] == INF and parent[v] == INF
        else:
            assert dist[v] == dist_exp[v]
    # parent = smallest in-neighbour achieving the distance
    best = {}
    for (a, b), c in zip(arcs, w):
        if dist_exp[a] != math.inf and dist_exp[a] + c == dist_exp[b] and b != src:
            best[b] = min(best.get(b, INF), a)
    for v in range(n):
        if v == src:
            assert parent[v] == src
        elif dist_exp[v] != math.inf:
            assert parent[v] == best[v]


@pytest.mark.parametrize("seed", range(6))
def test_bfs_and_sssp_vs_bellman_ford(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    m = int(rng.integers(0, min(n * (n - 1), 4 * n)))
    arcs, w = rand_digraph(rng, n, m)
    g = mk(orc, n, arcs, w)
    src = int(rng.integers(0, n))
    lv, pa = g.bfs(src)
    check_tree(n, arcs, [1] * len(arcs), src, bellman_ford(n, arcs, [1] * len(arcs), src), lv, pa)
    di, pa = g.sssp(src)
    check_tree(n, arcs, list(w), src, bellman_ford(n, arcs, list(w), src), di, pa)


def test_sssp_hand_example(orc):
    # 0->1 (4), 0->2 (1), 2->1 (3), 1->3 (1), 2->3 (5), 3->4 (2); 4 has two equal routes?
    arcs = [(0, 1), (0, 2), (2, 1), (1, 3), (2, 3), (3, 4), (5, 4)]
    w = [4, 1, 3, 1, 5, 2, 1]
    g = mk(orc, 6, arcs, w)
    di, pa = g.sssp(0)
    # d(1)=min(4, 1+3)=4 reached by 0 and by 2 -> parent 0 (smaller id); d(3)=5 via 1 or 2
    # -> parent 1; d(4)=7 via 3; vertex 5 is unreachable.
    assert list(di) == [0, 4, 1, 5, 7, INF]
    assert list(pa) == [0, 0, 0, 1, 3, INF]


# ---------------------------------------------------------------- WCC
@pytest.mark.parametrize("seed", range(5))
def test_wcc_vs_scipy(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 300))
    arcs, w = rand_digraph(rng, n, int(rng.integers(0, n)))
    g = mk(orc, n, arcs, w)
    lab = g.wcc()
    a = np.array(arcs, dtype=np.int64).reshape(-1, 2)
    mat = sp.coo_matrix((np.ones(len(a)), (a[:, 0], a[:, 1])), shape=(n, n))
    k, comp = connected_components(mat, directed=True, connection="weak")
    minid = {}
    for v in range(n):
        minid.setdefault(comp[v], v)
    assert [minid[comp[v]] for v in range(n)] == list(lab)


def test_wcc_disjoint_cycles(orc):
    arcs = []
    k, L = 7, 5
    for c in range(k):
        base = 3 + c * L
        arcs += [(base + i, base + (i + 1) % L) for i in range(L)]
    g = mk(orc, 3 + k * L, arcs)
    lab = g.wcc()
    assert len(set(lab.tolist())) == k + 3
    assert list(lab[:3]) == [0, 1, 2]


# ---------------------------------------------------------------- PageRank
def test_pagerank_directed_cycle_uniform(orc):
    n = 17
    g = mk(orc, n, [(i, (i + 1) % n) for i in range(n)])
    r, _ = g.pagerank()
    assert np.abs(r - 1.0 / n).max() < 1e-15


def test_pagerank_edgeless_uniform(orc):
    g = mk(orc, 9, np.zeros((0, 2)))
    r, _ = g.pagerank()
    assert np.abs(r - 1.0 / 9).max() < 1e-15


@pytest.mark.parametrize("seed", range(5))
def test_pagerank_dense_solve(orc, seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(2, 64))
    arcs, _ = rand_digraph(rng, n, int(rng.integers(0, 3 * n)))
    g = mk(orc, n, arcs)
    d = 0.85
    r, it = g.pagerank(damping=d)
    out = np.zeros(n)
    for a, b in arcs:
        out[a] += 1
    M = np.zeros((n, n))
    for a, b in arcs:
        M[b, a] += 1.0 / out[a]
    dang = (out == 0).astype(float)
    # x = (1-d)/N + d*(M x + (dang . x)/N)  <=>  (I - d M - d/N 1 dang^T) x = (1-d)/N 1
    A = np.eye(n) - d * M - d / n * np.outer(np.ones(n), dang)
    x = np.linalg.solve(A, np.full(n, (1 - d) / n))
    assert np.abs(x - r).sum() < 1e-11
    assert abs(r.sum() - 1.0) < 1e-12


# ---------------------------------------------------------------- triangles
@pytest.mark.parametrize("n", [3, 4, 5, 8, 13])
def test_triangles_complete_graph(orc, n):
    arcs = [(a, b) for a in range(n) for b in range(n) if a != b]
    g = mk(orc, n, arcs)
    assert g.triangles() == math.comb(n, 3) == g.triangles_brute()


def test_triangles_cycles_wheel_bipartite(orc):
    g = mk(orc, 3, [(0, 1), (1, 2), (2, 0)])  # a directed 3-cycle is one triangle
    assert g.triangles() == 1
    for n in (4, 5, 9):
        g = mk(orc, n, [(i, (i + 1) % n) for i in range(n)])
        assert g.triangles() == 0
    for n in (4, 6, 11):  # wheel: hub 0 + n-cycle on 1..n has n triangles
        pairs = [(0, i) for i in range(1, n + 1)] + [(i, i % n + 1) for i in range(1, n + 1)]
        g = mk(orc, n + 1, undirected(pairs))
        assert g.triangles() == n
    pairs = [(a, b) for a in range(5) for b in range(5, 12)]
    g = mk(orc, 12, pairs)
    assert g.triangles() == 0


@pytest.mark.parametrize("seed", range(6))
def test_triangles_vs_trace_and_brute(orc, seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(4, 40))
    arcs, _ = rand_digraph(rng, n, int(rng.integers(0, n * (n - 1) // 2)))
    g = mk(orc, n, arcs)
    A = np.zeros((n, n), dtype=np.int64)
    for a, b in arcs:
        A[a, b] = A[b, a] = 1
    t_trace = int(np.trace(A @ A @ A)) // 6
    assert g.triangles() == t_trace == g.triangles_brute()


def test_inclusion_exclusion_reading(orc):
    """The batch identities of the triangle-counting section, evaluated with dense
    matrices, equal the oracle's before/after difference (pins the reading that the
    per-batch count runs over both directions of the effective undirected batch)."""
    rng = np.random.default_rng(7)
    n = 24
    for trial in range(8):
        base, _ = rand_digraph(rng, n, 70)
        g = mk(orc, n, base)
        t0 = g.triangles()
        A = np.zeros((n, n), dtype=np.int64)
        for a, b in base:
            A[a, b] = A[b, a] = 1
        # effective undirected batch: pairs absent before (insert) or present (delete)
        cand = [(a, b) for a, b in itertools.combinations(range(n), 2)]
        rng.shuffle(cand)
        ins = trial % 2 == 0
        E = [(a, b) for a, b in cand if (A[a, b] == 0) == ins][:15]
        U = np.zeros_like(A)
        for a, b in E:
            U[a, b] = U[b, a] = 1
        post = A + U if ins else A - U
        arcs = undirected(E)
        S1 = sum(int(post[u] @ post[v]) for u, v in arcs)
        S2 = sum(int(post[u] @ U[v]) for u, v in arcs)
        S3 = sum(int(U[u] @ U[v]) for u, v in arcs)
        if ins:
            g.insert([a for a, b in arcs], [b for a, b in arcs])
            delta = (S1 - S2 + S3 // 3) // 2
            assert (S1 - S2 + S3 / 3) % 2 == 0
            assert g.triangles() - t0 == delta
        else:
            # delete both orientations so the undirected pair disappears
            g.delete([a for a, b in arcs], [b for a, b in arcs])
            delta = (S1 + S2 + S3 // 3) // 2
            assert t0 - g.triangles() == delta


# ---------------------------------------------------------------- triangles touching a batch
@pytest.mark.parametrize("n", [4, 6, 9])
def test_triangles_touching_closed_forms(orc, n):
    """In K_n an edge lies in n-2 triangles, two edges sharing a vertex in 2(n-2)-1, two
    disjoint edges in 2(n-2), and the edge set of K_n touches all C(n,3) triangles; pairs that
    are not edges, self-pairs and repeats add nothing."""
    arcs = [(a, b) for a in range(n) for b in range(n) if a != b]
    g = mk(orc, n, arcs)
    assert g.triangles_touching([0], [1]) == n - 2
    assert g.triangles_touching([1, 0, 0], [0, 1, 0]) == n - 2
    assert g.triangles_touching([0, 0], [1, 2]) == 2 * (n - 2) - 1
    assert g.triangles_touching([0, 2], [1, 3]) == 2 * (n - 2)
    a, b = zip(*itertools.combinations(range(n), 2))
    assert g.triangles_touching(a, b) == math.comb(n, 3)
    g2 = mk(orc, n, [(i, (i + 1) % n) for i in range(n)])  # a cycle: no triangle
    assert g2.triangles_touching(a, b) == (1 if n == 3 else 0)
    assert g.triangles_touching([], []) == 0


@pytest.mark.parametrize("seed", range(8))
def test_triangles_touching_equals_brute_difference(orc, seed):
    """On random graphs, the triangles touching a random set of pairs equal the triple-loop
    count minus the triple-loop count with those undirected edges removed."""
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(5, 30))
    arcs, _ = rand_digraph(rng, n, int(rng.integers(n, n * (n - 1) // 2)))
    g = mk(orc, n, arcs)
    k = int(rng.integers(1, 25))
    a = rng.integers(0, n, k)
    b = rng.integers(0, n, k)
    touched = g.triangles_touching(a, b)
    drop = {(int(x), int(y)) for x, y in zip(a, b)} | {(int(y), int(x)) for x, y in zip(a, b)}
    rest = [e for e in arcs if e not in drop]
    assert touched == g.triangles_brute() - mk(orc, n, rest).triangles_brute()
