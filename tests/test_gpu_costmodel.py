"""GPU tests of the cost model: the HIP MLP kernels against the FP64 oracle, the batch
features of all five algorithms against values built from the oracle's degrees, trees and
labels, and the trained policy's regret against the always-incremental rule on held-out
graph states."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from paper_2305_17813_amd import costmodel as CM
from paper_2305_17813_amd import inputs as I
from paper_2305_17813_amd import native
from parity import Pair, say, u32

pytestmark = pytest.mark.gpu


def _problem(seed, n):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, omlp.N_PARAMS)
    X = rng.normal(0, 1, (n, 12))
    T = rng.normal(0, 1, (n, 3))
    M = (rng.random((n, 3)) < 0.8).astype(float)
    return p, X, T, M


def _dev(a):
    return torch.as_tensor(np.asarray(a, np.float32)).cuda().contiguous()


@pytest.mark.parametrize("n", [1, 37, 300])
def test_forward_and_gradient_match_oracle(n):
    say(f"case: MLP forward/grad n={n}")
    p, X, T, M = _problem(n, n)
    net = CM.MLP("cuda")
    net.params.copy_(_dev(p))
    y = net.forward(_dev(X)).cpu().numpy()
    yo, _ = omlp.forward(p.astype(np.float32).astype(np.float64), X.astype(np.float32))
    assert np.abs(y - yo).max() <= 1e-4 * max(1.0, np.abs(yo).max())
    loss = float(net.gradient(_dev(X), _dev(T), _dev(M)))
    p32 = p.astype(np.float32).astype(np.float64)
    X32, T32 = X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64)
    go = omlp.grad(p32, X32, T32, M)
    g = net.grad.cpu().numpy()
    assert np.abs(g - go).max() <= 1e-4 * np.abs(go).max()
    assert abs(loss - omlp.loss(p32, X32, T32, M)) <= 1e-5 * max(1.0, loss)


def test_adam_matches_oracle_over_steps():
    say("case: MLP Adam steps")
    p, X, T, M = _problem(5, 64)
    net = CM.MLP("cuda")
    net.params.copy_(_dev(p))
    po = p.astype(np.float32).astype(np.float64)
    m = np.zeros_like(po)
    v = np.zeros_like(po)
    for step in range(1, 6):
        net.gradient(_dev(X), _dev(T), _dev(M))
        g = net.grad.cpu().numpy().astype(np.float64)  # same gradient on both sides
        net.adam(lr=1e-2)
        po, m, v = omlp.adam(po, g, m, v, step, lr=1e-2)
        assert np.abs(net.params.cpu().numpy() - po).max() <= 1e-5


INF = 0xFFFFFFFF


def _expected_features(p, algo, ins, dels, tree=None, labels=None, pending=0):
    """The twelve features of mk_batch_features, built in FP64 from the oracle's state:
    out-degrees, in-degrees (from its arcs), undirected degrees, the BFS/SSSP tree of the
    algorithm's last run (`tree` = (dist, parent)) and the WCC labels of its last run."""
    n_v = p.n
    out = p.o.out_degree().astype(np.float64)
    s_all, d_all, _ = p.o.export()
    indeg = np.bincount(d_all, minlength=n_v).astype(np.float64)
    und = p.o.undirected_degree().astype(np.float64)
    isrc, idst = u32(ins[0]), u32(ins[1])
    iw = u32(ins[2]) if len(ins) > 2 else np.ones_like(isrc)
    dsrc, ddst = u32(dels[0]), u32(dels[1])
    srcs = np.concatenate([isrc, dsrc])
    dsts = np.concatenate([idst, ddst])
    n = srcs.size
    if algo in (0, 1):
        if tree is None:
            aff, depth = 0.0, 0.0
        else:
            dist, par = (x.astype(np.uint64) for x in tree)
            w = np.ones_like(iw, dtype=np.uint64) if algo == 0 else iw.astype(np.uint64)
            relax = (dist[isrc] != INF) & (dist[isrc] + w < dist[idst])
            tree_arc = (dist[ddst] != INF) & (par[ddst] == dsrc)
            aff = (relax.sum() + tree_arc.sum()) / n
            fin = dist[dist != INF]
            depth = np.log2(1 + fin.max()) / 32
    elif algo == 2:
        joins = 0 if labels is None else (labels[isrc] != labels[idst]).sum()
        aff = (joins + dsrc.size) / n
        depth = 0.0
    elif algo == 3:
        aff = np.mean(1 / (1 + out[srcs]))
        depth = 0.0
    else:
        aff = np.mean(np.log2(1 + np.minimum(und[srcs], und[dsts]))) / 32
        depth = 0.0
    return np.asarray([np.log2(1 + n) / 32, isrc.size / n, dsrc.size / n, np.log2(n_v) / 32,
                       np.log2(1 + out.sum()) / 32, np.mean(np.log2(1 + out[srcs])) / 32,
                       np.log2(1 + out[srcs].max()) / 32, np.mean(np.log2(1 + indeg[dsts])) / 32,
                       aff, depth, np.log2(1 + pending) / 32, algo / 4], np.float32)


@pytest.mark.parametrize("algo", [0, 1, 2, 3, 4])
def test_batch_features_match_values_from_the_oracle(algo):
    """Every feature of every algorithm: sizes and mix, degrees of the touched vertices
    (out-, in- and undirected), the affected fraction (BFS/SSSP: inserts that would relax plus
    deleted tree arcs, from the oracle's tree; WCC: inserts joining two of the oracle's
    components plus deletions; PageRank: mean 1/(1+out-degree); triangles: mean log2 of the
    smaller undirected degree) and the tree depth from the oracle's distances."""
    say(f"case: batch features, algo {algo}")
    g = I.rmat_s(11)
    p = Pair(g.n, g.src, g.dst, g.w, source=I.max_out_degree_vertex(g))
    wl = I.Workload(g, 6 + algo)
    # a first batch, then the algorithm runs: its state is what the features read
    s, d, w = wl.insert_batch(200)
    p.insert(s, d, w)
    tree = labels = None
    if algo == 0:
        p.g.bfs(p.source)
        tree = p.o.bfs(p.source)
    elif algo == 1:
        p.g.sssp(p.source)
        tree = p.o.sssp(p.source)
    elif algo == 2:
        p.g.wcc()
        labels = p.o.wcc()
    elif algo == 3:
        p.g.pagerank()
    else:
        p.g.triangles()
    ins = wl.insert_batch(300)
    dels = wl.delete_batch(100)
    f = p.g.batch_features(algo, ins, dels)
    exp = _expected_features(p, algo, ins, dels, tree, labels)
    assert np.allclose(f, exp, rtol=1e-5, atol=1e-6), (algo, f, exp)
    # pending batches are counted, and the tree / labels stay those of the last run
    p.insert(*ins)
    p.delete(*dels)
    ins2 = wl.insert_batch(150)
    f2 = p.g.batch_features(algo, ins2, (torch.empty(0, dtype=torch.int32),) * 2)
    exp2 = _expected_features(p, algo, ins2, (np.empty(0, np.uint32),) * 2, tree, labels, pending=2)
    assert np.allclose(f2, exp2, rtol=1e-5, atol=1e-6), (algo, f2, exp2)


def test_trained_policy_beats_always_incremental():
    """Records from the method's own timings on a road-like grid and a power-law graph;
    the MLP is trained on the older graph states (HIP kernels) and judged on the newer ones."""
    say("case: cost-model regret")
    rec = CM.Records()
    g1 = I.grid_side(128)
    G1 = native.Graph(g1.n, g1.src, g1.dst, g1.w)
    CM.generate_records(G1, I.Workload(g1, 21), 0, 40, 30, 4000, seed=1, rec=rec, state_base=0)
    g2 = I.rmat_s(13)
    G2 = native.Graph(g2.n, g2.src, g2.dst, g2.w)
    CM.generate_records(G2, I.Workload(g2, 22), I.max_out_degree_vertex(g2), 40, 10, 4000, seed=2,
                        rec=rec, state_base=1000)
    # interleave the two graphs' states so both appear on each side of the split
    rec.state = [s % 1000 for s in rec.state]
    cm, hist, r = CM.fit(rec, epochs=300)
    say(f"  records {len(rec.X)}, loss {hist[0]:.3f} -> {hist[-1]:.4f}, held-out {r}")
    assert hist[-1] < 0.5 * hist[0]
    assert r["policy_ms"] < r["always_incremental_ms"]
    assert r["policy_regret_ms"] < r["heuristic_regret_ms"]


def test_slab_scale_output_trains_and_its_picks_hold_up():
    """The slab-scale output: graphs of several densities (R-MAT with edge factors 4, 16 and
    48, road-like grids) are built at slab scales 0.5, 1 and 2 and timed on the same work;
    the MLP (HIP kernels) trains on these records beside timing records, and on graphs it
    has not seen its picks cost no more than the default scale (10 % slack for timing noise)."""
    say("case: cost-model slab scale")
    rec = CM.Records()
    g0 = I.rmat_s(12)
    G0 = native.Graph(g0.n, g0.src, g0.dst, g0.w)
    CM.generate_records(G0, I.Workload(g0, 23), I.max_out_degree_vertex(g0), 12, 10, 2000, seed=3,
                        rec=rec, state_base=0, algos=["bfs", "wcc"])
    train = [I.rmat_graph(sc, ef, 100 + 7 * sc + ef) for sc in (13, 14) for ef in (4, 16, 48)]
    train += [I.grid_side(side, seed=200 + side) for side in (96, 128)]
    CM.slab_scale_records(train, seed=5, rec=rec, state_base=100)
    n_train = len(rec.X)
    test = [I.rmat_graph(14, ef, 300 + ef) for ef in (8, 32)] + [I.grid_side(112, seed=400)]
    CM.slab_scale_records(test, seed=6, rec=rec, state_base=1000)
    X, T, M, _, _, _, state = rec.arrays()
    assert M[:, 2].sum() == len(train) + len(test) and np.isfinite(T).all()
    cm, hist, _ = CM.fit(rec, holdout_frac=len(test) / len(rec.X) + 1e-6, epochs=300)
    sr = CM.scale_regret(cm, rec, range(n_train, len(rec.X)))
    picks = cm.slab_scale(np.stack(rec.X[n_train:]))
    say(f"  loss {hist[0]:.3f} -> {hist[-1]:.4f}; held-out picks {picks.tolist()}, {sr}; "
        f"labels {[2 ** v for v in rec.slab_scale[n_train:]]}")
    assert hist[-1] < 0.5 * hist[0]
    assert set(picks.tolist()) <= set(CM.SLAB_SCALES)
    assert sr["policy_ms"] <= 1.1 * sr["default_ms"]
