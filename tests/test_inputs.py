"""Generator checks: counts, no self-loops or duplicates, skew, grid sizes, batch shapes."""
import numpy as np
import torch

from paper_2305_17813_amd import inputs as I


def test_mix64_matches_reference_definition():
    xs = [0, 1, 12345, 2**63 - 1, 2**64 - 1]
    got = I.mix64(torch.tensor([I._s64(x) for x in xs], dtype=torch.int64))
    for x, g in zip(xs, got.tolist()):
        assert g & ((1 << 64) - 1) == I.mix64_py(x)
    # SplitMix64 with state 0: first output is the finaliser of 0x9E3779B97F4A7C15
    assert I.mix64_py(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF


def test_below_range_and_uniformity():
    r = I.draws(5, 1, 0, 200000)
    v = I.below(r, 100)
    assert int(v.min()) == 0 and int(v.max()) == 99
    counts = torch.bincount(v, minlength=100).double()
    assert float(counts.std() / counts.mean()) < 0.05


def test_er_graph_shape():
    g = I.er_4k()
    assert g.n == 4096 and g.m == 32768
    k = g.keys()
    assert torch.unique(k).numel() == g.m
    assert int((g.src == g.dst).sum()) == 0
    assert int(g.w.min()) >= 1 and int(g.w.max()) <= 100


def test_rmat_skew_and_dedupe():
    g = I.rmat_s(14)
    assert torch.unique(g.keys()).numel() == g.m
    assert int((g.src == g.dst).sum()) == 0
    assert 0.8 * 16 * 2**14 < g.m <= 16 * 2**14
    deg = torch.bincount(g.src, minlength=g.n).double()
    assert float(deg.max()) > 50 * float(deg.mean())  # power-law hubs


def test_grid_counts():
    side = 64
    g = I.grid_side(side)
    e_full = 2 * side * (side - 1)
    kept = e_full - int(round(0.1 * e_full))
    short = int(round(0.01 * kept))
    assert g.m == 2 * (kept + short)
    k = g.keys()
    assert torch.unique(k).numel() == g.m
    # symmetric, with equal weights on both arcs
    rev = I.key_of(g.dst, g.src)
    order = torch.argsort(k)
    pos = torch.searchsorted(k[order], rev)
    assert bool((k[order][pos] == rev).all())
    assert bool((g.w[order][pos] == g.w).all())


def test_grid_full_size_edge_count_formula():
    # 4096 x 4096 grid: 33,546,240 edges, 10% removed -> 30,191,616 (the stated sizes)
    e_full = 2 * 4096 * 4095
    assert e_full == 33546240
    assert e_full - int(round(0.1 * e_full)) == 30191616


def test_workload_batches():
    g = I.er_4k()
    wl = I.Workload(g, 3)
    before = wl.keys.clone()
    s, d, w = wl.insert_batch(1024)
    k = I.key_of(s, d)
    assert k.numel() == 1024 and torch.unique(k).numel() == 1024
    assert not bool(I.is_member(before, k).any())
    assert int((s == d).sum()) == 0
    assert bool((w == I.arc_weight(s, d, 100, g.wseed)).all())
    s2, d2 = wl.delete_batch(1024)
    k2 = I.key_of(s2, d2)
    assert torch.unique(k2).numel() == 1024
    assert bool(I.is_member(torch.sort(torch.cat([before, k])).values, k2).all())
    qs, qd = wl.query_batch(4096)
    pres = I.is_member(wl.keys, I.key_of(qs, qd))
    assert int(pres.sum()) == 2048


def test_workload_undirected_batches():
    g = I.grid_side(32)
    wl = I.Workload(g, 9)
    s, d, w = wl.insert_batch(100)
    assert s.numel() == 200
    assert bool((w[:100] == w[100:]).all())
    s, d = wl.delete_batch(50)
    assert s.numel() == 100


def test_generators_deterministic():
    a = I.rmat_s(10)
    b = I.rmat_s(10)
    assert torch.equal(a.src, b.src) and torch.equal(a.dst, b.dst) and torch.equal(a.w, b.w)
