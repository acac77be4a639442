"""Full-size parity: the 16M-vertex / 64M-edge graph in the launch
configuration the benchmark times, and the 1M-vertex planted power-law graph,
against per-tree results the CPU oracle wrote ahead of time
(tests/golden/make_fullsize_golden.py)."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import alg_scale
from paper_2311_00869_amd import synth, tune

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2311_00869_amd.frustration")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, f"fullsize_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


def _check(G, gold, schedule):
    G.set_schedule(**schedule)
    G.cloud_reset()
    t0, t1, seed = gold["t0"], gold["t1"], gold["seed"]
    sw = G.sweep_range(t0, t1, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
    want = np.array(gold["trees"], dtype=np.uint64)
    assert np.array_equal(sw, want[:, 0]), (schedule, sw, want[:, 0])
    assert np.array_equal(G.cloud(), np.array(gold["cloud"], dtype=np.uint64)), schedule
    assert list(G.min_frustration()) == gold["best"], schedule


def test_large_graph_bench_configuration():
    # trees 0..129: one full 128-tree pass of the benchmark's kernel (both
    # tree words of every lane, the 256-workgroup grid and the 1,024-vertex
    # root chunks of this size) plus two trees of the next pass.  All 130
    # states are distinct, so the cloud's entries (keyed, with their first
    # tree) give every tree's key
    gold = _golden("large")
    assert gold["t1"] - gold["t0"] >= 130
    g = synth.config_large(0)
    assert (g.n, g.nnz) == (gold["n"], gold["nnz"])
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=256)
    sched = tune.default_schedule(G.n, G.nnz)
    assert sched["path"] == 5
    _check(G, gold, sched)
    assert G.get_schedule()["path"] == 5
    _check(G, gold, dict(path=5, block=1024, grid=128))
    _check(G, gold, dict(path=4, block=1024))
    _check(G, gold, dict(path=3, block=512, heavy=256, batch=1))
    cloud = np.array(gold["cloud"], dtype=np.uint64)
    trees = np.array(gold["trees"], dtype=np.uint64)
    assert len(cloud) == len(trees)
    ft = cloud[:, 4].astype(np.int64) - gold["t0"]
    assert np.array_equal(cloud[:, 0:2], trees[ft, 1:3])
    # every tree's frustrated edges, recounted by the exact counter from its state
    words, s0 = G.tree_state(gold["seed"], gold["t0"])
    got = int(G.count(torch.from_numpy(words.view(np.int64))).item())
    assert got == s0 == gold["trees"][0][0]
    _check_bounded(G, gold, fmax=1, chunk=1)
    # more trees than the oracle can run here: the bounded cloud is the
    # F_max best states by (S, first tree) of the unbounded one, same counts
    G.set_schedule(path=4, block=1024)
    G.cloud_reset()
    G.sweep_range(0, 192, 7)
    full = G.cloud()
    C = fr.BoundedCloud(50, staging=256)
    G.sweep_bounded(C, 0, 192, 7, chunk=64)
    best = full[np.lexsort((full[:, 4], full[:, 3]))][:50]
    best = best[np.lexsort((best[:, 1], best[:, 0]))]
    assert np.array_equal(C.entries(), best)
    trees, dropped = C.stats()
    assert trees == 192 and dropped >= len(full) - 50
    C.close()
    # cloud statistics and the switch list at full size, by properties
    G.cloud_reset()
    sw = G.sweep_range(0, 64, 3, tree_switches=True)
    G.cloud_reset()
    vm, es = G.sweep_stats(0, 64, 3)
    assert int(es.sum()) == int(sw.sum())
    assert int(vm[0]) == 0 and int(vm.max()) <= 64 and int(es.max()) <= 64
    lst, k = G.switch_list(torch.from_numpy(words.view(np.int64)).cuda())
    assert k == gold["trees"][0][0] == len(lst)
    lst = lst.cpu().numpy().astype(np.int64)
    assert np.all(np.diff(lst[:, 0] * g.n + lst[:, 1]) > 0)
    pick = np.random.default_rng(0).choice(len(lst), 2000, replace=False)
    bit = lambda x: (words[x // 64] >> (x % 64).astype(np.uint64)) & np.uint64(1)
    u, v = lst[pick, 0], lst[pick, 1]
    rows = [np.searchsorted(g.col[g.row_ptr[a]:g.row_ptr[a + 1]], b) + g.row_ptr[a]
            for a, b in zip(u, v)]
    neg = (g.sign[rows] < 0).astype(np.uint64)
    assert np.all(neg ^ bit(u) ^ bit(v) == 1)
    _check_graphl_large(g, G)
    G.close()


def _check_graphl_large(g, G):
    """graphL on the 16M graph: one step against the oracle on sampled rows
    (the hubs among them), then 500 steps with the overflow policy."""
    from oracle import graphl as ogl
    R = 8
    gamma0 = torch.from_numpy(synth.graphl_init(g.n, R, 5)).cuda()
    step = G.graphl_step(gamma0, 0.001).cpu().numpy()
    deg = np.diff(g.row_ptr)
    rows = np.concatenate([np.argsort(deg)[-16:],
                           np.random.default_rng(1).choice(g.n, 2000, replace=False)])
    g0 = gamma0.cpu().numpy()
    want = g0[rows].astype(np.float64) - 0.001 * ogl.grad_rows(g, g0, rows)
    err = np.abs(step[rows] - want).max() / np.abs(want).max()
    assert err <= 1e-4, err
    a, sa = G.graphl_descend(gamma0, 500, 0.001)
    assert torch.isfinite(a).all()
    assert int(sa().max()) > 0  # the hub component needed rescaling
    b, sb = G.graphl_descend(gamma0, 500, 0.001, rescale_log2=32)
    ta = torch.ldexp(a.double(), sa().double())
    tb = torch.ldexp(b.double(), sb().double())
    assert torch.equal(ta, tb)
    del ta, tb
    ca = G.round_count(a)
    assert torch.equal(ca, G.round_count(b))
    assert int(ca.max()) <= G.m


def _check_bounded(G, gold, fmax, chunk):
    """Alg. alg-scale on the oracle's stored per-tree results."""
    t0, t1, seed = gold["t0"], gold["t1"], gold["seed"]
    c = alg_scale.bounded_cloud(gold["trees"], fmax, t0)
    want = np.array(alg_scale.as_rows(c), dtype=np.uint64).reshape(-1, 5)
    C = fr.BoundedCloud(fmax, staging=G.cloud_capacity)
    G.sweep_bounded(C, t0, t1, seed, chunk=chunk)
    assert np.array_equal(C.entries(), want)
    assert C.min_frustration() == alg_scale.frustration_index(c)
    C.close()


def test_planted_powerlaw_all_paths():
    gold = _golden("planted")
    g = synth.config_planted_powerlaw(0)
    assert (g.n, g.nnz) == (gold["n"], gold["nnz"])
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=256)
    for sched in [tune.default_schedule(G.n, G.nnz), dict(path=2, block=1024),
                  dict(path=3, block=1024, batch=8), dict(path=3, block=256, batch=3, heavy=64),
                  dict(path=4, block=1024), dict(path=4, block=512),
                  dict(path=5, block=1024), dict(path=5, block=512)]:
        _check(G, gold, sched)
    # the planted split frustrates exactly the flipped edges
    side = g.meta["side"]
    idx = np.flatnonzero(side == 1)
    w = np.zeros(G.nwords, np.uint64)
    np.bitwise_or.at(w, idx // 64, np.left_shift(np.uint64(1), (idx % 64).astype(np.uint64)))
    assert int(G.count(torch.from_numpy(w.view(np.int64))).item()) == gold["planted_flipped"]
    G.set_schedule(path=4, block=1024)
    _check_bounded(G, gold, fmax=3, chunk=3)
    G.close()


def test_planted_ten_thousand_trees_in_one_sweep():
    # the planted configuration as benchmarked: 10^4 trees in one sweep on the
    # automatic schedule.  Its first 32 trees against the oracle, and over all
    # of them what Alg. alg-index and Eq. eq-cloud fix: the counts add up to
    # K, each key carries one switch count (the readout checks every slot),
    # each state's S is the switch count of its first tree, and the minimum
    # is the smallest switch count at its first tree
    gold = _golden("planted")
    g = synth.config_planted_powerlaw(0)
    K = 10_000
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=K)
    G.set_schedule(**tune.default_schedule(G.n, G.nnz))
    sw = G.sweep_range(0, K, gold["seed"], tree_switches=True).cpu().numpy().astype(np.uint64)
    want = np.array(gold["trees"], dtype=np.uint64)
    assert np.array_equal(sw[gold["t0"]:gold["t1"]], want[:, 0])
    cloud = G.cloud()
    assert 1 <= len(cloud) == G.cloud_size() <= K
    assert int(cloud[:, 2].sum()) == K
    assert np.array_equal(cloud[:, 3], sw[cloud[:, 4].astype(np.int64)])
    assert len(np.unique(cloud[:, 4])) == len(cloud)
    s, t = G.min_frustration()
    assert s == int(sw.min()) and t == int(np.argmax(sw == sw.min()))
    # every tree's switch count is one its state carries: the trees whose
    # switch count no first tree has are repeats of some state with it
    assert set(sw.tolist()) == set(cloud[:, 3].tolist())
    G.close()


def test_uneven_batch_full_size_sampled():
    """The full uneven batch (4,096 graphs x 64 trees, the benchmark's batch
    leg) in one fi_batch_sweep, checked on 256 sampled graphs against the
    oracle's per-graph results (tests/golden/make_batch_golden.py), and on
    every graph against what holds at any size."""
    path = os.path.join(GOLDEN, "batch_uneven.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        gold = json.load(f)
    G, K = gold["graphs"], gold["trees_per_graph"]
    graphs = synth.config_batch_parallel(G, 0)
    B = fr.BatchGraph(graphs, cloud_capacity_per_graph=K)
    ms = [g.nnz // 2 for g in graphs]
    del graphs
    for sched in [tune.default_batch_schedule(B), dict(block=256, path=4), dict(block=1024, path=1)]:
        B.set_schedule(**sched)
        mn, ds = B.sweep(K, gold["seed"])
        mn, ds = mn.cpu().numpy(), ds.cpu().numpy()
        for g, n, nnz, s, first, distinct in gold["rows"]:
            assert int(B.nnz_offsets[g + 1] - B.nnz_offsets[g]) == nnz
            assert (mn[g, 0], mn[g, 1], ds[g]) == (s, first, distinct), (sched, g)
        assert np.all((ds >= 1) & (ds <= K))
        assert np.all((mn[:, 1] >= 0) & (mn[:, 1] < K))
        assert np.all(mn[:, 0] <= np.asarray(ms))
    B.close()
