"""Parity of the HIP sweep with the CPU oracle (bit-exact): per-tree switch
counts, canonical states, the cloud, the minimum, input validation, and
invariance to schedule, splitting and repetition."""
import numpy as np
import pytest
import torch

import oracle
from paper_2311_00869_amd import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2311_00869_amd.frustration")

SCHEDULES = [
    dict(path=1, block=256), dict(path=1, block=512), dict(path=1, block=1024),
    dict(path=2, block=256), dict(path=2, block=1024),
    dict(path=3, block=256, batch=1), dict(path=3, block=512, heavy=32, batch=3),
    dict(path=3, block=1024, heavy=64, batch=8), dict(path=3, block=256, batch=5, grid=40),
    dict(path=4, block=1024), dict(path=4, block=512), dict(path=4, block=256, grid=40),
    dict(path=5, block=1024), dict(path=5, block=512), dict(path=5, block=256, grid=40),
]


def _graph(g, cap=4096):
    return fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=cap)


def _cases():
    return {
        "small1000": synth.config_small(0),
        "disconnected": synth.random_small(300, 280, 3, p_pos=0.6),
        "isolated": synth.chung_lu(2000, 3000, 2.1, 5, p_pos=0.7),
        "fig_neg": synth.figure_graph([-1, 1, -1, 1, -1]),
        "k7neg": synth.complete_graph(7, -1),
        "cycle": synth.cycle_graph(33, (0, 5, 9)),
        "tree": synth.random_tree(200, 1),
        "empty": synth.isolated_vertices(65),
    }


def _sched_ok(g, s):
    if s["path"] == 1 and g.n * 12 + 32768 > 160 * 1024:
        return False
    return True


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_tree_switches_and_cloud_match_oracle(name):
    g = _cases()[name]
    K, seed = 96, 12345
    ref = oracle.sweep(g, seed, 0, K, checks=True)
    G = _graph(g)
    for s in SCHEDULES:
        if not _sched_ok(g, s):
            continue
        G.set_schedule(**s)
        G.cloud_reset()
        sw = G.sweep_range(0, K, seed, tree_switches=True)
        got = sw.cpu().numpy().astype(np.uint64)
        assert np.array_equal(got, ref.trees[:, 0]), (name, s)
        cloud = G.cloud()
        assert np.array_equal(cloud, ref.cloud), (name, s)
        assert G.min_frustration() == ref.best, (name, s)
    G.close()


@pytest.mark.parametrize("name", ["small1000", "disconnected", "isolated", "cycle"])
def test_canonical_states_match_oracle(name):
    g = _cases()[name]
    G = _graph(g)
    seed = 77
    for t in [0, 1, 5, 31]:
        _, _, st = oracle.tree(g, seed, t)
        want = oracle.canonical_words(g, st)
        for s in SCHEDULES[::3]:
            if not _sched_ok(g, s):
                continue
            G.set_schedule(**s)
            words, sw = G.tree_state(seed, t)
            assert np.array_equal(words, want), (name, t, s)
            assert sw == oracle.count(g, st)
    # tree_state leaves the cloud alone
    assert G.cloud_size() == 0
    G.close()


def test_split_sweep_and_repeat_are_identical():
    g = synth.erdos_renyi_connected(3000, 12000, 0.75, 9)
    G = _graph(g, cap=2048)
    G.sweep(300, 4)
    whole = G.cloud()
    best = G.min_frustration()
    G.cloud_reset()
    for a, b in [(0, 17), (17, 200), (200, 300)]:
        G.sweep_range(a, b, 4)
    assert np.array_equal(G.cloud(), whole)
    assert G.min_frustration() == best
    G.cloud_reset()
    G.set_schedule(path=3, block=256)
    G.sweep(300, 4)
    assert np.array_equal(G.cloud(), whole)
    ref = oracle.sweep(g, 4, 0, 300, checks=False)
    assert np.array_equal(whole, ref.cloud)
    G.close()


def test_cloud_checkpoint_resume():
    g = synth.config_small(2)
    G = _graph(g, cap=1024)
    G.sweep_range(0, 150, 8)
    saved = G.cloud()
    G.cloud_reset()
    G.cloud_load(saved)
    G.sweep_range(150, 400, 8)
    resumed = G.cloud()
    ref = oracle.sweep(g, 8, 0, 400, checks=False)
    assert np.array_equal(resumed, ref.cloud)
    assert G.min_frustration() == ref.best
    G.close()


def test_capacity_error_is_reported():
    g = synth.config_small(0)
    G = _graph(g, cap=4)
    G.sweep(200, 1)
    with pytest.raises(fr.FrustrationError) as e:
        G.status()
    assert e.value.code == -8
    G.cloud_reset()
    G.status()
    G.close()


@pytest.mark.parametrize("B", [1, 7, 64, 70])
def test_exact_count_matches_oracle(B):
    # groups of 64 states share one pass over the edge list: one state, a
    # partial group, a full one, and a full one plus a partial one
    g = synth.chung_lu(5000, 40000, 2.3, 3, p_pos=0.8)
    G = _graph(g)
    rng = np.random.default_rng(B)
    states = np.where(rng.random((B, g.n)) < 0.5, 1, -1).astype(np.int8)
    words = np.zeros((B, G.nwords), np.uint64)
    for b in range(B):
        idx = np.flatnonzero(states[b] < 0)
        np.bitwise_or.at(words[b], idx // 64, np.left_shift(np.uint64(1), (idx % 64).astype(np.uint64)))
    got = G.count(torch.from_numpy(words.view(np.int64))).cpu().numpy()
    want = [oracle.count(g, states[b]) for b in range(B)]
    assert got.tolist() == want
    G.close()


def test_planted_counter_pin():
    # the planted split frustrates exactly the flipped edges
    g = synth.chung_lu(20000, 100000, 2.1, 6, planted_flip=0.05)
    G = _graph(g)
    side = g.meta["side"]
    idx = np.flatnonzero(side == 1)
    w = np.zeros(G.nwords, np.uint64)
    np.bitwise_or.at(w, idx // 64, np.left_shift(np.uint64(1), (idx % 64).astype(np.uint64)))
    got = int(G.count(torch.from_numpy(w.view(np.int64))).item())
    assert got == g.meta["flipped"]
    G.close()


def _bad(kind):
    g = synth.random_small(10, 20, 1, p_pos=0.5, connected=True)
    rp, col, sg = g.row_ptr.copy(), g.col.copy(), g.sign.copy()
    if kind == "sign":
        sg[3] = 0
    elif kind == "selfloop":
        v = 2
        col[rp[v]] = v
        col[rp[v]:rp[v + 1]] = np.sort(col[rp[v]:rp[v + 1]])
    elif kind == "dup":
        v = 4
        col[rp[v] + 1] = col[rp[v]]
    elif kind == "unsorted":
        v = 5
        col[rp[v]:rp[v + 1]] = col[rp[v]:rp[v + 1]][::-1].copy()
    elif kind == "asym":
        sg[7] = -sg[7]
    elif kind == "range":
        col[0] = 99
    elif kind == "rowptr":
        rp[3] = rp[4] + 1
    return synth.SignedCSR(10, rp, col, sg)


@pytest.mark.parametrize("kind", ["sign", "selfloop", "dup", "unsorted", "asym", "range", "rowptr"])
def test_validation_matches_oracle(kind):
    g = _bad(kind)
    want = oracle.validate(g)
    assert want != 0
    with pytest.raises(fr.FrustrationError) as e:
        _graph(g)
    assert e.value.code == want


def test_powerlaw_multi_tile_all_paths():
    # several tiles, ragged tails, hubs above the heavy threshold
    g = synth.chung_lu(60000, 300000, 2.1, 11, p_pos=0.8)
    K, seed = 24, 99
    ref = oracle.sweep(g, seed, 0, K, checks=False)
    G = _graph(g, cap=256)
    for s in [dict(path=2, block=256), dict(path=2, block=1024),
              dict(path=3, block=256, heavy=64, batch=1), dict(path=3, block=512, heavy=512, batch=8),
              dict(path=3, block=1024, heavy=4096, batch=3), dict(path=3, block=512, batch=7, grid=17),
              dict(path=4, block=1024), dict(path=4, block=256, grid=17),
              dict(path=5, block=1024), dict(path=5, block=256, grid=17)]:
        G.set_schedule(**s)
        G.cloud_reset()
        sw = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
        assert np.array_equal(sw, ref.trees[:, 0]), s
        assert np.array_equal(G.cloud(), ref.cloud), s
    G.close()


@pytest.mark.parametrize("n,m", [(250000, 1000000), (60000, 480000), (40000, 200000), (30000, 100000),
                                 (8000, 32000), (3000, 15000)])
def test_automatic_schedule_past_the_crossover(n, m):
    # path 0 takes the 128-tree multi-tree kernel (1,024-thread workgroups, the
    # grid sized to the graph) once n + m/2 exceeds 135,000, else one tree per
    # workgroup (256 threads on the sparse 30,000-vertex graph; the last two
    # keep the tree in LDS, with 1,024 and 512 threads); 8 trees leave most of
    # the pass's lanes idle
    g = synth.chung_lu(n, m, 2.3, 21, p_pos=0.85)
    K, seed = 8, 5
    ref = oracle.sweep(g, seed, 0, K, checks=False)
    G = _graph(g, cap=64)
    G.set_schedule(path=0, block=256)
    sw = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
    assert np.array_equal(sw, ref.trees[:, 0])
    assert np.array_equal(G.cloud(), ref.cloud)
    G.close()


def _row_boundaries():
    """One graph whose rows sit on every class and chunk boundary of the
    multi-tree pull: cliques with rows of 31, 32, 33, 63, 64 and 65 edges, and
    stars with hubs of 2,048 and 2,049 edges (their leaves are rows of one
    edge), joined into one component by a path, with mixed signs."""
    rng = np.random.default_rng(7)
    us, vs = [], []
    off = 0
    anchors = []
    for k in (32, 33, 34, 64, 65, 66):
        for a in range(k):
            for b in range(a + 1, k):
                us.append(off + a)
                vs.append(off + b)
        anchors.append(off)
        off += k
    for leaves in (2048, 2049):
        for i in range(1, leaves + 1):
            us.append(off)
            vs.append(off + i)
        anchors.append(off)
        off += leaves + 1
    for a, b in zip(anchors[:-1], anchors[1:]):
        us.append(a + 1)
        vs.append(b + 1)
    sign = np.where(rng.random(len(us)) < 0.6, 1, -1)
    return synth.csr_from_edges(off, us, vs, sign)


def test_row_class_and_chunk_boundaries_all_paths():
    g = _row_boundaries()
    K, seed = 70, 31
    ref = oracle.sweep(g, seed, 0, K, checks=False)
    G = _graph(g, cap=128)
    for s in [dict(path=1, block=256), dict(path=2, block=512), dict(path=3, block=256, heavy=64, batch=2),
              dict(path=4, block=1024), dict(path=4, block=256, grid=9), dict(path=5, block=512),
              dict(path=5, block=1024, grid=13)]:
        G.set_schedule(**s)
        G.cloud_reset()
        sw = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
        assert np.array_equal(sw, ref.trees[:, 0]), s
        assert np.array_equal(G.cloud(), ref.cloud), s
    G.close()


def test_automatic_grid_several_passes_and_a_ragged_one():
    # a 100,000-vertex graph takes 128 trees per pass on a grid of 64
    # workgroups: 200 trees are one full pass and one of 72
    g = synth.chung_lu(100000, 500000, 2.3, 0, p_pos=0.85)
    K, seed = 200, 17
    ref = oracle.sweep(g, seed, 0, K, checks=False)
    G = _graph(g, cap=256)
    sw = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
    assert np.array_equal(sw, ref.trees[:, 0])
    assert np.array_equal(G.cloud(), ref.cloud)
    assert G.min_frustration() == ref.best
    G.close()


def test_autotune_keeps_a_schedule_with_oracle_results():
    # every candidate runs (each gives the same trees); the kept one still does
    from paper_2311_00869_amd import tune
    g = synth.chung_lu(20000, 100000, 2.3, 4, p_pos=0.85)
    K, seed = 40, 23
    ref = oracle.sweep(g, seed, 0, K, checks=False)
    G = _graph(g, cap=64)
    best, results = tune.autotune(G, trees=128, save=False)
    assert len(results) == len(tune.candidates(G.n, G.nnz))
    assert G.get_schedule()["path"] == best["path"]
    G.cloud_reset()
    sw = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
    assert np.array_equal(sw, ref.trees[:, 0]), best
    assert np.array_equal(G.cloud(), ref.cloud), best
    G.close()


def _deep_graphs():
    """Graphs whose BFS trees are thousands of levels deep: a 10,000-vertex
    path and a 2 x 5,000 ladder (5,001 fundamental cycles), both with shuffled
    vertex ids, and a 120 x 120 grid; mixed signs."""
    rng = np.random.default_rng(3)
    out = {}
    n = 10000
    perm = rng.permutation(n)
    out["path10000"] = synth.csr_from_edges(n, perm[:-1], perm[1:],
                                            np.where(rng.random(n - 1) < 0.7, 1, -1))
    L = 5000
    perm = rng.permutation(2 * L)
    a = np.arange(L)
    us = np.concatenate([a[:-1], a[:-1] + L, a])
    vs = np.concatenate([a[1:], a[1:] + L, a + L])
    out["ladder2x5000"] = synth.csr_from_edges(2 * L, perm[us], perm[vs],
                                               np.where(rng.random(us.size) < 0.8, 1, -1))
    k = 120
    idx = np.arange(k * k).reshape(k, k)
    us = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    vs = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    out["grid120"] = synth.csr_from_edges(k * k, us, vs, np.where(rng.random(us.size) < 0.6, 1, -1))
    return out


@pytest.mark.parametrize("name", ["path10000", "ladder2x5000", "grid120"])
def test_deep_trees_every_schedule(name):
    # BFS trees deeper than any fixed level field of a few bits: every
    # schedule, the automatic one included, matches the oracle
    g = _deep_graphs()[name]
    K, seed = 70, 41
    ref = oracle.sweep(g, seed, 0, K, checks=True)
    G = _graph(g, cap=128)
    for s in [dict(path=0, block=256), dict(path=1, block=256), dict(path=1, block=1024),
              dict(path=2, block=256), dict(path=3, block=256, batch=4),
              dict(path=3, block=1024, batch=1), dict(path=4, block=1024, grid=16),
              dict(path=5, block=1024, grid=16), dict(path=5, block=512)]:
        if not _sched_ok(g, s):
            continue
        G.set_schedule(**s)
        G.cloud_reset()
        sw = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
        assert np.array_equal(sw, ref.trees[:, 0]), (name, s)
        assert np.array_equal(G.cloud(), ref.cloud), (name, s)
        assert G.min_frustration() == ref.best, (name, s)
        G.status()
    # one tree's canonical state through fi_tree_state
    words, s0 = G.tree_state(seed, 5)
    _, _, state = oracle.tree(g, seed, 5)
    assert np.array_equal(words, oracle.canonical_words(g, state))
    assert s0 == int(ref.trees[5, 0])
    G.close()


def test_tree_order_blocks_match_oracle_and_plain_path():
    # more than one pass on a graph whose main component has 10^5 vertices:
    # the multi-tree path takes each block of up to 16,384 trees in its own
    # order (by root distance to the core); 16,500 trees are two blocks.
    # Every tree's switch count equals the plain one-tree-at-a-time path's
    # and, on sampled trees, the oracle's; the clouds agree
    g = synth.chung_lu(100000, 500000, 2.3, 3, p_pos=0.85)
    K, seed = 16500, 77
    G = _graph(g, cap=K)
    G.set_schedule(path=3, block=1024, batch=8)
    plain = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
    plain_cloud = G.cloud()
    for s in (dict(path=5, block=1024), dict(path=4, block=1024)):
        G.set_schedule(**s)
        G.cloud_reset()
        sw = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
        assert np.array_equal(sw, plain), s
        assert np.array_equal(G.cloud(), plain_cloud), s
    for t in (0, 1, 127, 8000, 16383, 16384, 16499):
        ref = oracle.sweep(g, seed, t, t + 1, checks=False)
        assert int(ref.trees[0, 0]) == int(plain[t]), t
    G.close()


def test_tree_order_on_a_component_above_2_20_vertices():
    # a main component of 1.42M vertices (above 2^20): the roots that order
    # each block of trees come from inverting the key (the smallest key held
    # by a component vertex) instead of scanning the component.  300 trees
    # are three passes; every tree's switch count equals the plain path's
    # and, on sampled trees, the oracle's
    g = synth.chung_lu(1500000, 6000000, 2.3, 3, p_pos=0.85)
    K, seed = 300, 77
    G = _graph(g, cap=K)
    G.set_schedule(path=3, block=1024, batch=8)
    plain = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
    plain_cloud = G.cloud()
    G.set_schedule(path=5, block=1024)
    G.cloud_reset()
    sw = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
    assert np.array_equal(sw, plain)
    assert np.array_equal(G.cloud(), plain_cloud)
    for t in (0, 151, 299):
        ref = oracle.sweep(g, seed, t, t + 1, checks=False)
        assert int(ref.trees[0, 0]) == int(plain[t]), t
    G.close()


def test_dense_graph_every_row_split_matches_oracle():
    # a complete graph on 2,200 vertices with random signs: every row is longer
    # than the 2,048 edges at which the multi-tree pull splits a row, so the
    # split-row minima use 2,200 rows, past half of their table.  The
    # workspace is carved from memory that held zeros (a zero minimum would
    # win every row if a row were not initialised).  Per-tree switches and
    # clouds on paths 5 and 4 equal the oracle's
    n = 2200
    iu, ju = np.triu_indices(n, 1)
    rng = np.random.default_rng(5)
    sg = np.where(rng.random(iu.size) < 0.6, 1, -1).astype(np.int8)
    g = synth.csr_from_edges(n, iu, ju, sg)
    K, seed = 200, 9
    ref = oracle.sweep(g, seed, 0, K, checks=False)
    import ctypes
    size = ctypes.c_size_t(0)
    assert fr.load_library().fi_graph_workspace_size(g.n, len(g.col), K, ctypes.byref(size)) == 0
    rp = torch.from_numpy(g.row_ptr).cuda()
    cl = torch.from_numpy(g.col).cuda()
    sgn = torch.from_numpy(g.sign).cuda()
    z = torch.zeros(size.value + 256, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    del z
    G = fr.Graph(rp, cl, sgn, cloud_capacity=K)
    for s in (dict(path=5, block=1024), dict(path=4, block=1024)):
        G.set_schedule(**s)
        G.cloud_reset()
        sw = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
        assert np.array_equal(sw, ref.trees[:, 0]), s
        assert np.array_equal(G.cloud(), ref.cloud), s
    G.close()


def test_autotune_picks_the_multi_tree_pass_past_the_crossover():
    # on a 100,000-vertex graph with the sweep's own tree count, the tuner
    # ranks the candidates on full passes and keeps the 128-tree path
    from paper_2311_00869_amd import tune
    g = synth.chung_lu(100000, 500000, 2.3, 0, p_pos=0.85)
    G = _graph(g, cap=1024)
    best, results = tune.autotune(G, trees=1024, save=False)
    assert best["path"] == 5, sorted((round(t, 4), s["path"], s["block"], s["grid"]) for t, s in results)[:5]
    G.close()


def test_phase_log_records_every_pass_and_changes_nothing():
    # the multi-tree kernel's phase log: one record per grid barrier from
    # workgroup 0, the passes' inserts counted, results unchanged
    g = synth.chung_lu(100000, 500000, 2.3, 0, p_pos=0.85)
    K, seed = 300, 5
    G = _graph(g, cap=K)
    G.set_schedule(path=5, block=1024)
    want = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy()
    G.cloud_reset()
    G.phase_log(4096)
    got = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy()
    recs = G.phase_records()
    G.phase_log(0)
    assert np.array_equal(got, want)
    phases = [p for p, _, _ in recs]
    assert phases.count(8) == 3 and phases.count(1) == 3  # three passes of up to 128 trees
    assert all(us >= 0 for _, _, us in recs)
    levels = {lv for p, lv, _ in recs if p == 5}
    assert min(levels) == 1 and max(levels) >= 3
    G.close()


def test_gather_probe_runs_and_clamps_indices():
    # the measurement aid reads records only: indices past the table are
    # clamped to its last record, and the sink keeps its value (the loads'
    # xor would have to equal one 32-bit constant to store)
    from paper_2311_00869_amd import frustration as fr
    g = synth.chung_lu(100000, 500000, 2.3, 0, p_pos=0.85)
    col = torch.from_numpy(np.ascontiguousarray(g.col, dtype=np.int32)).cuda()
    rec = torch.zeros(g.n * 16, dtype=torch.int32, device="cuda")
    sink = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    fr.probe_gather(col, rec, sink)
    far = torch.full((1000,), 0x7FFFFFFF, dtype=torch.int32, device="cuda")
    small = torch.zeros(16 * 16, dtype=torch.int32, device="cuda")
    fr.probe_gather(far, small, sink)
    fr.probe_gather(col[:0], rec, sink)
    torch.cuda.synchronize()
    assert int(sink.item()) == 7
