"""Parity of the batched sweep of many uneven graphs with the CPU oracle run
on each graph alone (bit-exact minimum and distinct-state count per graph),
its independence from block size and repetition, HIP graph capture replayed
against the eager result, and its input checks."""
import numpy as np
import pytest
import torch

import oracle
from paper_2311_00869_amd import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2311_00869_amd.frustration")


def _mixed():
    """Both size classes (in-LDS up to 6,144 vertices, workspace above) and
    the degenerate cases: edgeless, a tree, odd cycles, several components."""
    return [
        synth.config_small(0),
        synth.isolated_vertices(65),
        synth.figure_graph([-1, 1, -1, 1, -1]),
        synth.complete_graph(7, -1),
        synth.random_tree(200, 1),
        synth.cycle_graph(33, (0, 5, 9)),
        synth.random_small(300, 280, 3, p_pos=0.6),
        synth.random_small(1000, 300, 7, p_pos=0.5),  # hundreds of small components
        synth.chung_lu(2000, 3000, 2.1, 5, p_pos=0.7),
        synth.erdos_renyi_connected(6144, 20000, 0.75, 11),
        synth.erdos_renyi_connected(6145, 15000, 0.8, 12),
        synth.erdos_renyi_connected(20000, 60000, 0.85, 13),
        synth.isolated_vertices(1),
        synth.complete_graph(65, -1),  # rows of exactly 64 edges: one per chunk
        synth.complete_graph(66, 1),   # rows of 65: one wave per row
    ]


def _expect(graphs, K, seed, clouds=None):
    mins, distinct = [], []
    for g in graphs:
        r = oracle.sweep(g, seed, 0, K, checks=False)
        mins.append(r.best)
        distinct.append(len(r.cloud))
        if clouds is not None:
            clouds.append(r.cloud)
    return np.asarray(mins, np.int64), np.asarray(distinct, np.int64)


def test_mixed_batch_matches_oracle_per_graph():
    graphs = _mixed()
    K, seed = 40, 4242
    want_clouds = []
    want_min, want_distinct = _expect(graphs, K, seed, want_clouds)
    B = fr.BatchGraph(graphs, cloud_capacity_per_graph=K)
    # path 1: one workgroup per tree; path 4: 64 trees per workgroup pass
    for path in (1, 4):
        for block in (256, 512, 1024):
            B.set_schedule(block=block, path=path)
            mn, ds = B.sweep(K, seed)
            assert np.array_equal(mn.cpu().numpy(), want_min), (path, block)
            assert np.array_equal(ds.cpu().numpy(), want_distinct), (path, block)
            # every graph's whole cloud: keys, counts, switch counts, first trees
            for i in range(len(graphs)):
                assert np.array_equal(B.cloud(i), want_clouds[i]), (path, block, i)
    # more than one pass of 64 trees per graph, and a partial one
    K2 = 150
    w2_min, w2_distinct = _expect(graphs, K2, seed + 1)
    B2 = fr.BatchGraph(graphs, cloud_capacity_per_graph=K2)
    for path in (1, 4):
        B2.set_schedule(block=512, path=path)
        mn, ds = B2.sweep(K2, seed + 1)
        assert np.array_equal(mn.cpu().numpy(), w2_min), path
        assert np.array_equal(ds.cpu().numpy(), w2_distinct), path
    B2.close()
    B.set_schedule(block=256)
    # a second call starts from empty clouds
    mn, ds = B.sweep(K, seed)
    assert np.array_equal(mn.cpu().numpy(), want_min)
    assert np.array_equal(ds.cpu().numpy(), want_distinct)
    B.close()


def test_uneven_batch_sampled_graphs():
    """128 graphs of the uneven-batch recipe (n 100..12,000): every graph
    against the oracle."""
    G, K, seed = 128, 16, 99
    graphs = synth.config_batch(G, seed=3, n_lo=100, n_hi=12000)
    want_min, want_distinct = _expect(graphs, K, seed)
    B = fr.BatchGraph(graphs, cloud_capacity_per_graph=K)
    for path in (1, 4):
        B.set_schedule(block=512, grid=96, path=path)
        mn, ds = B.sweep(K, seed)
        assert np.array_equal(mn.cpu().numpy(), want_min), path
        assert np.array_equal(ds.cpu().numpy(), want_distinct), path
    B.close()


def test_batch_equals_single_graph_handles():
    graphs = _mixed()[:6]
    K, seed = 24, 5
    B = fr.BatchGraph(graphs, cloud_capacity_per_graph=K)
    mn, ds = B.sweep(K, seed)
    for i, g in enumerate(graphs):
        H = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=K)
        H.sweep(K, seed)
        assert tuple(mn[i].tolist()) == H.min_frustration()
        assert int(ds[i]) == H.cloud_size()
        H.close()
    B.close()


def test_hip_graph_capture_replays_match_eager():
    graphs = _mixed()
    K = 32
    B = fr.BatchGraph(graphs, cloud_capacity_per_graph=K)
    eager = {}
    for seed in (1, 2):
        mn, ds = B.sweep(K, seed)
        eager[seed] = (mn.clone(), ds.clone())
    mn = torch.zeros((B.G, 2), dtype=torch.int64, device="cuda")
    ds = torch.zeros(B.G, dtype=torch.int64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.sweep_into(K, 1, mn, ds)  # warm once outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        B.sweep_into(K, 1, mn, ds)
    for rep in range(4):
        mn.fill_(-7)
        ds.fill_(-7)
        graph.replay()
        torch.cuda.synchronize()
        B.status()
        assert torch.equal(mn, eager[1][0]), rep
        assert torch.equal(ds, eager[1][1]), rep
        # eager work with another seed between the replays
        m2, d2 = B.sweep(K, 2)
        assert torch.equal(m2, eager[2][0]) and torch.equal(d2, eager[2][1])
    del graph
    B.close()


def test_batch_capacity_error():
    graphs = [synth.config_small(0), synth.complete_graph(7, -1)]
    B = fr.BatchGraph(graphs, cloud_capacity_per_graph=1)
    with pytest.raises(fr.FrustrationError) as e:
        B.sweep(64, 3)
    assert e.value.code == -8
    B.close()


def test_batch_validation_codes():
    good = synth.config_small(0)
    bad = synth.complete_graph(5, -1)
    sg = bad.sign.copy()
    sg[0] = -sg[0]  # one direction of an edge flipped: asymmetric
    with pytest.raises(fr.FrustrationError) as e:
        fr.BatchGraph([good, (bad.row_ptr, bad.col, sg)])
    assert e.value.code == -2
    sg = bad.sign.copy()
    sg[3] = 0
    with pytest.raises(fr.FrustrationError) as e:
        fr.BatchGraph([(bad.row_ptr, bad.col, sg), good])
    assert e.value.code == -5
    col = bad.col.copy()
    col[0] = 99
    with pytest.raises(fr.FrustrationError) as e:
        fr.BatchGraph([good, (bad.row_ptr, col, bad.sign)])
    assert e.value.code == -1
    # a graph above the per-graph vertex limit
    with pytest.raises(fr.FrustrationError):
        fr.BatchGraph([synth.isolated_vertices(1_000_001)])
    # single-graph calls refuse a batch handle
    B = fr.BatchGraph([good])
    assert B.lib.fi_sweep(B.handle, 4, 1, None) == -1
    assert B.lib.fi_min_frustration(B.handle, None, None, None) == -1
    B.close()


def test_deep_graphs_in_a_batch():
    # BFS trees of several thousand levels (a path, a ladder, a grid) beside
    # small graphs, on both batch schedules
    from test_sweep_gpu import _deep_graphs
    graphs = list(_deep_graphs().values()) + [synth.config_small(0), synth.cycle_graph(33, (0, 5, 9))]
    K, seed = 40, 8
    want_min, want_distinct = _expect(graphs, K, seed)
    B = fr.BatchGraph(graphs, cloud_capacity_per_graph=K)
    for path, block in ((1, 256), (1, 1024), (4, 512), (0, 1024)):
        B.set_schedule(block=block, path=path)
        mn, ds = B.sweep(K, seed)
        assert np.array_equal(mn.cpu().numpy(), want_min), (path, block)
        assert np.array_equal(ds.cpu().numpy(), want_distinct), (path, block)
    B.status()
    B.close()
