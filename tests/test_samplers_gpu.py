"""Parity of the other tree samplers (randomized DFS, the RDFS-BFS hybrid of
Alg. alg-hybrid, Kruskal on random weights) with the oracle: per-tree switch
counts, the whole cloud and the canonical states, bit-exact, in LDS and in
workspace slots, plus the sampler's argument checks."""
import numpy as np
import pytest
import torch

import oracle
from paper_2311_00869_amd import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2311_00869_amd.frustration")


def _graphs():
    return [
        ("small", synth.config_small(0)),
        ("components", synth.random_small(400, 330, 4, p_pos=0.5)),
        ("complete9", synth.complete_graph(9, -1)),
        ("cycle33", synth.cycle_graph(33, (0, 5, 9))),
        ("tree", synth.random_tree(200, 1)),
        ("powerlaw", synth.chung_lu(2000, 3000, 2.1, 5, p_pos=0.7)),
        ("isolated", synth.isolated_vertices(70)),
        ("er20k", synth.erdos_renyi_connected(20000, 60000, 0.85, 13)),  # workspace slots
    ]


@pytest.mark.parametrize("sampler", ["rdfs", "hybrid", "kruskal"])
@pytest.mark.parametrize("name,g", _graphs(), ids=[n for n, _ in _graphs()])
def test_sampler_matches_oracle(name, g, sampler):
    K, seed = 64, 77
    ref = oracle.sweep(g, seed, 0, K, checks=True, sampler=sampler)
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=K)
    G.set_sampler(sampler)
    assert G.get_sampler() == sampler
    scheds = [dict(path=2, block=1024), dict(path=4, block=512)]
    if g.n <= 8000:  # the tree fits LDS
        scheds.insert(0, dict(path=1, block=256))
    for sched in scheds:
        G.set_schedule(**sched)
        G.cloud_reset()
        sw = G.sweep_range(0, K, seed, tree_switches=True).cpu().numpy().astype(np.uint64)
        assert np.array_equal(sw, ref.trees[:, 0]), (name, sampler, sched)
        assert np.array_equal(G.cloud(), ref.cloud), (name, sampler, sched)
        assert G.min_frustration() == ref.best
    for t in (0, 3):
        words, s = G.tree_state(seed, t)
        _, _, st = oracle.tree(g, seed, t, sampler)
        assert np.array_equal(words, oracle.canonical_words(g, st)), (name, sampler, t)
        assert s == int(ref.trees[t, 0])
    G.close()


def test_sampler_arguments():
    g = synth.config_small(0)
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=16)
    for bad in (-1, 4, 99):
        with pytest.raises(fr.FrustrationError) as e:
            G.set_sampler(bad)
        assert e.value.code == -1
    G.set_sampler("rdfs")
    with pytest.raises(fr.FrustrationError) as e:
        G.sweep_stats(0, 4, 1)
    assert e.value.code == -1
    # switching back to BFS restores the default results
    G.set_sampler("bfs")
    G.cloud_reset()
    sw = G.sweep_range(0, 16, 5, tree_switches=True).cpu().numpy().astype(np.uint64)
    assert np.array_equal(sw, oracle.sweep(g, 5, 0, 16, checks=False).trees[:, 0])
    G.close()


def test_samplers_with_bounded_cloud_and_switch_lists():
    g = synth.chung_lu(3000, 6000, 2.2, 8, p_pos=0.65)
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=128)
    G.set_sampler("hybrid")
    r = oracle.sweep(g, 3, 0, 200, checks=False, sampler="hybrid")
    from oracle import alg_scale, switches
    C = fr.BoundedCloud(10, staging=128)
    G.sweep_bounded(C, 0, 200, 3, chunk=50)
    want = np.array(alg_scale.as_rows(alg_scale.bounded_cloud(r.trees, 10)), np.uint64)
    assert np.array_equal(C.entries(), want)
    C.close()
    G.set_sampler("kruskal")
    words, s = G.tree_state(3, 1)
    lst, k = G.switch_list(torch.from_numpy(words.view(np.int64)).cuda())
    level, parent, _ = oracle.tree(g, 3, 1, "kruskal")
    flip = oracle.balance(g, level, parent)[1]
    want = switches.upper_edges(g)[flip[switches._upper_mask(g)] != 0]
    assert k == s == len(want)
    assert np.array_equal(lst.cpu().numpy(), want)
    G.close()
