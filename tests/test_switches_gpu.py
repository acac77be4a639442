"""Parity of the switch lists (Sigma' as edges to switch) and of the cloud
statistics with the oracle: exact edge lists for tree states, random states
and rounded graphL states, truncation at the caller's capacity, and the
per-vertex / per-edge tree counts of a sweep."""
import numpy as np
import pytest
import torch

import oracle
from oracle import graphl as ogl
from oracle import switches
from paper_2311_00869_amd import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2311_00869_amd.frustration")


def _graphs():
    return [
        ("small", synth.config_small(0)),
        ("components", synth.random_small(400, 330, 4, p_pos=0.5)),
        ("complete9", synth.complete_graph(9, -1)),
        ("powerlaw", synth.chung_lu(3000, 9000, 2.1, 5, p_pos=0.7)),
        ("er20k", synth.erdos_renyi_connected(20000, 60000, 0.85, 13)),  # several tiles, ragged
        ("edgeless", synth.isolated_vertices(70)),
    ]


def _words(state_pm1):
    n = len(state_pm1)
    w = np.zeros((n + 63) // 64, np.uint64)
    idx = np.flatnonzero(np.asarray(state_pm1) < 0)
    np.bitwise_or.at(w, idx // 64, np.left_shift(np.uint64(1), (idx % 64).astype(np.uint64)))
    return torch.from_numpy(w.view(np.int64)).cuda()


@pytest.mark.parametrize("name,g", _graphs(), ids=[n for n, _ in _graphs()])
def test_edge_and_switch_lists(name, g):
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=64)
    assert np.array_equal(G.edge_list().cpu().numpy(), switches.upper_edges(g))
    seed = 17
    for t in (0, 1, 5):
        want, s = switches.tree_switch_list(g, seed, t)
        words, s_gpu = G.tree_state(seed, t)
        got, k = G.switch_list(torch.from_numpy(words.view(np.int64)).cuda())
        assert k == s == s_gpu, (name, t)
        assert np.array_equal(got.cpu().numpy(), want), (name, t)
    rng = np.random.default_rng(5)
    for _ in range(3):
        st = np.where(rng.random(g.n) < 0.5, -1, 1).astype(np.int8)
        want = switches.frustrated_edges(g, st)
        got, k = G.switch_list(_words(st))
        assert k == len(want)
        assert np.array_equal(got.cpu().numpy(), want)
        # a short output buffer keeps the first edges and reports the count
        cap = len(want) // 3
        got, k = G.switch_list(_words(st), cap=cap)
        assert k == len(want)
        assert np.array_equal(got.cpu().numpy(), want[:cap])
    G.close()


def test_graphl_flip_lists():
    g = synth.config_small(0)
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=16)
    R = 6
    gamma = synth.graphl_init(g.n, R, 3)
    gamma[::97, 0] = 0.0  # the rounding rule at zero
    gamma[1::89, 1] = -0.0
    counts, bits = G.round_count(torch.from_numpy(gamma).cuda(), return_bits=True)
    theta = ogl.round_states(gamma)
    for r in range(R):
        want = switches.frustrated_edges(g, theta[:, r])
        got, k = G.switch_list(bits[r])
        assert k == len(want) == int(counts[r])
        assert np.array_equal(got.cpu().numpy(), want), r
    G.close()


@pytest.mark.parametrize("name,g", _graphs()[:5], ids=[n for n, _ in _graphs()[:5]])
def test_sweep_stats_match_oracle(name, g):
    K, seed = 90, 23
    want_v, want_e = switches.sweep_stats(g, seed, 0, K)
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=K)
    for sched in (dict(path=0), dict(path=4, block=512), dict(path=1, block=256),
                  dict(path=5, block=1024)):
        if sched["path"] == 1 and g.n > 12000:
            continue
        G.set_schedule(**sched)
        G.cloud_reset()
        # two calls accumulate; the second starts mid-pass
        vm, es = G.sweep_stats(0, 37, seed)
        G.sweep_stats(37, K, seed, vm, es)
        assert np.array_equal(vm.cpu().numpy(), want_v), (name, sched)
        assert np.array_equal(es.cpu().numpy(), want_e), (name, sched)
        # the trees entered the cloud as with a plain sweep
        r = oracle.sweep(g, seed, 0, K, checks=False) if sched["path"] == 0 else r
        assert np.array_equal(G.cloud(), r.cloud)
    G.close()
