"""Pins of the switch-list and cloud-statistics oracle (oracle/switches.py).

Checked against Theorem t:HararyCut (switching the listed edges leaves a
graph that 2-colours with every negative edge across, and only non-tree
edges are switched), closed forms (planted splits, trees, single cycles,
all-negative complete graphs) and invariants of the sums."""
from collections import deque

import numpy as np
import pytest

import oracle
from oracle import switches
from paper_2311_00869_amd import synth


def _two_colourable_after_switch(g, switched):
    """Independent BFS: flip the listed edges, then look for a side
    assignment with positive edges inside and negative edges across."""
    flip = {(int(u), int(v)) for u, v in switched}
    rp, col, sg = g.row_ptr, g.col, g.sign
    side = np.full(g.n, -1, np.int64)
    for r in range(g.n):
        if side[r] >= 0:
            continue
        side[r] = 0
        q = deque([r])
        while q:
            u = q.popleft()
            for k in range(rp[u], rp[u + 1]):
                v = int(col[k])
                s = int(sg[k])
                if (min(u, v), max(u, v)) in flip:
                    s = -s
                want = side[u] if s > 0 else 1 - side[u]
                if side[v] < 0:
                    side[v] = want
                    q.append(v)
                elif side[v] != want:
                    return False
    return True


GRAPHS = [
    synth.config_small(0),
    synth.random_small(120, 300, 4, p_pos=0.5),  # several components
    synth.complete_graph(8, -1),
    synth.chung_lu(500, 1500, 2.1, 3, p_pos=0.7),
]


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_switch_lists_balance_the_graph(gi):
    g = GRAPHS[gi]
    r = oracle.sweep(g, 11, 0, 6, checks=False)
    for t in range(6):
        edges, s = switches.tree_switch_list(g, 11, t)
        assert s == int(r.trees[t, 0])
        assert np.all(edges[:, 0] < edges[:, 1])
        assert np.all(np.diff(edges[:, 0].astype(np.int64) * g.n + edges[:, 1]) > 0)
        assert _two_colourable_after_switch(g, edges)
        # only non-tree edges are switched
        _, parent, state = oracle.tree(g, 11, t)
        for u, v in edges:
            assert parent[u] != v and parent[v] != u
        # the walk's list is the set of edges the propagated state frustrates
        assert np.array_equal(switches.frustrated_edges(g, state), edges)


def test_closed_forms():
    # all-negative K_n, state all +1: every edge is frustrated
    g = synth.complete_graph(9, -1)
    assert len(switches.frustrated_edges(g, np.ones(9, np.int8))) == 36
    # a planted split frustrates exactly the flipped edges
    g = synth.planted_er(400, 1500, 0.1, 5)
    st = np.where(g.meta["side"] == 1, -1, 1)
    assert len(switches.frustrated_edges(g, st)) == g.meta["flipped"]
    # a tree has nothing to switch; a cycle with an odd number of negative
    # edges has exactly one edge switched per spanning tree
    t = synth.random_tree(60, 2)
    vm, es = switches.sweep_stats(t, 1, 0, 5)
    assert es.sum() == 0 and len(es) == 59
    c = synth.cycle_graph(21, (0, 4, 7))
    vm, es = switches.sweep_stats(c, 3, 0, 40)
    assert es.sum() == 40 and es.max() < 40


def test_sweep_stats_invariants():
    g = synth.random_small(150, 260, 9, p_pos=0.55)
    K = 30
    vm, es = switches.sweep_stats(g, 7, 0, K)
    r = oracle.sweep(g, 7, 0, K, checks=False)
    # every switched edge is counted once per tree: the sums match the switches
    assert es.sum() == int(r.switches.sum())
    # anchors are +1 in every canonical state
    ncomp, anchor = oracle.components(g)
    assert np.all(vm[np.unique(anchor)] == 0)
    assert vm.max() <= K and es.max() <= K
    # vertex counts agree with the canonical words the cloud keys are made from
    want = np.zeros(g.n, np.int64)
    for t in range(K):
        _, _, st = oracle.tree(g, 7, t)
        w = oracle.canonical_words(g, st)
        bits = (w[np.arange(g.n) // 64] >> (np.arange(g.n) % 64).astype(np.uint64)) & np.uint64(1)
        want += bits.astype(np.int64)
    assert np.array_equal(vm, want)
    # splitting the tree range adds up
    a = switches.sweep_stats(g, 7, 0, 11)
    b = switches.sweep_stats(g, 7, 11, K)
    assert np.array_equal(a[0] + b[0], vm) and np.array_equal(a[1] + b[1], es)


def test_planted_balanced_graph_stats():
    # a balanced planted graph: every tree reaches the planted split
    g = synth.planted_er(300, 900, 0.0, 8)
    K = 12
    vm, es = switches.sweep_stats(g, 2, 0, K)
    side = g.meta["side"].astype(np.int64)
    assert es.sum() == 0
    assert np.array_equal(vm, K * (side != side[0]))
