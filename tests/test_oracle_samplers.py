"""Pins of the oracle's other tree samplers (Section "Tree-Sampling
techniques for graphBpp", Alg. alg-hybrid): the DFS-tree property and closed
forms for the randomized DFS, scipy's minimum spanning tree for Kruskal on
random weights, the coin of the hybrid, and the balancing invariants that
hold for every spanning tree."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle
from oracle import brute
from paper_2311_00869_amd import synth

SAMPLERS = ("bfs", "rdfs", "hybrid", "kruskal")


def _ancestors(parent, v):
    out = set()
    while parent[v] >= 0:
        v = int(parent[v])
        out.add(v)
    return out


@pytest.mark.parametrize("gi", range(3))
def test_rdfs_is_a_depth_first_tree(gi):
    g = [synth.random_small(150, 400, 3, p_pos=0.5),
         synth.chung_lu(300, 900, 2.1, 2, p_pos=0.6),
         synth.erdos_renyi_connected(120, 600, 0.7, 5)][gi]
    for t in range(4):
        level, parent, _ = oracle.tree(g, 9, t, "rdfs")
        rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        for u, v in zip(rows, g.col):
            if u < v and parent[u] != v and parent[v] != u:
                # no cross edges: one endpoint is an ancestor of the other
                assert u in _ancestors(parent, v) or v in _ancestors(parent, u)
        for v in range(g.n):
            if parent[v] >= 0:
                assert level[v] == level[parent[v]] + 1


def test_rdfs_closed_forms():
    # on K_n every vertex is adjacent to all unvisited ones, so the search is
    # a path through the vertices in increasing key order
    g = synth.complete_graph(12, -1)
    salt = oracle.tree_salt(4, 3)
    level, parent, _ = oracle.tree(g, 4, 3, "rdfs")
    order = sorted(range(12), key=lambda u: oracle.vertex_key(salt, u))
    assert [int(level[u]) for u in order] == list(range(12))
    assert all(parent[order[i]] == order[i - 1] for i in range(1, 12))
    # on a cycle the search walks all the way round: depth n - 1 (BFS: n / 2)
    c = synth.cycle_graph(31, (0, 4))
    assert oracle.tree(c, 1, 0, "rdfs")[0].max() == 30
    assert oracle.tree(c, 1, 0, "bfs")[0].max() == 15


def _kruskal_ranks(g, salt):
    """Rank of every undirected edge in Kruskal's order (weight, then its
    position in the sorted edge list), as a symmetric sparse matrix."""
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    keep = rows < g.col
    u, v = rows[keep], g.col[keep]
    keys = [(oracle.kruskal_weight(salt, int(a), int(b)), i) for i, (a, b) in enumerate(zip(u, v))]
    rank = np.empty(len(keys))
    rank[np.argsort([w * 2**32 + i for w, i in keys], kind="stable")] = np.arange(1, len(keys) + 1)
    return sp.coo_matrix((rank, (u, v)), shape=(g.n, g.n)).tocsr(), u, v


@pytest.mark.parametrize("gi", range(3))
def test_kruskal_is_the_minimum_spanning_forest(gi):
    g = [synth.random_small(150, 400, 3, p_pos=0.5),
         synth.chung_lu(300, 900, 2.1, 2, p_pos=0.6),
         synth.complete_graph(9, 1)][gi]
    for t in range(3):
        salt = oracle.tree_salt(2, t)
        W, _, _ = _kruskal_ranks(g, salt)
        mst = csg.minimum_spanning_tree(W).tocoo()
        want = {(min(a, b), max(a, b)) for a, b in zip(mst.row, mst.col)}
        _, parent, _ = oracle.tree(g, 2, t, "kruskal")
        got = {(min(v, int(parent[v])), max(v, int(parent[v]))) for v in range(g.n) if parent[v] >= 0}
        assert got == want
        # rooted at each component's smallest vertex
        ncomp, anchor = oracle.components(g)
        assert all(parent[a] == -1 for a in np.unique(anchor))


def test_hybrid_coin_and_trees():
    coins = [oracle.hybrid_coin(oracle.tree_salt(0, t)) for t in range(4000)]
    assert abs(np.mean(coins) - 0.5) < 0.03  # 4 sigma of a fair coin
    g = synth.random_small(200, 500, 8, p_pos=0.5)
    seen = set()
    for t in range(12):
        z = oracle.hybrid_coin(oracle.tree_salt(6, t))
        seen.add(z)
        want = oracle.tree(g, 6, t, "rdfs" if z else "bfs")
        got = oracle.tree(g, 6, t, "hybrid")
        assert all(np.array_equal(a, b) for a, b in zip(got, want))
    assert seen == {0, 1}


@pytest.mark.parametrize("sampler", SAMPLERS)
def test_every_sampler_balances_and_bounds_the_index(sampler):
    # the sweep's own cross-checks (cycle walk = propagated state, Harary
    # 2-colouring, |E| - |V| + c non-tree edges) hold for any spanning tree,
    # and no tree can beat the exact index
    for seed in range(3):
        g = synth.random_small(14, 30, seed, p_pos=0.5)
        fi = brute.frustration_index(g)
        r = oracle.sweep(g, seed, 0, 30, checks=True, sampler=sampler)
        assert r.best[0] >= fi
    g = synth.planted_er(200, 600, 0.0, 3)
    r = oracle.sweep(g, 1, 0, 10, checks=True, sampler=sampler)
    assert r.best[0] == 0 and len(r.cloud) == 1
    with pytest.raises(KeyError):
        oracle.sweep(g, 1, 0, 1, sampler="prim")
