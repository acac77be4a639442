"""The balanced state as a list of edges to switch, and cloud statistics.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

* ``tree_switch_list``: the edges Alg. alg-balance switches for tree t, taken
  from the literal fundamental-cycle walk (``oracle.balance``); the paper's
  concluding remarks name this list as the method's output besides the index.
* ``frustrated_edges``: the edges a +1/-1 state frustrates, sign * s_u * s_v
  = -1, which is what Alg. alg-gradient flips after rounding a graphL state.
* ``sweep_stats``: over trees t0 .. t1-1, per vertex the number of trees
  whose canonical state (each component's smallest vertex at +1) puts it at
  -1, and per edge the number of trees whose walk switches it.  Each state of
  the cloud is thereby weighted by its count C (Eq. eq-cloud).

Edges are the undirected pairs (u, v) with u < v in increasing order.
"""
from __future__ import annotations

import numpy as np

import oracle


def upper_edges(g):
    """int32 [m, 2]: (u, v), u < v, in increasing (u, v) order."""
    rp = np.asarray(g.row_ptr, np.int64)
    col = np.asarray(g.col, np.int64)
    u = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(rp))
    keep = u < col
    return np.stack([u[keep], col[keep]], axis=1).astype(np.int32)


def _upper_mask(g):
    rp = np.asarray(g.row_ptr, np.int64)
    u = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(rp))
    return u < np.asarray(g.col, np.int64)


def tree_switch_list(g, seed: int, t: int):
    """(edges switched by Alg. alg-balance on tree t as int32 [S, 2], S)."""
    level, parent, _ = oracle.tree(g, seed, t)
    s, flip = oracle.balance(g, level, parent)
    edges = upper_edges(g)[flip[_upper_mask(g)] != 0]
    if len(edges) != s:
        raise RuntimeError("walk flipped an edge in one direction only")
    return edges, s


def frustrated_edges(g, state_pm1):
    """int32 [k, 2]: the edges with sign * s_u * s_v = -1."""
    st = np.asarray(state_pm1, np.int64)
    rp = np.asarray(g.row_ptr, np.int64)
    u = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(rp))
    col = np.asarray(g.col, np.int64)
    sg = np.asarray(g.sign, np.int64)
    hit = (u < col) & (sg * st[u] * st[col] == -1)
    return np.stack([u[hit], col[hit]], axis=1).astype(np.int32)


def sweep_stats(g, seed: int, t0: int, t1: int):
    """(vertex_minus int64[n], edge_switched int64[m]) over trees t0 .. t1-1."""
    _, anchor = oracle.components(g)
    upper = _upper_mask(g)
    vminus = np.zeros(g.n, np.int64)
    eswitch = np.zeros(int(upper.sum()), np.int64)
    for t in range(t0, t1):
        level, parent, state = oracle.tree(g, seed, t)
        _, flip = oracle.balance(g, level, parent)
        canon = state.astype(np.int64) * state[anchor].astype(np.int64)
        vminus += canon == -1
        eswitch += flip[upper] != 0
    return vminus, eswitch
