"""Exact frustration index by enumeration (oracle; test infrastructure only).

Fr(Sigma) is the least number of edges whose sign must change for the graph
to become balanced (Definition def-SignedGraph).  By Theorem t:HararyCut
(item 4) every balanced result corresponds to a vertex 2-colouring, and the
edges to change are exactly those frustrated by it, so Fr is the minimum over
all +1/-1 vertex states of the frustrated-edge count.  One vertex per
connected component can be fixed to +1 (flipping a whole component changes no
edge's frustration), leaving 2^(n-c) states.
"""
from __future__ import annotations

import numpy as np


def _components(g):
    comp = -np.ones(g.n, dtype=np.int64)
    for s in range(g.n):
        if comp[s] >= 0:
            continue
        comp[s] = s
        stack = [s]
        while stack:
            u = stack.pop()
            for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
                if comp[v] < 0:
                    comp[v] = s
                    stack.append(v)
    return comp


def frustration_index(g, return_state: bool = False):
    """Minimum frustrated-edge count over all vertex states (n - c <= 24)."""
    comp = _components(g)
    free = [v for v in range(g.n) if comp[v] != v]  # anchors fixed to +1
    k = len(free)
    if k > 24:
        raise ValueError("too many free vertices for enumeration")
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    keep = rows < g.col
    u, v, neg = rows[keep], g.col[keep], (g.sign[keep] < 0).astype(np.uint8)
    bitpos = -np.ones(g.n, dtype=np.int64)
    bitpos[free] = np.arange(k)
    states = np.arange(1 << k, dtype=np.uint32)

    def bit(x):
        if bitpos[x] < 0:
            return np.zeros_like(states, dtype=np.uint8)
        return ((states >> np.uint32(bitpos[x])) & 1).astype(np.uint8)

    total = np.zeros(states.size, dtype=np.int32)
    for a, b, ng in zip(u, v, neg):
        total += (bit(a) ^ bit(b) ^ ng).astype(np.int32)
    best = int(total.min())
    if not return_state:
        return best
    s = int(np.argmin(total))
    state = np.ones(g.n, dtype=np.int8)
    for x in free:
        if (s >> bitpos[x]) & 1:
            state[x] = -1
    return best, state
