"""graphL in float64 numpy (oracle; test infrastructure only).

Follows Section "graphL: optimization formulation":
  * Eq. eq-loss_imbalance_new: L = sum over edges (i, j) of (1 - e_ij G_i G_j) / 2,
    with every undirected edge counted once (the only reading under which the
    printed gradient -1/2 sum_j G_j e_ij is the derivative of L);
  * the gradient dL/dG_i = -1/2 sum over neighbours j of G_j e_ij;
  * Alg. alg-gradient: G <- G - alpha * dL/dG for a fixed number of updates,
    then theta_i = +1 where G_i >= 0 and -1 otherwise (the comparison of its
    final loop), and frustration = sum over edges of (1 - e_ij theta_i theta_j)/2.
Restarts are the columns of a [n, R] array and are independent.
"""
from __future__ import annotations

import numpy as np


def edges_of(g):
    """Undirected edges (u < v) and their signs as float64."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    keep = rows < g.col
    return rows[keep], g.col[keep].astype(np.int64), g.sign[keep].astype(np.float64)


def loss(g, gamma):
    """L_r for every restart column r of gamma [n, R]."""
    u, v, e = edges_of(g)
    G = np.asarray(gamma, dtype=np.float64)
    return ((1.0 - e[:, None] * G[u] * G[v]) / 2.0).sum(axis=0)


def grad(g, gamma):
    """dL/dG [n, R] = -1/2 * sum over neighbours j of e_ij G_j."""
    u, v, e = edges_of(g)
    G = np.asarray(gamma, dtype=np.float64)
    out = np.zeros_like(G)
    np.add.at(out, u, -0.5 * e[:, None] * G[v])
    np.add.at(out, v, -0.5 * e[:, None] * G[u])
    return out


def grad_rows(g, gamma, rows):
    """dL/dG for the given vertices only, [len(rows), R], from their CSR rows
    (the same gradient, for sampling outputs of a large graph)."""
    G = np.asarray(gamma)
    out = np.zeros((len(rows), G.shape[1]), np.float64)
    for k, i in enumerate(rows):
        a, b = int(g.row_ptr[i]), int(g.row_ptr[i + 1])
        nb = g.col[a:b].astype(np.int64)
        e = g.sign[a:b].astype(np.float64)
        out[k] = -0.5 * (e[:, None] * G[nb].astype(np.float64)).sum(axis=0)
    return out


def descent(g, gamma0, steps: int, alpha: float):
    """The update loop of Alg. alg-gradient; returns the final G (float64)."""
    G = np.asarray(gamma0, dtype=np.float64).copy()
    for _ in range(steps):
        G = G - alpha * grad(g, G)
    return G


def round_states(gamma):
    """theta = +1 where G >= 0, else -1 (int8, [n, R])."""
    return np.where(np.asarray(gamma) >= 0, 1, -1).astype(np.int8)


def frustration(g, theta):
    """sum over edges of (1 - e theta_i theta_j) / 2 per restart (exact integers)."""
    u, v, e = edges_of(g)
    th = np.asarray(theta, dtype=np.int64)
    return ((1 - e.astype(np.int64)[:, None] * th[u] * th[v]) // 2).sum(axis=0)


def signed_adjacency(g):
    """Dense signed adjacency A (A_ij = e_ij), float64, for small n."""
    A = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    A[rows, g.col] = g.sign
    return A
