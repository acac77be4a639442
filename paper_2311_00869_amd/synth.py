"""Seeded synthetic signed graphs.

This module only *makes inputs*: simple undirected signed graphs in symmetric
CSR form (row_ptr int32[n+1], col int32[2m], sign int8[2m], rows sorted by
column, no self-loops, no duplicates, both directions carrying the same sign)
plus the seeded float arrays graphL starts from.  It holds none of the
frustration method's arithmetic, and both the CPU oracle and the HIP path read
exactly the arrays it returns.

The shapes stand in for the paper's real signed networks (SNAP, Konect and
Amazon graphs, Section "Signed Graph Benchmarks" and Tables tab-SNAPdata,
tab-KonectData, tab-AmazonCharac), which are not available here: heavy-tailed
degree distributions, 31-95 % positive edges, up to ~10^7 vertices.
"""
from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass
class SignedCSR:
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[nnz]
    sign: np.ndarray     # int8[nnz], +1 / -1
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def edges(self):
        """Undirected edge list (u < v) with signs, in CSR order."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        keep = rows < self.col
        return rows[keep], self.col[keep].astype(np.int64), self.sign[keep]


def csr_from_edges(n: int, u, v, sign, meta=None) -> SignedCSR:
    """Symmetric sorted CSR from an undirected edge list (u != v, unique pairs).

    Each pair is stored in both directions with the same sign.  Sorting packs
    (row, col, negative-flag) into one int64 so one sort orders everything.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    neg = (np.asarray(sign) < 0).astype(np.int64)
    if u.size and (np.any(u == v) or u.min() < 0 or v.min() < 0 or max(u.max(), v.max()) >= n):
        raise ValueError("edge list has self-loops or out-of-range endpoints")
    rows = np.concatenate([u, v])
    cols = np.concatenate([v, u])
    negs = np.concatenate([neg, neg])
    del u, v, neg
    keys = (rows * n + cols) * 2 + negs
    del rows, cols, negs
    keys.sort(kind="stable" if keys.size < 1 << 20 else "quicksort")
    negbit = (keys & 1).astype(np.int8)
    keys >>= 1
    rows = keys // n
    col = (keys - rows * n).astype(np.int32)
    del keys
    counts = np.bincount(rows, minlength=n)
    del rows
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    sign_arr = (1 - 2 * negbit).astype(np.int8)
    return SignedCSR(n=n, row_ptr=row_ptr.astype(np.int32), col=col, sign=sign_arr,
                     meta=dict(meta or {}))


def _unique_pairs(n, a, b):
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    ok = lo != hi
    return np.unique(lo[ok] * np.int64(n) + hi[ok])


def _fill_unique(rng, n, m, draw, have=None):
    """Draw endpoint pairs with ``draw(k)`` until ``m`` distinct non-loop pairs exist.

    ``have`` holds pairs that must be kept (encoded lo*n+hi).  Returns the
    encoded pairs, exactly m of them, in random order of acceptance.
    """
    keys = np.zeros(0, dtype=np.int64) if have is None else np.asarray(have, dtype=np.int64)
    keys = np.unique(keys)
    base = keys.size
    if base > m:
        raise ValueError("more forced edges than m")
    rounds = 0
    while keys.size < m:
        need = m - keys.size
        k = int(need * 1.08) + 1024
        a, b = draw(k)
        new = _unique_pairs(n, a, b)
        new = np.setdiff1d(new, keys, assume_unique=True)
        if new.size > need:
            pick = rng.choice(new.size, size=need, replace=False)
            new = new[np.sort(pick)]
        keys = np.union1d(keys, new)
        rounds += 1
        if rounds > 200:
            raise RuntimeError("could not reach m unique edges")
    return keys


def erdos_renyi_connected(n: int, m: int, p_pos: float, seed, extra_meta=None) -> SignedCSR:
    """Connected random signed graph: a random Hamiltonian path (n-1 edges) plus
    uniformly random distinct non-loop pairs up to m edges; each sign is +1 with
    probability p_pos, independently."""
    if m < n - 1 or m > n * (n - 1) // 2:
        raise ValueError("m out of range")
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n).astype(np.int64)
    path = _unique_pairs(n, perm[:-1], perm[1:])

    def draw(k):
        return rng.integers(0, n, size=k, dtype=np.int64), rng.integers(0, n, size=k, dtype=np.int64)

    keys = _fill_unique(rng, n, m, draw, have=path)
    u, v = keys // n, keys % n
    sign = np.where(rng.random(keys.size) < p_pos, 1, -1).astype(np.int8)
    meta = {"recipe": "path+uniform", "n": n, "m": m, "p_pos": p_pos, "seed": str(seed)}
    meta.update(extra_meta or {})
    return csr_from_edges(n, u, v, sign, meta)


def _power_law_endpoints(rng, n, gamma, k):
    """k vertex ids with P(i) ~ (i+1)^(-1/(gamma-1)), by inverting the CDF of the
    continuous density x^(-a) on [1, n+1) and flooring (a = 1/(gamma-1))."""
    a = 1.0 / (gamma - 1.0)
    e = 1.0 - a
    top = (n + 1.0) ** e
    u = rng.random(k)
    x = (1.0 + u * (top - 1.0)) ** (1.0 / e)
    i = np.floor(x).astype(np.int64) - 1
    np.clip(i, 0, n - 1, out=i)
    return i


def chung_lu(n: int, m: int, gamma: float, seed, p_pos: float | None = 0.85,
             planted_flip: float | None = None) -> SignedCSR:
    """Chung-Lu style power-law graph with exactly m unique non-loop edges.

    Endpoints are drawn independently with weight ~ (i+1)^(-1/(gamma-1)) and
    pairs are rejected if they are loops or repeats.  Signs:
      * p_pos given, planted_flip None: +1 with probability p_pos, iid;
      * planted_flip given: each vertex picks a side by a fair coin, an edge is
        +1 inside a side and -1 across, then each sign is flipped with
        probability planted_flip.  meta records the sides and the flip count.
    Vertices may be isolated and the graph may be disconnected.
    """
    rng = np.random.default_rng(seed)

    def draw(k):
        return _power_law_endpoints(rng, n, gamma, k), _power_law_endpoints(rng, n, gamma, k)

    keys = _fill_unique(rng, n, m, draw)
    u, v = keys // n, keys % n
    del keys
    meta = {"recipe": "chung-lu", "n": n, "m": m, "gamma": gamma, "seed": str(seed)}
    if planted_flip is None:
        sign = np.where(rng.random(u.size) < p_pos, 1, -1).astype(np.int8)
        meta["p_pos"] = p_pos
    else:
        side = rng.integers(0, 2, size=n, dtype=np.int8)
        sign = np.where(side[u] == side[v], 1, -1).astype(np.int8)
        flip = rng.random(u.size) < planted_flip
        sign[flip] = -sign[flip]
        meta.update({"planted_flip": planted_flip, "flipped": int(flip.sum()), "side": side})
    return csr_from_edges(n, u, v, sign, meta)


def planted_er(n: int, m: int, flip: float, seed) -> SignedCSR:
    """Connected path+uniform graph with a planted two-way vertex split: +1 inside a
    side, -1 across, then each sign flipped with probability ``flip``."""
    g = erdos_renyi_connected(n, m, 1.0, seed)
    rng = np.random.default_rng([int(x) for x in np.atleast_1d(seed)] + [7])
    side = rng.integers(0, 2, size=n, dtype=np.int8)
    u, v, _ = g.edges()
    sign = np.where(side[u] == side[v], 1, -1).astype(np.int8)
    fl = rng.random(u.size) < flip
    sign[fl] = -sign[fl]
    return csr_from_edges(n, u, v, sign, {"recipe": "planted-path+uniform", "n": n, "m": m,
                                          "planted_flip": flip, "flipped": int(fl.sum()),
                                          "side": side, "seed": str(seed)})


# ---------------------------------------------------------------- fixed shapes

def config_small(seed=0) -> SignedCSR:
    """n = 1,000, m = 5,000, signs +1 w.p. 0.8 (the small sweep workload)."""
    return erdos_renyi_connected(1000, 5000, 0.8, seed)


def config_planted_powerlaw(seed=0, n=1_000_000, m=10_000_000) -> SignedCSR:
    """Chung-Lu exponent 2.1, planted two-way split, 5 % of signs flipped."""
    return chung_lu(n, m, 2.1, seed, planted_flip=0.05)


def config_large(seed=0, n=16_000_000, m=64_000_000) -> SignedCSR:
    """Chung-Lu exponent 2.3, 85 % positive signs (the bandwidth workload)."""
    return chung_lu(n, m, 2.3, seed, p_pos=0.85)


def config_batch_shapes(G=4096, seed=0, n_lo=100, n_hi=50_000):
    """Per-graph (n, m, p_pos) of the uneven batch: n ~ U{n_lo..n_hi}, average
    degree ~ U[4, 16], positive fraction ~ U[0.7, 0.9]."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=G)
    deg = rng.uniform(4.0, 16.0, size=G)
    ms = np.maximum(ns - 1, np.round(ns * deg / 2).astype(np.int64))
    ms = np.minimum(ms, ns * (ns - 1) // 2)
    pp = rng.uniform(0.7, 0.9, size=G)
    return ns.astype(np.int64), ms.astype(np.int64), pp


def config_batch(G=4096, seed=0, n_lo=100, n_hi=50_000, indices=None):
    """The uneven batch: graph g is erdos_renyi_connected with seed (seed, g)."""
    ns, ms, pp = config_batch_shapes(G, seed, n_lo, n_hi)
    idx = range(G) if indices is None else indices
    return [erdos_renyi_connected(int(ns[g]), int(ms[g]), float(pp[g]), (seed, g)) for g in idx]


def _batch_one(args):
    n, m, p, seed = args
    return erdos_renyi_connected(n, m, p, seed)


def config_batch_parallel(G=4096, seed=0, n_lo=100, n_hi=50_000, indices=None, workers=None):
    """config_batch generated by worker processes (spawned, so a parent that
    already uses the GPU is never forked); the graphs are identical."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os

    ns, ms, pp = config_batch_shapes(G, seed, n_lo, n_hi)
    idx = list(range(G) if indices is None else indices)
    jobs = [(int(ns[g]), int(ms[g]), float(pp[g]), (seed, g)) for g in idx]
    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1 or len(jobs) < 8:
        return [_batch_one(j) for j in jobs]
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_batch_one, jobs, chunksize=max(1, len(jobs) // (8 * workers))))


def graphl_init(n: int, R: int, seed) -> np.ndarray:
    """Gamma_0 ~ U(-1, 1) in float32, laid out [n, R] (restart r is column r)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(n, R)).astype(np.float32)


# ---------------------------------------------------------------- small fixtures

def figure_graph(signs) -> SignedCSR:
    """The 4-vertex, 5-edge graph of the paper's Figure fig-Balance: edges
    a=01, b=12, c=23, d=30, e=02 (the fundamental cycles 0-1-2 and 0-3-2 are
    named in Definition def-FundamentalCycle).  ``signs`` gives (a,b,c,d,e)."""
    u = [0, 1, 2, 0, 0]
    v = [1, 2, 3, 3, 2]
    return csr_from_edges(4, u, v, np.asarray(signs, dtype=np.int8), {"recipe": "figure"})


def complete_graph(n: int, sign: int = -1) -> SignedCSR:
    iu, ju = np.triu_indices(n, 1)
    return csr_from_edges(n, iu, ju, np.full(iu.size, sign, dtype=np.int8), {"recipe": f"K{n}"})


def cycle_graph(n: int, neg_edges=()) -> SignedCSR:
    u = np.arange(n)
    v = (u + 1) % n
    s = np.ones(n, dtype=np.int8)
    s[list(neg_edges)] = -1
    return csr_from_edges(n, u, v, s, {"recipe": "cycle"})


def random_tree(n: int, seed, p_pos=0.5) -> SignedCSR:
    rng = np.random.default_rng(seed)
    par = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
    child = np.arange(1, n)
    s = np.where(rng.random(n - 1) < p_pos, 1, -1).astype(np.int8)
    return csr_from_edges(n, par, child, s, {"recipe": "tree"})


def random_small(n: int, m: int, seed, p_pos=0.5, connected=False) -> SignedCSR:
    """Uniform random simple signed graph (possibly disconnected)."""
    if connected:
        return erdos_renyi_connected(n, m, p_pos, seed)
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    m = min(m, iu.size)
    pick = np.sort(rng.choice(iu.size, size=m, replace=False))
    s = np.where(rng.random(m) < p_pos, 1, -1).astype(np.int8)
    return csr_from_edges(n, iu[pick], ju[pick], s, {"recipe": "uniform-small"})


def isolated_vertices(n: int) -> SignedCSR:
    return SignedCSR(n=n, row_ptr=np.zeros(n + 1, dtype=np.int32), col=np.zeros(0, dtype=np.int32),
                     sign=np.zeros(0, dtype=np.int8), meta={"recipe": "empty"})
