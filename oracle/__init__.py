"""CPU oracle for the graphBpp sweep and for graphL.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the library.  It shares no code with
the HIP path (paper_2311_00869_amd); the only inputs both see are the arrays
made by paper_2311_00869_amd.synth, which holds none of the method.

* ``oracle.cpp`` (built into ``liboracle.so`` with g++): trees, the literal
  fundamental-cycle balancing of Alg. alg-balance, the exact frustration
  count, canonical states and their 128-bit keys, and the full sweep of
  Alg. alg-index with a std::map cloud.
* ``graphl.py``: graphL (Eq. eq-loss_imbalance_new, its gradient and
  Alg. alg-gradient) in float64 numpy.
* ``brute.py``: the exact frustration index by enumeration (small graphs).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

ERRORS = {
    0: "ok", -1: "EINVAL", -2: "EASYM", -3: "ESELFLOOP", -4: "EDUP", -5: "ESIGN",
    -6: "ERANGE", -7: "EUNSORTED", -20: "ECOLLISION", -21: "ESTATE", -22: "ESTRING", -23: "ECAP",
}


def build(force: bool = False) -> str:
    """Compile oracle.cpp into liboracle.so (g++ -O2, host only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = ctypes.CDLL(build())
            i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
            i8p = np.ctypeslib.ndpointer(np.int8, flags="C")
            u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
            c = ctypes
            L.orc_validate.argtypes = [c.c_int32, c.c_int64, i32p, i32p, i8p]
            L.orc_validate.restype = c.c_int
            L.orc_components.argtypes = [c.c_int32, i32p, i32p, i32p]
            L.orc_components.restype = c.c_int32
            L.orc_tree_salt.argtypes = [c.c_uint64, c.c_int64]
            L.orc_tree_salt.restype = c.c_uint64
            L.orc_vertex_key.argtypes = [c.c_uint64, c.c_int32]
            L.orc_vertex_key.restype = c.c_uint64
            L.orc_vertex_keys.argtypes = [c.c_uint64, c.c_int64, c.c_int64, c.c_int32,
                                          np.ctypeslib.ndpointer(np.uint32, flags="C")]
            L.orc_vertex_keys.restype = None
            L.orc_tree.argtypes = [c.c_int32, i32p, i32p, i8p, c.c_uint64, c.c_int64, c.c_int,
                                   i32p, i32p, i8p]
            L.orc_tree.restype = c.c_int
            L.orc_balance.argtypes = [c.c_int32, i32p, i32p, i8p, i32p, i32p, i8p]
            L.orc_balance.restype = c.c_int64
            L.orc_count.argtypes = [c.c_int32, i32p, i32p, i8p, i8p]
            L.orc_count.restype = c.c_int64
            L.orc_canonical.argtypes = [c.c_int32, i32p, i32p, i8p, u64p]
            L.orc_canonical.restype = None
            L.orc_hash128.argtypes = [c.c_int64, u64p, u64p]
            L.orc_hash128.restype = None
            L.orc_splitmix.argtypes = [c.c_uint64]
            L.orc_splitmix.restype = c.c_uint64
            L.orc_fmix32.argtypes = [c.c_uint32]
            L.orc_fmix32.restype = c.c_uint32
            L.orc_hybrid_coin.argtypes = [c.c_uint64]
            L.orc_hybrid_coin.restype = c.c_int
            L.orc_kruskal_weight.argtypes = [c.c_uint64, c.c_int32, c.c_int32]
            L.orc_kruskal_weight.restype = c.c_uint32
            L.orc_sweep.argtypes = [c.c_int32, i32p, i32p, i8p, c.c_uint64, c.c_int64, c.c_int64,
                                    c.c_int, c.c_void_p, c.c_void_p, c.c_int64,
                                    c.POINTER(c.c_int64), c.c_void_p, c.c_int]
            L.orc_sweep.restype = c.c_int
            _lib = L
    return _lib


def _g(g):
    return (int(g.n), np.ascontiguousarray(g.row_ptr, np.int32), np.ascontiguousarray(g.col, np.int32),
            np.ascontiguousarray(g.sign, np.int8))


def validate(g) -> int:
    n, rp, col, sg = _g(g)
    return int(lib().orc_validate(n, int(col.size), rp, col, sg))


def components(g):
    """(number of components, anchor id per vertex = smallest id in its component)."""
    n, rp, col, _ = _g(g)
    comp = np.empty(n, np.int32)
    c = lib().orc_components(n, rp, col, comp)
    return int(c), comp


def tree_salt(seed: int, t: int) -> int:
    return int(lib().orc_tree_salt(seed & (2**64 - 1), t))


def vertex_key(salt: int, u: int) -> int:
    return int(lib().orc_vertex_key(salt, u))


def vertex_keys(seed: int, t0: int, t1: int, n: int):
    """Keys of vertices 0..n-1 in trees t0..t1-1: uint32 [t1 - t0, n]."""
    out = np.empty((t1 - t0, n), np.uint32)
    lib().orc_vertex_keys(seed & (2**64 - 1), t0, t1, n, out)
    return out


def splitmix(x: int) -> int:
    return int(lib().orc_splitmix(x & (2**64 - 1)))


def fmix32(x: int) -> int:
    return int(lib().orc_fmix32(x & 0xFFFFFFFF))


SAMPLERS = {"bfs": 0, "rdfs": 1, "hybrid": 2, "kruskal": 3}


def _sampler(s) -> int:
    return SAMPLERS[s] if isinstance(s, str) else int(s)


def hybrid_coin(salt: int) -> int:
    """Alg. alg-hybrid's 0/1 for a tree's salt (0: BFS, 1: RDFS)."""
    return int(lib().orc_hybrid_coin(salt & (2**64 - 1)))


def kruskal_weight(salt: int, u: int, v: int) -> int:
    """Random weight of edge (u, v), u < v, in the tree with this salt."""
    return int(lib().orc_kruskal_weight(salt & (2**64 - 1), u, v))


def tree(g, seed: int, t: int, sampler="bfs"):
    """(level, parent, state +1/-1) of tree t with the given sampler."""
    n, rp, col, sg = _g(g)
    level = np.empty(n, np.int32)
    parent = np.empty(n, np.int32)
    state = np.empty(n, np.int8)
    rc = lib().orc_tree(n, rp, col, sg, seed & (2**64 - 1), t, _sampler(sampler), level, parent,
                        state)
    if rc != 0:
        raise RuntimeError(f"oracle tree failed: {ERRORS.get(rc, rc)}")
    return level, parent, state


def balance(g, level, parent):
    """Alg. alg-balance by fundamental-cycle walks: (switches, flip per CSR entry)."""
    n, rp, col, sg = _g(g)
    flip = np.empty(col.size, np.int8)
    s = lib().orc_balance(n, rp, col, sg, np.ascontiguousarray(level, np.int32),
                          np.ascontiguousarray(parent, np.int32), flip)
    return int(s), flip


def count(g, state_pm1) -> int:
    """Frustrated undirected edges under a +1/-1 state."""
    n, rp, col, sg = _g(g)
    return int(lib().orc_count(n, rp, col, sg, np.ascontiguousarray(state_pm1, np.int8)))


def canonical_words(g, state_pm1):
    n, rp, col, _ = _g(g)
    w = np.zeros((n + 63) // 64, np.uint64)
    lib().orc_canonical(n, rp, col, np.ascontiguousarray(state_pm1, np.int8), w)
    return w


def hash128(words):
    w = np.ascontiguousarray(words, np.uint64)
    out = np.zeros(2, np.uint64)
    lib().orc_hash128(int(w.size), w, out)
    return int(out[0]), int(out[1])


class SweepResult:
    def __init__(self, trees, cloud, best):
        self.trees = trees  # uint64 [T, 3]: switches, key_hi, key_lo
        self.cloud = cloud  # uint64 [E, 5]: key_hi, key_lo, freq, switches, first_tree
        self.best = best    # (min switches, first tree reaching it)

    @property
    def switches(self):
        return self.trees[:, 0].astype(np.int64)


def sweep(g, seed: int, t0: int, t1: int, checks: bool = True, paper_strings: bool = False,
          cloud_cap: int | None = None, sampler="bfs") -> SweepResult:
    """Alg. alg-index over trees t0..t1-1 with the given tree sampler.
    Raises on any failed self-check."""
    n, rp, col, sg = _g(g)
    T = t1 - t0
    trees = np.zeros((max(T, 0), 3), np.uint64)
    cap = T if cloud_cap is None else cloud_cap
    cloud = np.zeros((max(cap, 1), 5), np.uint64)
    size = ctypes.c_int64(0)
    best = np.zeros(2, np.uint64)
    flags = (1 if checks else 0) | (2 if paper_strings else 0)
    rc = lib().orc_sweep(n, rp, col, sg, seed & (2**64 - 1), t0, t1, flags,
                         trees.ctypes.data, cloud.ctypes.data, cap, ctypes.byref(size),
                         best.ctypes.data, _sampler(sampler))
    if rc != 0:
        raise RuntimeError(f"oracle sweep failed: {ERRORS.get(rc, rc)}")
    return SweepResult(trees, cloud[: size.value].copy(), (int(best[0]), int(best[1])))


def cloud_from_trees(trees, t0: int = 0):
    """Alg. alg-index's cloud rebuilt from per-tree rows (switches, key_hi,
    key_lo) of consecutive trees t0, t0+1, ...: a new key enters with C = 1,
    S = s and its tree as first tree; a key seen before gets C + 1 and must
    carry the same S (Eq. eq-cloud).  Returns (cloud rows key_hi, key_lo,
    freq, switches, first_tree sorted by key, (min S, first tree reaching
    it)).  Used to join sweeps of disjoint tree ranges run in separate
    processes."""
    cloud = {}
    best = None
    for i, (s, hi, lo) in enumerate(np.asarray(trees, np.uint64).tolist()):
        t = t0 + i
        e = cloud.get((hi, lo))
        if e is None:
            cloud[(hi, lo)] = [1, s, t]
        else:
            if e[1] != s:
                raise RuntimeError(f"tree {t}: key seen before with {e[1]} switches, now {s}")
            e[0] += 1
        if best is None or s < best[0]:
            best = (s, t)
    rows = [[hi, lo, f, s, ft] for (hi, lo), (f, s, ft) in sorted(cloud.items())]
    return np.array(rows, np.uint64).reshape(-1, 5), best
