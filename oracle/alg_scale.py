"""Memory-bound frustration cloud of Alg. alg-scale (appendix, scaling section).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: never imported by the
library.

Input: the per-tree results of a sweep in tree order, each (S, key_hi, key_lo)
with S the switch count of tree t (Alg. alg-balance) and (key_hi, key_lo) the
128-bit key of its canonical balanced state, as ``oracle.sweep(...).trees``
returns them.  Output: the bounded cloud as a dict key -> [C, S, first tree].

Alg. alg-scale is garbled in three places; this module takes these readings:

* the replacement index is printed as argmin S, which would evict the best
  state the cloud holds; the prose around the algorithm says the cloud keeps
  the F_max best states, so the evicted entry is the worst one, largest S,
  and among equal S the one first reached last (the latest first tree);
* the increment of a repeated state sits under the test "frInd < max S", so a
  repeat of the current worst state would not be counted; the prose says C is
  the count through all k iterations, so a repeat of a kept state is always
  counted;
* below F_max entries a new state is always kept (the test "frInd < max S"
  applies to replacement only), so that with F_max at least the number of
  distinct states the result is the cloud of Alg. alg-index.

A new state whose S equals the worst kept S does not replace it (the test is
strict, as printed).
"""
from __future__ import annotations


def bounded_cloud(trees, f_max: int, t0: int = 0) -> dict:
    """Alg. alg-scale over the trees t0, t0 + 1, ... in order."""
    if f_max < 1:
        raise ValueError("F_max must be at least 1")
    cloud = {}  # (key_hi, key_lo) -> [C, S, first tree]
    for i, row in enumerate(trees):
        t = t0 + i
        S, khi, klo = int(row[0]), int(row[1]), int(row[2])
        key = (khi, klo)
        entry = cloud.get(key)
        if entry is not None:  # the state is held: C(i)++
            if entry[1] != S:
                raise RuntimeError("one state met two switch counts")
            entry[0] += 1
            continue
        if len(cloud) < f_max:  # room left: i++, S(i), B(i), C(i) = 1
            cloud[key] = [1, S, t]
            continue
        # full: the worst held state by (S, first tree)
        worst = max(cloud, key=lambda k: (cloud[k][1], cloud[k][2]))
        if S < cloud[worst][1]:  # frInd < max S: replace it
            del cloud[worst]
            cloud[key] = [1, S, t]
    return cloud


def frustration_index(cloud: dict):
    """Fr = min_i S(i) and the first tree reaching it (ties: earliest tree)."""
    if not cloud:
        raise ValueError("empty cloud")
    return min((v[1], v[2]) for v in cloud.values())


def as_rows(cloud: dict):
    """Rows (key_hi, key_lo, C, S, first tree) sorted by key, the layout of
    the library's cloud read-out."""
    return sorted((k[0], k[1], v[0], v[1], v[2]) for k, v in cloud.items())
