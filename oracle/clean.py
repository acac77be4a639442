"""Input cleaning of a signed edge list (Section "Implementation": duplicates,
inconsistencies, self-loops and invalid signs are detected and eliminated).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

Reading of the cleaning rules (the paper names them without details):
* an entry whose endpoint lies outside 0 .. n-1 or whose sign is not +1 or -1
  is invalid and dropped;
* a self-loop (u, u) is dropped;
* entries are grouped by unordered pair {u, v}; a pair whose entries all
  carry one sign keeps one edge with that sign (the others are duplicates);
  a pair met with both signs is inconsistent and dropped entirely.
The result is a simple signed graph as symmetric CSR, rows sorted.
"""
from __future__ import annotations

import numpy as np


def clean(n: int, src, dst, sign):
    """(row_ptr int32[n+1], col int32[2m], sign int8[2m], counts) with counts =
    {kept, invalid, self_loops, duplicates, inconsistent_pairs}."""
    pairs = {}
    invalid = loops = 0
    for u, v, s in zip(np.asarray(src).tolist(), np.asarray(dst).tolist(), np.asarray(sign).tolist()):
        if not (0 <= u < n and 0 <= v < n) or s not in (1, -1):
            invalid += 1
            continue
        if u == v:
            loops += 1
            continue
        pairs.setdefault((min(u, v), max(u, v)), []).append(s)
    kept = {}
    dups = incons = 0
    for key, ss in pairs.items():
        if len(set(ss)) > 1:
            incons += 1
            continue
        kept[key] = ss[0]
        dups += len(ss) - 1
    entries = sorted([(u, v, s) for (u, v), s in kept.items()] +
                     [(v, u, s) for (u, v), s in kept.items()])
    row_ptr = np.zeros(n + 1, np.int64)
    for u, _, _ in entries:
        row_ptr[u + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    col = np.array([v for _, v, _ in entries], np.int32)
    sg = np.array([s for _, _, s in entries], np.int8)
    counts = {"kept": len(kept), "invalid": invalid, "self_loops": loops, "duplicates": dups,
              "inconsistent_pairs": incons}
    return row_ptr, col, sg, counts
