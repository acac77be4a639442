"""Schedule choice for the sweep: a default by graph size, and an autotuner
that times candidate schedules and keeps the fastest.  Schedules never
change results (every path computes the same trees), so tuning only trades
speed.  Candidates are timed on as many trees as the caller will sweep (by
default two full passes of the 128-tree path), so that the multi-tree paths
run with every lane busy and with their tree order in effect.
"""
from __future__ import annotations

import json
import os
import time

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")

LDS_BYTES = 160 * 1024


def candidates(n: int, nnz: int):
    out = []
    if 12 * n + 32768 <= LDS_BYTES:
        for b in (256, 512, 1024):
            out.append(dict(path=1, block=b, grid=0, heavy=512, batch=1))
    if n <= 1_000_000:
        for b in (256, 512, 1024):
            out.append(dict(path=2, block=b, grid=0, heavy=512, batch=1))
    for b in (256, 512, 1024):
        for batch in (1, 4, 8):
            out.append(dict(path=3, block=b, grid=0, heavy=512, batch=batch))
    # the multi-tree paths also at fixed small grids (0 = sized to the graph)
    for b in (512, 1024):
        for grid in (0, 64, 128):
            out.append(dict(path=4, block=b, grid=grid, heavy=512, batch=1))
            out.append(dict(path=5, block=b, grid=grid, heavy=512, batch=1))
    return out


def _key(n, nnz):
    return f"{n}:{nnz}"


def default_schedule(n: int, nnz: int):
    cache = _load()
    if _key(n, nnz) in cache:
        return dict(cache[_key(n, nnz)])
    if 12 * n + 32768 <= LDS_BYTES:
        # the fewer trees' LDS a CU holds, the wider each workgroup
        block = 256 if 12 * n <= 24576 else 512 if 12 * n <= 65536 else 1024
        return dict(path=1, block=block, grid=0, heavy=512, batch=1)
    if n + nnz // 4 <= 135_000:  # nnz // 4 = m / 2 (m undirected edges)
        return dict(path=2, block=256 if nnz <= 10 * n else 1024, grid=0, heavy=512, batch=1)
    return dict(path=5, block=1024, grid=0, heavy=512, batch=1)


def _load():
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def autotune(graph, trees: int = 256, seed: int = 12345, save: bool = True, verbose=False):
    """Time each candidate schedule on `trees` trees (pass the number of trees
    the sweep will take; at least 128 fills a pass of the multi-tree path);
    keep the fastest."""
    import torch

    best = None
    results = []
    for s in candidates(graph.n, graph.nnz):
        try:
            graph.set_schedule(**s)
        except Exception:
            continue
        graph.cloud_reset()
        graph.sweep_range(0, min(trees, 2), seed)
        torch.cuda.synchronize()
        graph.cloud_reset()
        t0 = time.perf_counter()
        graph.sweep_range(0, trees, seed)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        results.append((el, s))
        if verbose:
            print(f"# tune {s}: {trees / el:.1f} trees/s", flush=True)
        if best is None or el < best[0]:
            best = (el, s)
    graph.cloud_reset()
    graph.set_schedule(**best[1])
    if save:
        cache = _load()
        cache[_key(graph.n, graph.nnz)] = best[1]
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return best[1], results


def _batch_key(batch):
    import hashlib
    h = hashlib.sha256(batch.vertex_offsets.tobytes() + batch.nnz_offsets.tobytes()).hexdigest()
    return f"batch:{h[:16]}"


def default_batch_schedule(batch):
    cache = _load()
    if _batch_key(batch) in cache:
        return dict(cache[_batch_key(batch)])
    return dict(block=512, grid=0, path=0)


def autotune_batch(batch, trees: int = 64, seed: int = 12345, save: bool = True, verbose=False):
    """Time the batched sweep's two schedules (path 1: one tree per
    workgroup; path 4: 64 trees of one graph per workgroup) at each block
    size on `trees` trees per graph (pass the number the sweep will take);
    keep the fastest (results do not depend on the choice)."""
    import torch

    best, results = None, []
    for path, b in [(p, b) for p in (1, 4) for b in (256, 512, 1024)]:
        batch.set_schedule(block=b, path=path)
        batch.sweep(1, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.sweep(trees, seed)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s = dict(block=b, grid=0, path=path)
        results.append((el, s))
        if verbose:
            print(f"# tune batch {s}: {trees * batch.G / el:.1f} trees/s", flush=True)
        if best is None or el < best[0]:
            best = (el, s)
    batch.set_schedule(**best[1])
    if save:
        cache = _load()
        cache[_batch_key(batch)] = best[1]
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return best[1], results
