"""Write the expected per-tree results of the full-size workloads.

Runs only the CPU oracle (oracle/) on the seeded synthetic graphs, so that
the GPU tests can check the HIP path at full size without running the oracle
beside them.  Trees are independent, so each worker process sweeps one
tree at a time (the graph is made once and shared by fork), and the cloud is
joined from the per-tree rows by oracle.cloud_from_trees.

Usage:  python tests/golden/make_fullsize_golden.py [large] [planted] [--workers N]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2311_00869_amd import synth  # noqa: E402

CASES = {
    # 16M vertices / 64M edges, Chung-Lu exponent 2.3, 85 % positive: one
    # full 128-tree pass of the multi-tree kernel plus two trees of the next
    "large": dict(make=lambda: synth.config_large(0), seed=0, trees=(0, 130)),
    # 1M vertices / 10M edges, Chung-Lu exponent 2.1, planted split, 5 % flips
    "planted": dict(make=lambda: synth.config_planted_powerlaw(0), seed=0, trees=(0, 32)),
}

_G = None


def _tree(args):
    seed, t = args
    res = oracle.sweep(_G, seed, t, t + 1, checks=True)
    return t, [int(x) for x in res.trees[0]]


def main(names, workers):
    global _G
    for name in names:
        c = CASES[name]
        t = time.time()
        _G = c["make"]()
        g = _G
        t0, t1 = c["trees"]
        rows = {}
        with mp.get_context("fork").Pool(workers) as pool:
            for i, row in pool.imap_unordered(_tree, [(c["seed"], i) for i in range(t0, t1)]):
                rows[i] = row
                print(f"{name}: tree {i} done, {len(rows)}/{t1 - t0} after "
                      f"{time.time() - t:.0f}s", flush=True)
        trees = np.array([rows[i] for i in range(t0, t1)], np.uint64)
        cloud, best = oracle.cloud_from_trees(trees, t0)
        out = {
            "workload": name, "n": g.n, "nnz": g.nnz, "seed": c["seed"], "t0": t0, "t1": t1,
            "trees": [[int(x) for x in row] for row in trees.tolist()],
            "cloud": [[int(x) for x in row] for row in cloud.tolist()],
            "best": [int(best[0]), int(best[1])],
            "note": "per-tree rows: switches, key_hi, key_lo; cloud rows: key_hi, key_lo, freq, "
                    "switches, first_tree; written by the CPU oracle with its self-checks on, "
                    "one tree per process, the cloud joined by oracle.cloud_from_trees",
        }
        if "flipped" in g.meta:
            out["planted_flipped"] = int(g.meta["flipped"])
        with open(os.path.join(HERE, f"fullsize_{name}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(f"{name}: {t1 - t0} trees in {time.time() - t:.1f}s", flush=True)
        _G = None


if __name__ == "__main__":
    argv = sys.argv[1:]
    workers = 6
    if "--workers" in argv:
        i = argv.index("--workers")
        workers = int(argv[i + 1])
        del argv[i:i + 2]
    main(argv or list(CASES), workers)
