"""Write the expected per-graph results of the uneven batch (4,096 graphs,
64 trees each, sweep seed 0) for 256 sampled graphs.

Runs only the CPU oracle (oracle/) on the seeded synthetic graphs, each graph
alone, so that the GPU test can check the batched sweep at full size.
Usage:  python tests/golden/make_batch_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2311_00869_amd import synth  # noqa: E402

G, TREES, SEED, SAMPLE = 4096, 64, 0, 256


def sample_indices():
    """256 graphs: the 8 largest, the 8 smallest and 240 drawn uniformly."""
    ns, _, _ = synth.config_batch_shapes(G, 0)
    order = np.argsort(ns, kind="stable")
    fixed = set(order[:8].tolist()) | set(order[-8:].tolist())
    rest = [g for g in np.random.default_rng(2024).permutation(G).tolist() if g not in fixed]
    return sorted(fixed | set(rest[: SAMPLE - len(fixed)]))


def main():
    t = time.time()
    idx = sample_indices()
    graphs = synth.config_batch_parallel(G, 0, indices=idx)
    rows = []
    for g, gr in zip(idx, graphs):
        r = oracle.sweep(gr, SEED, 0, TREES, checks=False)
        rows.append([g, gr.n, gr.nnz, int(r.best[0]), int(r.best[1]), int(len(r.cloud))])
    out = {
        "workload": "uneven batch: 4,096 path+uniform graphs, n ~ U{100..50,000}, "
                    "average degree ~ U[4,16], p+ ~ U[0.7,0.9], graph g seeded (0, g)",
        "graphs": G, "trees_per_graph": TREES, "seed": SEED,
        "rows": rows,
        "note": "rows: graph index, n, nnz, min switches, first tree reaching it, distinct states; "
                "written by the CPU oracle, each graph swept alone",
    }
    with open(os.path.join(HERE, "batch_uneven.json"), "w") as f:
        json.dump(out, f, indent=0)
    print(f"{len(rows)} graphs x {TREES} trees in {time.time() - t:.1f}s", flush=True)


if __name__ == "__main__":
    main()
