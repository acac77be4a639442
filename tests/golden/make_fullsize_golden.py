"""Write the expected per-tree results of the full-size workloads.

Runs only the CPU oracle (oracle/) on the seeded synthetic graphs, so that
the GPU tests can check the HIP path at full size without running the oracle
on the GPU machine.  Usage:  python tests/golden/make_fullsize_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2311_00869_amd import synth  # noqa: E402

CASES = {
    # 16M vertices / 64M edges, Chung-Lu exponent 2.3, 85 % positive
    "large": dict(make=lambda: synth.config_large(0), seed=0, trees=(0, 2)),
    # 1M vertices / 10M edges, Chung-Lu exponent 2.1, planted split, 5 % flips
    "planted": dict(make=lambda: synth.config_planted_powerlaw(0), seed=0, trees=(0, 8)),
}


def main(names):
    for name in names:
        c = CASES[name]
        t = time.time()
        g = c["make"]()
        t0, t1 = c["trees"]
        res = oracle.sweep(g, c["seed"], t0, t1, checks=True)
        out = {
            "workload": name, "n": g.n, "nnz": g.nnz, "seed": c["seed"], "t0": t0, "t1": t1,
            "trees": [[int(x) for x in row] for row in res.trees.tolist()],
            "cloud": [[int(x) for x in row] for row in res.cloud.tolist()],
            "best": list(res.best),
            "note": "per-tree rows: switches, key_hi, key_lo; cloud rows: key_hi, key_lo, freq, "
                    "switches, first_tree; written by the CPU oracle with its self-checks on",
        }
        if "flipped" in g.meta:
            out["planted_flipped"] = int(g.meta["flipped"])
        with open(os.path.join(HERE, f"fullsize_{name}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(f"{name}: {t1 - t0} trees in {time.time() - t:.1f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
