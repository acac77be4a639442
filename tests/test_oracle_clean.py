"""Pins of the input-cleaning oracle (oracle/clean.py): a fixture worked by
hand, the validator of the graph contract on every output, and invariants
(idempotence, independence from entry order and direction, entry counts)."""
import json
import os

import numpy as np

import oracle
from oracle import clean as oclean

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class _G:
    def __init__(self, n, rp, col, sg):
        self.n, self.row_ptr, self.col, self.sign = n, rp, col, sg


def test_hand_worked_fixture():
    with open(os.path.join(GOLDEN, "clean_fixture.json")) as f:
        fx = json.load(f)
    e = np.array(fx["edges"])
    rp, col, sg, counts = oclean.clean(fx["n"], e[:, 0], e[:, 1], e[:, 2])
    assert rp.tolist() == fx["expected"]["row_ptr"]
    assert col.tolist() == fx["expected"]["col"]
    assert sg.tolist() == fx["expected"]["sign"]
    assert counts == fx["expected"]["counts"]


def _messy(rng, n, E):
    src = rng.integers(-2, n + 2, E)
    dst = rng.integers(-2, n + 2, E)
    sign = rng.choice([1, -1, 1, -1, 0, 2], E)
    # repeats of earlier entries, some reversed, some with the other sign
    k = E // 3
    pick = rng.integers(0, E, k)
    flip = rng.random(k) < 0.5
    src[-k:], dst[-k:] = np.where(flip, dst[pick], src[pick]), np.where(flip, src[pick], dst[pick])
    sign[-k:] = np.where(rng.random(k) < 0.8, sign[pick], -sign[pick])
    return src, dst, sign


def test_outputs_satisfy_the_graph_contract_and_invariants():
    rng = np.random.default_rng(3)
    for trial in range(6):
        n, E = int(rng.integers(5, 300)), int(rng.integers(0, 3000))
        src, dst, sign = _messy(rng, n, E)
        rp, col, sg, c = oclean.clean(n, src, dst, sign)
        assert oracle.validate(_G(n, rp, col, sg)) == 0
        assert len(col) == 2 * c["kept"]
        # every entry is accounted for exactly once
        valid = (src >= 0) & (src < n) & (dst >= 0) & (dst < n) & np.isin(sign, [1, -1])
        assert c["invalid"] == int((~valid).sum())
        assert c["self_loops"] == int((valid & (src == dst)).sum())
        # idempotent, and blind to entry order and direction
        rows = np.repeat(np.arange(n), np.diff(rp))
        again = oclean.clean(n, rows, col, sg)
        assert np.array_equal(again[0], rp) and np.array_equal(again[1], col)
        assert again[3]["duplicates"] == c["kept"] and again[3]["inconsistent_pairs"] == 0
        perm = rng.permutation(E)
        sw = rng.random(E) < 0.5
        s2, d2 = np.where(sw, dst, src)[perm], np.where(sw, src, dst)[perm]
        other = oclean.clean(n, s2, d2, sign[perm])
        assert all(np.array_equal(a, b) for a, b in zip(other[:3], (rp, col, sg)))
        assert other[3] == c
