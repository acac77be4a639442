"""Parity of the GPU input cleaning (fi_clean) with the oracle: the
hand-worked fixture, messy random edge lists (invalid ids and signs,
self-loops, repeats in both directions, conflicting signs), the empty list,
and a sweep of the cleaned graph."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import clean as oclean

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2311_00869_amd.frustration")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _check(n, src, dst, sign):
    rp, col, sg, counts = fr.clean(n, src, dst, sign)
    want = oclean.clean(n, src, dst, sign)
    assert np.array_equal(rp.cpu().numpy(), want[0])
    assert np.array_equal(col.cpu().numpy(), want[1])
    assert np.array_equal(sg.cpu().numpy(), want[2])
    assert counts == want[3]
    return rp, col, sg


def test_fixture():
    with open(os.path.join(GOLDEN, "clean_fixture.json")) as f:
        fx = json.load(f)
    e = np.array(fx["edges"], np.int32)
    _check(fx["n"], e[:, 0], e[:, 1], e[:, 2])


@pytest.mark.parametrize("seed", range(5))
def test_messy_edge_lists(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 5000))
    E = int(rng.integers(1, 60000))
    src = rng.integers(-3, n + 3, E).astype(np.int32)
    dst = rng.integers(-3, n + 3, E).astype(np.int32)
    sign = rng.choice([1, -1, 1, -1, 0, 3], E).astype(np.int32)
    k = E // 3
    pick = rng.integers(0, E, k)
    flip = rng.random(k) < 0.5
    src[-k:], dst[-k:] = np.where(flip, dst[pick], src[pick]), np.where(flip, src[pick], dst[pick])
    sign[-k:] = np.where(rng.random(k) < 0.8, sign[pick], -sign[pick])
    _check(n, src, dst, sign)


def test_empty_and_all_invalid():
    z = np.zeros(0, np.int32)
    rp, col, sg, c = fr.clean(4, z, z, z)
    assert rp.tolist() == [0] * 5 and len(col) == 0 and c["kept"] == 0
    _check(3, np.array([0, 1, 2], np.int32), np.array([0, 5, 1], np.int32),
           np.array([1, 1, 0], np.int32))


def test_cleaned_graph_sweeps_like_the_oracle():
    rng = np.random.default_rng(11)
    n, E = 800, 6000
    src = rng.integers(0, n, E).astype(np.int32)
    dst = rng.integers(0, n, E).astype(np.int32)
    sign = rng.choice([1, -1], E).astype(np.int32)
    rp, col, sg = _check(n, src, dst, sign)
    G = fr.Graph(rp, col, sg, cloud_capacity=64)
    want = oclean.clean(n, src, dst, sign)

    class _G:
        pass
    g = _G()
    g.n, g.row_ptr, g.col, g.sign = n, want[0], want[1], want[2]
    ref = oracle.sweep(g, 4, 0, 64, checks=True)
    sw = G.sweep_range(0, 64, 4, tree_switches=True).cpu().numpy().astype(np.uint64)
    assert np.array_equal(sw, ref.trees[:, 0])
    assert np.array_equal(G.cloud(), ref.cloud)
    G.close()
