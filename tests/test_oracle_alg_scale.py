"""Pins of the memory-bound cloud oracle (Alg. alg-scale).

Checked against a sequence worked by hand (tests/golden/alg_scale_sequence.json),
against the prose's description of the result (the F_max best distinct states
by switch count, each with its count through all k trees), and against the
unbounded cloud of Alg. alg-index when F_max is large enough.
"""
import json
import os
import random

import numpy as np
import pytest

import oracle
from oracle import alg_scale
from paper_2311_00869_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fixture():
    with open(os.path.join(GOLDEN, "alg_scale_sequence.json")) as f:
        return json.load(f)


def test_hand_worked_sequence():
    fx = _fixture()
    labels = sorted({s for s, _ in fx["sequence"]})
    code = {s: i for i, s in enumerate(labels)}
    trees = [(S, 0, code[s]) for s, S in fx["sequence"]]
    for fmax, want in fx["expected"].items():
        got = alg_scale.bounded_cloud(trees, int(fmax))
        got_rows = sorted((labels[k[1]], v[0], v[1], v[2]) for k, v in got.items())
        assert got_rows == [tuple(r) for r in want], fmax
        assert list(alg_scale.frustration_index(got)) == fx["frustration_index"]
    with pytest.raises(ValueError):
        alg_scale.bounded_cloud(trees, 0)


def _prose_cloud(trees, fmax, t0=0):
    """The F_max best distinct states by (S, first tree) with total counts."""
    stats = {}
    for i, (S, khi, klo) in enumerate(trees):
        e = stats.setdefault((khi, klo), [0, S, t0 + i])
        e[0] += 1
    best = sorted(stats, key=lambda k: (stats[k][1], stats[k][2]))[:fmax]
    return {k: stats[k] for k in best}


@pytest.mark.parametrize("trial", range(40))
def test_random_sequences_keep_the_best_states_with_full_counts(trial):
    rnd = random.Random(trial)
    nstates = rnd.randint(1, 60)
    s_of = [rnd.randint(0, 12) for _ in range(nstates)]  # many ties in S
    K = rnd.randint(1, 300)
    weights = [rnd.random() ** 3 for _ in range(nstates)]
    picks = rnd.choices(range(nstates), weights=weights, k=K)
    trees = [(s_of[p], p >> 3, p) for p in picks]
    t0 = rnd.randint(0, 1000)
    for fmax in (1, 2, 3, 5, 8, 17, nstates, nstates + 5):
        got = alg_scale.bounded_cloud(trees, fmax, t0)
        assert got == _prose_cloud(trees, fmax, t0), fmax


def test_large_bound_gives_the_alg_index_cloud():
    g = synth.random_small(400, 900, 21, p_pos=0.55)
    K = 120
    r = oracle.sweep(g, 77, 0, K, checks=False)
    unbounded = sorted(tuple(int(x) for x in row) for row in r.cloud)
    for fmax in (len(r.cloud), len(r.cloud) + 1, 10 * K):
        got = alg_scale.as_rows(alg_scale.bounded_cloud(r.trees, fmax))
        assert got == unbounded, fmax
    # every bound keeps the minimum of Eq. eq-obj and the first tree reaching it
    for fmax in (1, 2, 7):
        assert alg_scale.frustration_index(alg_scale.bounded_cloud(r.trees, fmax)) == r.best


def test_bounded_cloud_size_and_counts():
    g = synth.random_small(300, 700, 5, p_pos=0.6)
    K = 200
    r = oracle.sweep(g, 3, 0, K, checks=False)
    distinct = len(r.cloud)
    assert distinct > 10  # the bound below must bite
    total = {(int(a), int(b)): int(c) for a, b, c, _, _ in r.cloud}
    for fmax in (1, 4, distinct // 2):
        c = alg_scale.bounded_cloud(r.trees, fmax)
        assert len(c) == fmax
        for k, v in c.items():
            assert v[0] == total[k]
        # trees continue from t0: the same result as one call over all trees
        first = alg_scale.bounded_cloud(r.trees[:K // 2], fmax)
        assert all(t < K // 2 for _, _, t in first.values())
    assert np.all(r.switches >= r.best[0])
