"""Hand-worked pins of the oracle's capacity repair and logit statistics.

Each fixture under tests/golden/ carries its derivation.  Beside the
expected result it lists what plausible misreadings would return (proposals
accepted in token order, ties broken towards the higher index, a sample
instead of a population std, the C-th instead of the (C+1)-th largest
value); the tests check that the oracle returns the expected result and that
every listed misreading returns something else, so the fixture rejects it.
"""
import json
import os

import numpy as np
import pytest

from oracle import mlp as M
from oracle import routing as R

GOLD = os.path.join(os.path.dirname(__file__), "golden")
F32 = np.float32


def _load(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


REPAIR = _load("repair_hand.json")["examples"]


@pytest.mark.parametrize("ex", REPAIR, ids=[e["name"] for e in REPAIR])
def test_repair_hand_worked(ex):
    s = np.array(ex["s"], dtype=F32)
    T, E = s.shape
    k, C = ex["k"], ex["C"]
    r = R.route(s, k, C, 0, np.zeros(E, F32), "given")
    assert r["status"] == R.OK and r["enforced"]
    assert r["rounds"] == ex["rounds"]
    np.testing.assert_array_equal(r["sel"], ex["sel"])
    np.testing.assert_array_equal(r["load"], ex["load"])
    # the same through the repair entry on the plain top-k routing
    sel0, _, _, _ = R.topk_under_prices(s, np.zeros(E, F32), k)
    sel, st, rounds = R.enforce_capacity(s, np.zeros(E, F32), sel0, k, C)
    assert st == R.OK and rounds == ex["rounds"]
    np.testing.assert_array_equal(sel, ex["sel"])
    for name, alt in ex["mutants"].items():
        assert not np.array_equal(np.array(alt), np.array(ex["sel"])), name
        # each misreading's routing is still feasible (so only the order
        # rule, not an invariant, tells it apart)
        assert np.bincount(np.array(alt).ravel(), minlength=E).max() <= C, name


def test_repair_hand_worked_given_prices_shift_keys():
    """Given prices enter through the keys a = s - p.  In the first example
    with p_1 = 2: t4 ranks expert 2 first (a = [1, 1, 2]) and keeps it, so
    expert 1 starts empty; t2 and t3 are evicted from expert 0 as before and
    both propose to expert 1 (a = 3 and 4, above expert 2's 0), which has
    room 2 and accepts both in one round."""
    ex = REPAIR[0]
    s = np.array(ex["s"], dtype=F32)
    p = np.array([0.0, 2.0, 0.0], F32)
    r = R.route(s, 1, 2, 0, p, "given")
    assert r["status"] == R.OK and r["enforced"]
    np.testing.assert_array_equal(r["sel"], [[0], [0], [1], [1], [2]])
    assert r["rounds"] == 1


FEAT = _load("features_hand.json")


@pytest.mark.parametrize("scale,shift", [(1.0, 0.0), (2.0, 3.0)])
def test_features_hand_computed(scale, shift):
    s = (np.array(FEAT["s"], np.float64) * scale + shift).astype(F32)
    got = M.features(s, FEAT["k"], FEAT["C"])
    np.testing.assert_allclose(got, np.array(FEAT["features"]), rtol=0, atol=1e-12)


def test_features_fixture_rejects_misreadings():
    s = np.array(FEAT["s"], np.float64)
    want = np.array(FEAT["features"])
    mut = FEAT["mutants"]
    # sample std
    ddof1 = s.std(axis=0, ddof=1) / s.std()
    np.testing.assert_allclose(ddof1, mut["sample std (ddof = 1) in f1"], atol=1e-12)
    assert np.abs(ddof1 - want[:, 1]).max() > 0.05
    # C-th largest instead of (C+1)-th
    C = FEAT["C"]
    qC = np.sort(s, axis=0)[::-1][C - 1]
    np.testing.assert_allclose(qC, mut["C-th instead of (C+1)-th largest in f3"], atol=1e-12)
    assert np.abs(qC - want[:, 3]).max() > 0.5
    # ties to the higher expert: token 3 would take expert 1
    load_alt = np.array([3, 1]) / C
    np.testing.assert_allclose(load_alt, mut["ties ranked to the higher expert (t3 -> 1): load0/C"])
    assert np.abs(load_alt - want[:, 4]).max() > 0.4
    # without mu / without sigma: the shifted and scaled batch separates them
    s2 = 2.0 * s + 3.0
    assert abs(s2[:, 0].mean() / s2.std() - want[0, 0]) > 0.5
    assert abs(s2[:, 0].max() - s2.mean() - want[0, 2]) > 0.5
