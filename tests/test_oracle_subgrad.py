"""Pins of the oracle's projected dual subgradient rule (oracle/routing.py,
"subgrad"), independent of its own arithmetic:

* the update moves along a subgradient of the dual D: a one-sided finite
  difference of D(p) (FP64, in the direction of one expert) equals
  C - load_e of the top-k ranking under p, so the rule's step direction
  load_e - C is the negative subgradient (a sign or index mistake fails);
* prices stay non-negative, a converged routing respects every capacity,
  and a batch already within capacity at zero prices is plain top-k with
  no update;
* weak duality against HiGHS: at the end, primal (after the repair) <=
  LP optimum <= D(p), and on tiny batches the brute-force optimum lies in
  the same bracket.
"""
import numpy as np
import pytest

from oracle import certify, routing as R

F32 = np.float32


def _logits(T, E, seed, skew=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.standard_normal((T, E)) + skew * np.linspace(1.5, 0.0, E)[None, :]
    return s.astype(F32)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_update_direction_is_the_negative_dual_subgradient(seed):
    T, E, k, C = 40, 6, 2, 16
    s = _logits(T, E, seed).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    p = rng.uniform(0.0, 0.5, E)
    a = s - p[None, :]
    order = np.argsort(-a, axis=1, kind="stable")
    load = np.bincount(order[:, :k].ravel(), minlength=E)
    # the smallest gap between rank k and rank k+1 bounds the step
    srt = -np.sort(-a, axis=1)
    gap = float(np.min(srt[:, k - 1] - srt[:, k]))
    h = gap / 8.0
    base = R.dual_objective(s, p, k, C)
    for e in range(E):
        q = p.copy()
        q[e] += h
        fd = (R.dual_objective(s, q, k, C) - base) / h
        assert abs(fd - (C - load[e])) < 1e-6, (e, fd, C - load[e])


@pytest.mark.parametrize("seed,skew", [(4, 1.0), (5, 2.0), (6, 0.5)])
def test_invariants_and_weak_duality(seed, skew):
    T, E, k = 120, 8, 2
    C = int(np.ceil(1.25 * T * k / E))
    s = _logits(T, E, seed, skew)
    r = R.route(s, k, C, max_iters=60, mode="subgrad")
    assert r["status"] == R.OK
    assert np.all(r["p"] >= 0)
    assert np.all(r["load"] <= C)
    if r["converged"]:
        assert not r["enforced"]
    primal = R.primal_objective(s, r["sel"])
    dual = R.dual_objective(s, r["p"], k, C)
    lp, _ = certify.lp_opt(s, k, C)
    assert primal <= lp + 1e-6 <= dual + 2e-6


def test_feasible_batch_needs_no_update():
    T, E, k = 64, 8, 2
    s = _logits(T, E, 7, skew=0.0)
    C = T * k  # every expert can take every token
    r = R.route(s, k, C, mode="subgrad")
    assert r["iters"] == 0 and r["converged"]
    assert np.all(r["p"] == 0)
    top = R.route(s, k, C, mode="none")
    np.testing.assert_array_equal(r["sel"], top["sel"])


@pytest.mark.parametrize("seed", [8, 9])
def test_tiny_batches_bracket_the_brute_force_optimum(seed):
    T, E, k, C = 6, 3, 1, 2
    s = _logits(T, E, seed, skew=2.0)
    r = R.route(s, k, C, max_iters=200, mode="subgrad")
    opt, _ = certify.brute_force_opt(s, k, C)
    primal = R.primal_objective(s, r["sel"])
    dual = R.dual_objective(s, r["p"], k, C)
    assert primal <= opt + 1e-9 <= dual + 1e-6


def test_overloaded_price_rises_while_the_others_stay_at_zero():
    # every token prefers expert 0 by a wide margin: while expert 0 stays
    # over capacity its price rises every update and the idle experts keep
    # price zero (their subgradient component C - 0 > 0 projects to 0).
    # Later the near-tied experts 1-3 take the overflow in turns: the plain
    # subgradient step oscillates on such ties, and the repair ends it.
    T, E, k, C = 32, 4, 1, 8
    s = np.zeros((T, E), F32)
    s[:, 0] = 5.0
    s += _logits(T, E, 10, skew=0.0) * F32(0.01)
    prev = F32(0.0)
    for it in (1, 2, 3):
        r = R.subgrad_prices(s, k, C, max_iters=it)
        assert r["iters"] == it and r["load"][0] == T
        assert r["p"][0] > prev and np.all(r["p"][1:] == 0)
        prev = r["p"][0]
    full = R.route(s, k, C, max_iters=400, mode="subgrad")
    assert full["status"] == R.OK and np.all(full["load"] <= C)
