"""Pins of the routing oracle against facts that do not come from it:
a hand-worked example, the zero-price special case, exhaustive enumeration,
an LP solver, weak duality, a max-flow, and order-theoretic identities."""
import json
import math
import os

import numpy as np
import pytest
import scipy.special

from oracle import certify, routing as R
from paper_2606_17065_amd import synth

F32 = np.float32
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _independent_topk(s, k):
    """Plain top-k by Python's sort on (value desc, expert asc)."""
    out = []
    for row in np.asarray(s, np.float64):
        order = sorted(range(len(row)), key=lambda e: (-row[e], e))
        out.append(order[:k])
    return np.array(out)


def test_hand_worked_example():
    g = json.load(open(os.path.join(GOLD, "acp_hand_3x3.json")))
    s = np.array(g["s"], dtype=F32)
    r = R.route(s, g["k"], g["C"])
    assert r["status"] == R.OK and r["converged"] and not r["enforced"]
    assert r["iters"] == g["iters"]
    assert abs(float(r["sigma"]) - g["sigma"]) < 1e-6
    np.testing.assert_allclose(r["p"], g["p"], atol=1e-6)
    np.testing.assert_array_equal(r["sel"], g["sel"])
    assert abs(R.primal_objective(s, r["sel"]) - g["objective"]) == 0
    assert abs(R.dual_objective(s, r["p"], g["k"], g["C"]) - g["objective"]) < 1e-6


def test_key_order_matches_float_order():
    rng = np.random.default_rng(3)
    v = np.concatenate([
        rng.standard_normal(2000).astype(F32) * F32(1e3),
        np.array([0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-45, 3.4e38, -3.4e38], dtype=F32),
    ]).astype(F32)
    key = R.f32_key(v)
    for i in range(0, v.shape[0], 7):
        for j in range(0, v.shape[0], 11):
            a, b = float(v[i]), float(v[j])
            if a < b:
                assert key[i] < key[j]
            elif a > b:
                assert key[i] > key[j]
    # -0 sorts strictly below +0
    assert R.f32_key(np.array([-0.0], F32))[0] < R.f32_key(np.array([0.0], F32))[0]


@pytest.mark.parametrize("mode", ["none", "given"])
def test_ties_rank_the_lower_expert_first(mode):
    """Equal price-adjusted scores are ranked by expert index, lowest first:
    the oracle's selection equals a brute-force Python sort of each token's
    (-key, e) pairs, on logits with exact ties everywhere (a 0.5 grid) and,
    in the given-price mode, prices on the same grid (more ties)."""
    rng = np.random.default_rng(11)
    T, E, k = 60, 12, 4
    s = (np.round(rng.standard_normal((T, E)) * 2.0) / 2.0).astype(F32)
    p = None
    if mode == "given":
        p = (np.round(rng.uniform(0.0, 1.0, E) * 2.0) / 2.0).astype(F32)
    r = R.route(s, k, T * k, 0, p, mode)
    a = s if p is None else (s - p[None, :]).astype(F32)
    key = R.f32_key(a)
    for t in range(T):
        want = [e for _, e in sorted((-int(key[t, e]), e) for e in range(E))[:k]]
        assert r["sel"][t].tolist() == want, t
    assert (np.sort(key, axis=1)[:, :-1] == np.sort(key, axis=1)[:, 1:]).any()  # ties exist


def test_sigma_is_the_population_std():
    s = synth.make_logits(3000, 17, 1.2, seed=5)
    S1, S2 = R.score_sums(s)
    v = s.astype(np.float64).ravel()
    assert abs(S1 - math.fsum(v)) <= 1e-9 * abs(math.fsum(np.abs(v)))
    assert abs(S2 - math.fsum(v * v)) <= 1e-12 * math.fsum(v * v)
    sig = R.score_sigma(s)
    assert abs(float(sig) - float(np.std(v))) <= 2e-7 * float(np.std(v))


@pytest.mark.parametrize("seed", range(6))
def test_zero_price_reduction_when_capacity_is_slack(seed):
    T, E, k = 50, 6, 2
    s = synth.tiny_logits(T, E, seed)
    r = R.route(s, k, C=T)
    assert r["iters"] == 0 and r["converged"] and not r["enforced"]
    assert np.all(r["p"] == 0)
    np.testing.assert_array_equal(r["sel"], _independent_topk(s, k))


def test_feasible_plain_topk_stops_before_any_update():
    rng = np.random.default_rng(11)
    s = (0.01 * rng.standard_normal((64, 8))).astype(F32)
    sel = _independent_topk(s, 2)
    C = int(np.bincount(sel.ravel(), minlength=8).max())
    r = R.route(s, 2, C)
    assert r["iters"] == 0 and np.all(r["p"] == 0)
    np.testing.assert_array_equal(r["sel"], sel)


def _check_invariants(r, T, E, k, C):
    sel = r["sel"]
    assert sel.shape == (T, k)
    for row in sel:
        assert len(set(row.tolist())) == k
    assert np.all((sel >= 0) & (sel < E))
    load = np.bincount(sel.ravel(), minlength=E)
    np.testing.assert_array_equal(load, r["load"])
    assert load.max() <= C
    np.testing.assert_allclose(r["w"].sum(axis=1), 1.0, rtol=0, atol=1e-12)
    assert np.all(r["w"] > 0)
    assert np.all(r["p"] >= 0)


@pytest.mark.parametrize("T,E,k", [(6, 4, 2), (5, 4, 2), (6, 3, 1), (6, 4, 1), (4, 4, 3)])
@pytest.mark.parametrize("seed", range(8))
def test_brute_force_bracket(T, E, k, seed):
    s = synth.tiny_logits(T, E, 100 + seed)
    C = synth.capacity(T, k, E)
    r = R.route(s, k, C)
    assert r["status"] == R.OK
    _check_invariants(r, T, E, k, C)
    opt, _ = certify.brute_force_opt(s, k, C)
    prim = R.primal_objective(s, r["sel"])
    D = R.dual_objective(s, r["p"], k, C)
    assert prim <= opt + 1e-12
    assert opt <= D + 1e-9  # weak duality, any p >= 0
    if not r["enforced"]:
        # certificate identity: D - primal = sum_e p_e (C - load_e)
        ident = float(np.sum(r["p"].astype(np.float64) * (C - r["load"])))
        assert abs((D - prim) - ident) <= 1e-6 * max(1.0, abs(D))


@pytest.mark.parametrize("seed", range(3))
def test_lp_bracket_small_config(seed):
    sh = synth.SHAPES[1]
    inp = synth.make_inputs(sh, 1, rep=seed, experts=False)
    s = (inp["X"].astype(np.float64) @ inp["Wr"].T.astype(np.float64) + inp["br"]).astype(F32)
    C = sh.capacity
    r = R.route(s, sh.k, C)
    assert r["status"] == R.OK
    _check_invariants(r, sh.T, sh.E, sh.k, C)
    opt, x = certify.lp_opt(s, sh.k, C)
    # the LP optimum is integral (total unimodularity)
    assert np.max(np.minimum(np.abs(x), np.abs(1 - x))) < 1e-6
    prim = R.primal_objective(s, r["sel"])
    D = R.dual_objective(s, r["p"], sh.k, C)
    assert prim <= opt + 1e-9 <= D + 2e-9
    # the price rule's suboptimality is bounded by the certificate gap
    gap = (D - prim) / abs(D)
    assert (opt - prim) / abs(opt) <= gap + 1e-12
    assert gap < 5e-3


def test_acp_first_update_matches_definition():
    # After one update, an overloaded expert's price admits at most C of the
    # tokens whose margin at the old prices exceeds it.
    s = synth.make_logits(400, 8, 1.1, seed=9)
    k, C = 2, synth.capacity(400, 2, 8)
    r0 = R.acp_prices(s, k, C, max_iters=0)
    r1 = R.acp_prices(s, k, C, max_iters=1)
    assert r0["iters"] == 0 and r1["iters"] == 1
    over = np.nonzero(r0["load"] > C)[0]
    assert over.size > 0
    a = s.astype(np.float64)
    sel0 = r0["sel"]
    srt = np.sort(a, axis=1)[:, ::-1]
    kap1, kap2 = srt[:, k - 1], srt[:, k]
    for e in range(8):
        held = np.any(sel0 == e, axis=1)
        m = a[:, e] - np.where(held, kap2, kap1)
        if e in over:
            assert np.sum(m >= r1["p"][e]) <= C
            assert r1["p"][e] > 0
        else:
            assert r1["p"][e] == 0


def test_enforcement_repairs_a_capped_run():
    s = synth.make_logits(300, 8, 1.3, seed=21)
    k, C = 2, synth.capacity(300, 2, 8)
    r = R.route(s, k, C, max_iters=1)
    assert r["enforced"] and not r["converged"]
    assert r["status"] == R.OK
    _check_invariants(r, 300, 8, k, C)
    # tokens the repair did not touch keep the capped run's choice
    raw = R.acp_prices(s, k, C, max_iters=1)
    sel0 = raw["sel"]
    over = np.nonzero(raw["load"] > C)[0]
    untouched = ~np.isin(sel0, over).any(axis=1)
    np.testing.assert_array_equal(np.sort(r["sel"][untouched], 1), np.sort(sel0[untouched], 1))
    # each overloaded expert kept holders that rank at least as high as any
    # holder it evicted
    a = (s - raw["p"][None, :]).astype(F32)
    key = R.f32_key(a).astype(np.int64)
    for e in over:
        before = np.nonzero((sel0 == e).any(axis=1))[0]
        after = set(np.nonzero((r["sel"] == e).any(axis=1))[0].tolist())
        kept = [t for t in before if t in after]
        gone = [t for t in before if t not in after]
        assert len(kept) == C
        if gone:
            assert min((key[t, e], -t) for t in kept) > max((key[t, e], -t) for t in gone)


def test_max_flow_agrees_on_feasibility():
    # the capped repair result is one feasible routing; max-flow must agree
    s = synth.make_logits(120, 6, 1.5, seed=4)
    k, C = 2, synth.capacity(120, 2, 6)
    r = R.route(s, k, C, max_iters=0)
    assert r["status"] == R.OK
    allowed = np.zeros((120, 6), bool)
    allowed[np.arange(120)[:, None], r["sel"]] = True
    assert certify.max_flow_feasible(allowed, k, C)
    assert certify.max_flow_feasible(np.ones((120, 6), bool), k, C)
    assert not certify.max_flow_feasible(np.ones((120, 6), bool), k, (120 * k) // 6 - 1)


def test_status_codes():
    s = synth.tiny_logits(10, 4, 0)
    assert R.route(s, 5, 100)["status"] == R.EINFEASIBLE  # k > E
    assert R.route(s, 2, 4)["status"] == R.EINFEASIBLE  # E*C < T*k
    bad = s.copy()
    bad[3, 1] = np.nan
    assert R.route(bad, 2, 10)["status"] == R.ENAN


def test_gate_weights_are_the_softmax_of_the_selected_logits():
    s = synth.tiny_logits(40, 7, 2)
    r = R.route(s, 3, 40)
    z = np.take_along_axis(s.astype(np.float64), r["sel"], axis=1)
    np.testing.assert_allclose(r["w"], scipy.special.softmax(z, axis=1), rtol=1e-14)
