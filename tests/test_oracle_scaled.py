"""Pins of the epsilon-scaled restarts of the clearing-price update (the
price-rule variant): exhaustive enumeration and the HiGHS LP bracket the
routing it returns, the zero-price case stays at p = 0, the first stage is
the plain update, and on the small workload (and the 4096-token, 64-expert
batches below) the certificate gap it reaches is below the plain update's."""
import numpy as np
import pytest

from oracle import certify, routing as R
from paper_2606_17065_amd import synth

F32 = np.float32
STAGES = 3


def _gap(s, r, k, C):
    prim = R.primal_objective(s, r["sel"])
    D = R.dual_objective(s, r["p"], k, C)
    return prim, D, (D - prim) / abs(D)


@pytest.mark.parametrize("T,E,k", [(6, 4, 2), (5, 4, 2), (6, 3, 1), (4, 4, 3)])
@pytest.mark.parametrize("seed", range(6))
def test_scaled_brute_force_bracket(T, E, k, seed):
    s = synth.tiny_logits(T, E, 300 + seed)
    C = synth.capacity(T, k, E)
    r = R.route(s, k, C, stages=STAGES)
    assert r["status"] == R.OK
    load = np.bincount(r["sel"].ravel(), minlength=E)
    assert load.max() <= C and all(len(set(row)) == k for row in r["sel"].tolist())
    opt, _ = certify.brute_force_opt(s, k, C)
    prim, D, _ = _gap(s, r, k, C)
    assert prim <= opt + 1e-12 <= D + 1e-9
    if not r["enforced"]:
        ident = float(np.sum(r["p"].astype(np.float64) * (C - r["load"])))
        assert abs((D - prim) - ident) <= 1e-6 * max(1.0, abs(D))


@pytest.mark.parametrize("seed", range(3))
def test_scaled_lp_bracket_and_smaller_gap_small_config(seed):
    sh = synth.SHAPES[1]
    inp = synth.make_inputs(sh, 1, rep=seed, experts=False)
    s = (inp["X"].astype(np.float64) @ inp["Wr"].T.astype(np.float64) + inp["br"]).astype(F32)
    C = sh.capacity
    plain = R.route(s, sh.k, C)
    r = R.route(s, sh.k, C, stages=STAGES)
    assert r["status"] == R.OK
    if not plain["converged"]:
        # no restart after a stage that hit the cap: the plain routing
        np.testing.assert_array_equal(r["sel"], plain["sel"])
        assert r["iters"] == plain["iters"]
        return
    assert r["converged"]
    opt, _ = certify.lp_opt(s, sh.k, C)
    prim, D, gap = _gap(s, r, sh.k, C)
    assert prim <= opt + 1e-9 <= D + 2e-9
    assert (opt - prim) / abs(opt) <= gap + 1e-12
    _, _, gap0 = _gap(s, plain, sh.k, C)
    assert gap <= gap0
    assert gap <= 1e-4


def test_scaled_gap_shrinks_on_wider_batches():
    for seed in (1, 2):
        T, E, k = 4096, 64, 8
        s = synth.make_logits(T, E, 1.2, seed)
        C = synth.capacity(T, k, E)
        plain = R.route(s, k, C)
        r = R.route(s, k, C, stages=STAGES)
        assert r["converged"] and not r["enforced"]
        _, _, g0 = _gap(s, plain, k, C)
        _, _, g = _gap(s, r, k, C)
        assert g < 0.25 * g0, (g, g0)


def test_scaled_first_stage_is_the_plain_update():
    s = synth.make_logits(800, 16, 1.2, seed=5)
    k, C = 4, synth.capacity(800, 4, 16)
    plain = R.acp_prices(s, k, C, 50)
    one = R.acp_scaled_prices(s, k, C, 50, stages=0)
    np.testing.assert_array_equal(plain["p"].view(np.uint32), one["p"].view(np.uint32))
    assert one["iters"] == plain["iters"] and one["stages_run"] == 0
    # one restart: prices start 4 increments lower (not below 0), the
    # increment is an eighth
    two = R.acp_scaled_prices(s, k, C, 50, stages=1)
    assert two["stages_run"] == 1 and two["eps"] == F32(plain["eps"] / F32(8))
    p1 = (plain["p"] - F32(4 * plain["eps"])).astype(F32)
    p1 = np.where(p1 > 0, p1, F32(0)).astype(F32)
    three = R.acp_prices(s, k, C, 50, p0=p1, eps=two["eps"])
    np.testing.assert_array_equal(three["p"].view(np.uint32), two["p"].view(np.uint32))
    assert two["iters"] == plain["iters"] + three["iters"]


def test_scaled_stops_once_the_gap_is_zero():
    """A stage that ends with every priced expert full (zero gap) is not
    restarted: the 512-token workload's third batch reaches that in the
    plain update already."""
    sh = synth.SHAPES[1]
    inp = synth.make_inputs(sh, 1, rep=2, experts=False)
    s = (inp["X"].astype(np.float64) @ inp["Wr"].T.astype(np.float64) + inp["br"]).astype(F32)
    plain = R.route(s, sh.k, sh.capacity)
    r = R.route(s, sh.k, sh.capacity, stages=STAGES)
    _, _, g0 = _gap(s, plain, sh.k, sh.capacity)
    assert g0 == 0.0
    assert r["iters"] == plain["iters"] and r["eps"] == plain["eps"]
    np.testing.assert_array_equal(r["p"].view(np.uint32), plain["p"].view(np.uint32))


def test_scaled_zero_prices_when_capacity_is_slack():
    s = synth.tiny_logits(50, 6, 3)
    r = R.route(s, 2, 50, stages=STAGES)
    assert r["iters"] == 0 and np.all(r["p"] == 0) and not r["enforced"]
