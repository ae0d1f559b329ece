"""GPU parity of the price-rule variant with epsilon-scaled restarts
(cfg.price_stages > 0) against the FP32 replica of the oracle, through the
C ABI: prices, summed update counts, the last run's increment, the routing,
loads and weights bit-identical given the same logits, in every entry point
that runs the update (route from tokens, route from logits, the update
alone, warm starts, the judged routing)."""
import numpy as np
import pytest
import torch

from oracle import routing as R
from paper_2606_17065_amd import _lib as L
from paper_2606_17065_amd import layer
from paper_2606_17065_amd import price as P
from paper_2606_17065_amd import synth

from _helpers import assert_route_matches, cfg_for, device_inputs, replica_route

pytestmark = pytest.mark.gpu

F32 = np.float32


def _cfg(T, E, k, stages, mode=L.MOE_PRICE_ACP, max_iters=50):
    return L.make_cfg(T, 8, E, k, 1, synth.capacity(T, k, E), max_iters, L.MOE_F32, L.MOE_F32,
                      mode, 0.9, stages)


# (T, E, k, Zipf, logit scale, seed, restarts): the small FP32 workload's
# shape, an uneven batch, the BF16 workload's shape, a 256-expert batch of
# the learned-price shape, a batch past the 16384-token switch of the
# selection
SCALED_CASES = [(512, 8, 2, 1.1, 0.226, 201, 3), (3001, 48, 6, 1.2, 0.64, 202, 3),
                (16384, 64, 8, 1.2, 0.64, 203, 3), (9001, 256, 8, 1.3, 0.905, 204, 2),
                (20000, 64, 8, 1.2, 0.64, 205, 1)]


@pytest.mark.parametrize("T,E,k,s_z,scale,seed,stages", SCALED_CASES)
def test_scaled_restarts_bit_exact(T, E, k, s_z, scale, seed, stages):
    s = synth.make_logits(T, E, s_z, seed, scale)
    cfg = _cfg(T, E, k, stages)
    r = P.route_logits(cfg, torch.from_numpy(s).cuda())
    torch.cuda.synchronize()
    ref = replica_route(cfg, s)
    assert ref["status"] == R.OK
    assert_route_matches(cfg, r, ref)
    # the restarts ran and did not raise the certificate gap of the plain rule
    plain = R.route(s, k, cfg.capacity, 50)
    assert ref["iters"] > plain["iters"]
    C = cfg.capacity
    g_plain = R.dual_objective(s, plain["p"], k, C) - R.primal_objective(s, plain["sel"])
    g_scaled = R.dual_objective(s, ref["p"], k, C) - R.primal_objective(s, ref["sel"])
    assert g_scaled <= g_plain


def test_scaled_restarts_warm_start_and_update_alone():
    T, E, k = 4000, 40, 5
    s = synth.make_logits(T, E, 1.2, 211, 0.64)
    sd = torch.from_numpy(s).cuda()
    p0 = torch.full((E,), 0.05, dtype=torch.float32, device="cuda")
    cfg = _cfg(T, E, k, 3, mode=L.MOE_PRICE_WARM)
    r = P.route_logits(cfg, sd, p0.clone())
    price, info = P.price_update(cfg, sd, p0.clone())
    torch.cuda.synchronize()
    ref = replica_route(cfg, s, p0.cpu().numpy())
    assert_route_matches(cfg, r, ref)
    np.testing.assert_array_equal(price.cpu().numpy().view(np.uint32),
                                  np.asarray(ref["p"], F32).view(np.uint32))
    np.testing.assert_array_equal(info.cpu().numpy(), r["info"].cpu().numpy())


def test_scaled_restarts_in_the_layer_route_from_tokens():
    """moe_route (router GEMM included) at the small FP32 workload."""
    shape = synth.SHAPES[1]
    inp = synth.make_inputs(shape, 1)
    d, _ = device_inputs(shape, inp)
    cfg = cfg_for(shape)
    cfg.price_stages = 3
    r = layer.route(cfg, d["X"], d["Wr"], d["br"])
    torch.cuda.synchronize()
    ref = replica_route(cfg, r["logits"].cpu().numpy())
    assert_route_matches(cfg, r, ref)


@pytest.mark.parametrize("tol", [1.0, 0.0])
def test_scaled_restarts_in_the_judged_route(tol):
    """Both passes of the judged routing run the restarts: the warm-started
    one (kept at tol 1) and the fallback from zero prices (tol 0)."""
    T, E, k = 3001, 48, 6
    s = synth.make_logits(T, E, 1.2, 212, 0.64)
    cfg = _cfg(T, E, k, 2)
    pstar = R.route(s, k, cfg.capacity, 50)["p"]
    phat = (pstar * F32(0.9)).astype(F32)
    r = P.judged_route(cfg, torch.from_numpy(s).cuda(), torch.from_numpy(phat).cuda(), "warm",
                       gap_tol=tol)
    torch.cuda.synchronize()
    ref = R.judged_route(s, k, cfg.capacity, phat, "warm", 0.9, tol, 50, 2)
    v = P.verdict_dict(r)
    assert v["kept"] == ref["kept"] == (tol == 1.0)
    assert v["learned_iters"] == ref["learned_iters"]
    np.testing.assert_array_equal(r["idx"].cpu().numpy(), ref["sel"])
    np.testing.assert_array_equal(r["price"].cpu().numpy().view(np.uint32),
                                  np.asarray(ref["p"], F32).view(np.uint32))
    assert int(r["info"][L.INFO_ITERS]) == ref["iters"]
    assert abs(v["gap"] - ref["gap"]) <= 1e-12
