"""GPU parity of the projected dual subgradient price rule
(MOE_PRICE_SUBGRAD) against the FP32 replica of the oracle, through the C
ABI: prices, update count, increment, routing, loads and weights
bit-identical given the same logits (route from logits and from tokens),
including batches that stop at the update cap and go through the capacity
repair."""
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


def _cfg(T, E, k, max_iters=50, cap=None):
    C = synth.capacity(T, k, E) if cap is None else cap
    return L.make_cfg(T, 8, E, k, 1, C, max_iters, L.MOE_F32, L.MOE_F32, L.MOE_PRICE_SUBGRAD)


# (T, E, k, Zipf, logit scale, seed, update cap): the small FP32 workload's
# shape, an uneven batch, the BF16 workload's shape, 256 experts, a batch
# past 16384 tokens, a top-16 batch, a cap of 3 updates (repair runs)
CASES = [(512, 8, 2, 1.1, 0.226, 301, 50), (3001, 48, 6, 1.2, 0.64, 302, 50),
         (16384, 64, 8, 1.2, 0.64, 303, 50), (9001, 256, 8, 1.3, 0.905, 304, 50),
         (20000, 64, 8, 1.2, 0.64, 305, 30), (2000, 40, 16, 1.2, 0.64, 306, 50),
         (4096, 32, 4, 1.4, 0.8, 307, 3)]


@pytest.mark.parametrize("T,E,k,s_z,scale,seed,cap", CASES)
def test_subgradient_route_bit_exact(T, E, k, s_z, scale, seed, cap):
    s = synth.make_logits(T, E, s_z, seed, scale)
    cfg = _cfg(T, E, k, cap)
    r = P.route_logits(cfg, torch.from_numpy(s).cuda())
    torch.cuda.synchronize()
    ref = replica_route(cfg, s)
    assert ref["status"] == R.OK
    assert_route_matches(cfg, r, ref)
    assert ref["iters"] >= 1  # these batches start over capacity
    assert np.all(ref["load"] <= cfg.capacity)


def test_subgradient_cap_of_zero_is_plain_top_k_then_repair():
    T, E, k = 3000, 16, 2
    s = synth.make_logits(T, E, 1.3, 311, 0.64)
    cfg = _cfg(T, E, k, max_iters=0)
    r = P.route_logits(cfg, torch.from_numpy(s).cuda())
    torch.cuda.synchronize()
    ref = replica_route(cfg, s)
    assert ref["iters"] == 0 and ref["enforced"]
    assert_route_matches(cfg, r, ref)


def test_subgradient_route_from_tokens():
    shape = synth.SHAPES[1]
    inp = synth.make_inputs(shape, 1, experts=False)
    d, _ = device_inputs(shape, inp)
    cfg = cfg_for(shape, price_mode=L.MOE_PRICE_SUBGRAD)
    r = layer.route(cfg, d["X"], d["Wr"], d["br"])
    torch.cuda.synchronize()
    assert_route_matches(cfg, r, replica_route(cfg, r["logits"].cpu().numpy()))
