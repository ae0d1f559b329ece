"""GPU parity of the layer forward against the CPU oracle, through the C ABI.

Routing (indices, loads, prices, iteration counts, sigma, eps) must be
bit-identical to the FP32 replica run on the GPU's own logits; logits and
outputs are compared with the FP64 oracle within stated tolerances:
  logits   rel. Frobenius <= 1e-6 (FP32 accumulation over d <= 4096)
  FP32 layer outputs      <= 1e-5
  BF16 layer outputs      <= 1.5e-2 (h, Y, out stored in BF16; the oracle
                           sees the same BF16-rounded X and weights)
Each output bar holds for the relative Frobenius error, for max |diff| /
max |ref| and (at twice the bar) for the worst row's relative error, so a
single wrong row at a ragged tile edge cannot hide in the norm.  BF16
storage alone gives about 4e-3 on the last two (FP64 emulation of the
roundings at the ragged and tiny shapes).
"""
import numpy as np
import pytest
import torch

from oracle import ffn, routing as R
from paper_2606_17065_amd import _lib as L
from paper_2606_17065_amd import layer, synth

from _helpers import (assert_close, assert_route_matches, cfg_for, device_inputs, rel_fro,
                      replica_route)

pytestmark = pytest.mark.gpu

MID = synth.MoEShape("bf16-ragged", T=3000, d=256, E=16, k=4, f=192, zipf=1.2, act="bf16", w="bf16")
SMALL_BF16 = synth.MoEShape("bf16-tiny", T=200, d=128, E=8, k=2, f=64, zipf=1.0, act="bf16", w="bf16")
# every expert GEMM on the 256-row tile path, several ragged row tiles per expert
BIG_TILES = synth.MoEShape("bf16-bigtile", T=2100, d=512, E=8, k=2, f=384, zipf=1.1, act="bf16", w="bf16")
# top-8 (the slot count the combine kernel unrolls)
TOP8 = synth.MoEShape("bf16-top8", T=700, d=256, E=16, k=8, f=128, zipf=1.2, act="bf16", w="bf16")


def _run_route(shape, config, mode=L.MOE_PRICE_ACP, max_iters=None, price=None, rep=0):
    inp = synth.make_inputs(shape, config, rep, experts=False)
    d, h = device_inputs(shape, inp)
    cfg = cfg_for(shape, mode, max_iters)
    pr = None if price is None else torch.from_numpy(np.asarray(price, np.float32)).cuda()
    r = layer.route(cfg, d["X"], d["Wr"], d["br"], price=pr.clone() if pr is not None else None)
    torch.cuda.synchronize()
    return cfg, inp, d, h, r


@pytest.mark.parametrize("shape,config", [(synth.SHAPES[1], 1), (MID, 11), (synth.SHAPES[2], 2)])
def test_route_acp_bit_exact(shape, config):
    cfg, inp, d, h, r = _run_route(shape, config)
    s = r["logits"].cpu().numpy()
    assert rel_fro(s, R.logits_fp64(h["X"], h["Wr"], h["br"])) <= 1e-6
    ref = replica_route(cfg, s)
    assert ref["iters"] > 0  # the skewed bias overloads plain top-k
    assert_route_matches(cfg, r, ref)


@pytest.mark.parametrize("mode", [L.MOE_PRICE_NONE, L.MOE_PRICE_GIVEN, L.MOE_PRICE_WARM])
def test_route_other_price_modes(mode):
    shape = MID
    price = np.linspace(0.0, 0.5, shape.E).astype(np.float32)
    cfg, inp, d, h, r = _run_route(shape, 12, mode, price=price)
    s = r["logits"].cpu().numpy()
    ref = replica_route(cfg, s, price)
    assert_route_matches(cfg, r, ref)


@pytest.mark.parametrize("max_iters", [0, 1, 3])
def test_route_capped_loop_runs_the_repair(max_iters):
    cfg, inp, d, h, r = _run_route(MID, 13, L.MOE_PRICE_ACP, max_iters=max_iters)
    s = r["logits"].cpu().numpy()
    ref = replica_route(cfg, s)
    assert ref["enforced"]
    assert_route_matches(cfg, r, ref)
    idx = r["idx"].cpu().numpy()
    assert np.bincount(idx.ravel(), minlength=MID.E).max() <= MID.capacity


def test_route_nan_logit_reports_status():
    shape = SMALL_BF16
    inp = synth.make_inputs(shape, 14)
    inp["X"][17, 3] = np.nan
    d, h = device_inputs(shape, inp)
    cfg = cfg_for(shape)
    r = layer.route(cfg, d["X"], d["Wr"], d["br"])
    torch.cuda.synchronize()
    assert int(r["info"][L.INFO_STATUS]) == L.MOE_ENAN
    # defined outputs: the placeholder routing idx[t][j] = j with NaN
    # weights and its loads, so nothing downstream reads unwritten memory
    np.testing.assert_array_equal(r["idx"].cpu().numpy(),
                                  np.tile(np.arange(shape.k, dtype=np.int32), (shape.T, 1)))
    assert torch.isnan(r["w"]).all()
    np.testing.assert_array_equal(r["load"].cpu().numpy(),
                                  [shape.T if e < shape.k else 0 for e in range(shape.E)])
    # the layer raises on it (checked forward), or leaves a NaN output
    with pytest.raises(L.MoEError) as e:
        layer.forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"])
    assert e.value.status == L.MOE_ENAN
    out = layer.forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"], check=False)
    torch.cuda.synchronize()
    assert torch.isnan(out["out"].float()).all()


def test_route_empty_batch():
    shape = SMALL_BF16.with_tokens(0)
    inp = synth.make_inputs(shape, 15, experts=False)
    d, h = device_inputs(shape, inp)
    r = layer.route(cfg_for(shape, capacity=0), d["X"], d["Wr"], d["br"])
    torch.cuda.synchronize()
    info = r["info"].cpu().numpy()
    assert info[L.INFO_STATUS] == 0 and info[L.INFO_CONVERGED] == 1
    assert np.all(r["load"].cpu().numpy() == 0)


def test_route_is_deterministic():
    cfg, inp, d, h, r1 = _run_route(MID, 16)
    r2 = layer.route(cfg, d["X"], d["Wr"], d["br"])
    torch.cuda.synchronize()
    for key in ("logits", "idx", "w", "load", "price", "info"):
        assert torch.equal(r1[key], r2[key]), key


@pytest.mark.parametrize("shape,config", [(synth.SHAPES[1], 1), (MID, 17)])
def test_dispatch_exact(shape, config):
    cfg, inp, d, h, r = _run_route(shape, config)
    dsp = layer.dispatch(cfg, d["X"], r["idx"])
    torch.cuda.synchronize()
    sel = r["idx"].cpu().numpy()
    off, row_map, inv = ffn.dispatch_maps(sel, shape.E)
    np.testing.assert_array_equal(dsp["offsets"].cpu().numpy(), off)
    np.testing.assert_array_equal(dsp["row_map"].cpu().numpy(), row_map)
    np.testing.assert_array_equal(dsp["inv_map"].cpu().numpy(), inv)
    assert torch.equal(dsp["X_perm"], d["X"][dsp["row_map"].long()])


def _layer_check(shape, config, tol):
    inp = synth.make_inputs(shape, config)
    d, h = device_inputs(shape, inp)
    cfg = cfg_for(shape)
    out = layer.forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"])
    torch.cuda.synchronize()
    sel = out["idx"].cpu().numpy()
    assert_route_matches(cfg, out, replica_route(cfg, out["logits"].cpu().numpy()))
    # FP64 oracle on the same routing, weights from the FP64 logits
    s64 = R.logits_fp64(h["X"], h["Wr"], h["br"])
    w64 = R.gate_weights(s64, sel)
    ref = ffn.layer_forward(h["X"], sel, w64, h["W13"], h["W2"])
    errY = assert_close(out["Y"].float().cpu().numpy(), ref["Y"], tol, "Y")
    errO = assert_close(out["out"].float().cpu().numpy(), ref["out"], tol, "out")
    return errY, errO


def test_layer_forward_fp32_small_config():
    _layer_check(synth.SHAPES[1], 1, 1e-5)


def test_layer_forward_fp32_unaligned_widths():
    """FP32 layer with d and d_ff that fill no tile (d = 72, d_ff = 40):
    the guarded FP32 kernels against the FP64 oracle."""
    shape = synth.MoEShape("fp32-odd", T=300, d=72, E=6, k=2, f=40, zipf=1.1, act="f32", w="f32")
    _layer_check(shape, 41, 1e-5)


def test_layer_forward_bf16_ragged():
    _layer_check(MID, 18, 1.5e-2)


def test_layer_forward_bf16_big_tiles():
    _layer_check(BIG_TILES, 21, 1.5e-2)


def test_layer_forward_bf16_tiny():
    _layer_check(SMALL_BF16, 19, 1.5e-2)


@pytest.mark.parametrize("shape", [MID, TOP8], ids=["top4", "top8"])
def test_combine_matches_oracle_on_gpu_y(shape):
    inp = synth.make_inputs(shape, 20)
    d, h = device_inputs(shape, inp)
    cfg = cfg_for(shape)
    out = layer.forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"])
    torch.cuda.synchronize()
    Y = out["Y"].float().cpu().double().numpy()
    ref = ffn.combine(Y, out["inv_map"].cpu().numpy(), out["w"].cpu().numpy().astype(np.float64))
    got = out["out"].float().cpu().numpy()
    # only the final BF16 rounding separates the two
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3)) <= 2 ** -8


def test_layer_forward_bf16_scale_config_sampled():
    shape = synth.SHAPES[2]
    inp = synth.make_inputs(shape, 2)
    d, h = device_inputs(shape, inp, host_weights=False)
    del inp
    cfg = cfg_for(shape)
    out = layer.forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"])
    torch.cuda.synchronize()
    sel = out["idx"].cpu().numpy()
    assert_route_matches(cfg, out, replica_route(cfg, out["logits"].cpu().numpy()))
    rng = np.random.default_rng(0)
    toks = np.sort(rng.choice(shape.T, 48, replace=False))
    s64 = R.logits_fp64(h["X"][toks], h["Wr"], h["br"])
    w64 = R.gate_weights(s64, sel[toks])
    got = out["out"].float().cpu().numpy()[toks]
    exp = np.zeros_like(got, dtype=np.float64)
    for i, t in enumerate(toks):
        for j in range(shape.k):
            e = sel[t, j]
            W13e = d["W13"][e].float().cpu().double().numpy()
            W2e = d["W2"][e].float().cpu().double().numpy()
            _, _, _, y = ffn.expert_forward(h["X"][t:t + 1], W13e, W2e)
            exp[i] += w64[i, j] * y[0]
    assert_close(got, exp, 1.5e-2, "out (sampled tokens)")


@pytest.mark.parametrize("base", ["ragged", "fused"])
@pytest.mark.parametrize("T", [0, 1, 5, 130])
def test_layer_forward_tiny_batches(T, base):
    """Empty, single-token and sub-tile batches through every stage of the
    layer, on the explicit-permute path (d_ff = 192) and on the path with
    the permute fused into the first expert product."""
    full = MID if base == "ragged" else BIG_TILES
    shape = full.with_tokens(T)
    cfg = cfg_for(shape, capacity=max(1, synth.capacity(T, shape.k, shape.E)))
    assert layer.gather_fused(cfg) == (base == "fused")
    inp = synth.make_inputs(full.with_tokens(max(T, 1)), 19)
    d, h = device_inputs(shape, {**inp, "X": inp["X"][:T]})
    r = layer.forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"])
    torch.cuda.synchronize()
    assert int(r["info"][L.INFO_STATUS]) == 0
    assert r["out"].shape == (T, shape.d)
    if T == 0:
        assert int(r["load"].sum()) == 0
        return
    sel = r["idx"].cpu().numpy()
    assert all(len(set(row)) == shape.k for row in sel)
    ref = ffn.layer_forward(h["X"], sel, r["w"].cpu().numpy().astype(np.float64), h["W13"],
                            h["W2"])
    assert_close(r["out"].float().cpu().numpy(), ref["out"], 1.5e-2, "out")


@pytest.mark.parametrize("which", ["bigtile", "scale"])
def test_fused_gather_matches_separate_permute(which):
    """The first expert product reading X through row_map gives the same
    bits as the explicit permute followed by the product, at a small shape
    and at 16384 tokens (E = 64, top-8), whose 256-row tiles fill the XCDs'
    runs unevenly."""
    shape = BIG_TILES if which == "bigtile" else synth.SHAPES[2]
    cfg = cfg_for(shape)
    assert layer.gather_fused(cfg)
    inp = synth.make_inputs(shape, 23 if which == "bigtile" else 2)
    d, _ = device_inputs(shape, inp, host_weights=False)
    a = layer.forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"], fuse=True)
    b = layer.forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"], fuse=False)
    torch.cuda.synchronize()
    assert a["X_perm"] is None and b["X_perm"] is not None
    assert torch.equal(a["Y"], b["Y"]) and torch.equal(a["out"], b["out"])
