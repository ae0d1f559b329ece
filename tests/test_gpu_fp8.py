"""GPU parity of the FP8 (OCP e4m3, per-block scales) expert path against
the CPU oracle, through the C ABI.

Bars:
  quantisation (tokens 1 x 128 in the dispatch, weights 128 x 128, h):
      codes and scales bit-identical to the oracle's quantiser run on the
      same FP32 / BF16 values;
  expert outputs Y and layer output: rel. Frobenius <= 1e-2 against the
      FP8-emulating FP64 oracle (its h is rounded to BF16 and re-quantised
      like the GPU's; a BF16 rounding of h on either side can move an FP8
      code by one step, up to an eighth of that element), worst row <= 1e-1
      (one moved code of a large h element shifts a row of Y by a few 1e-2
      at d_ff = 128; a wrong or zeroed row gives about 1), max |diff| /
      max |ref| <= 3e-2: when the BF16 rounding of a block's largest h
      element differs, that block's scale differs and every one of its 128
      codes can move by a step at once (1.3-1.5e-2 of max |Y| measured at
      these shapes, with GEMM 2 on the GPU's own h codes agreeing to 2.3e-3,
      the BF16 rounding of Y); rel. Frobenius <= 8e-2 against the FP64 layer
      on the same BF16 tokens and unquantised weights (the FP8 rounding
      itself, about 6.4e-2 in an FP64 emulation at these shapes).
"""
import numpy as np
import pytest
import torch

from oracle import ffn, fp8
from oracle import routing as R
from paper_2606_17065_amd import _lib as L
from paper_2606_17065_amd import layer, synth

from _helpers import assert_close, assert_route_matches, cfg_for, device_inputs, rel_fro, replica_route

pytestmark = pytest.mark.gpu

F32 = np.float32


def _bf16(x):
    return torch.from_numpy(np.asarray(x, F32)).to(torch.bfloat16)


def _mixed_rows(R_, C, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((R_, C)) * np.exp(rng.uniform(-6, 6, (R_, 1)))
    x[3, :128] = 0.0  # an all-zero block
    x[4, 128:256] = -0.0
    x[5, :] *= 1e-3
    x[6, 5] = 1e4
    return x.astype(F32)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_quantize_rows_bit_exact(dtype):
    x = _mixed_rows(333, 384, 1)
    xd = torch.from_numpy(x).to(dtype).cuda()
    q, s = layer.quantize_fp8(xd, 1)
    torch.cuda.synchronize()
    xv = xd.float().cpu().numpy()
    rq, rs = fp8.quantize_blocks(xv, 1, 128)
    np.testing.assert_array_equal(q.cpu().numpy(), rq)
    np.testing.assert_array_equal(s.cpu().numpy().view(np.uint32), rs.view(np.uint32))


def test_quantize_rows_codes_at_every_rounding_midpoint():
    """Every e4m3 value, every midpoint between neighbours (ties to even)
    and the FP32 values just beside each midpoint, both signs: in 1 x 128
    blocks whose largest magnitude is 448, so the
    inverse scale is exactly 1 and each code is the encoding of the value
    itself; the GPU codes must equal the oracle's."""
    mags = fp8.decode(np.arange(0, 127, dtype=np.uint8)).astype(np.float64)  # 0 .. 448
    mids = (mags[:-1] + mags[1:]) / 2.0
    m32 = mids.astype(F32)
    assert np.array_equal(m32.astype(np.float64), mids)  # midpoints are FP32 values
    below = np.nextafter(m32, F32(0.0))
    above = np.nextafter(m32, F32(np.inf))
    pos = np.concatenate([mags.astype(F32), m32, below, above, F32([2.0 ** -10, 2.0 ** -12])])
    pos = pos[pos <= 448.0]
    v = np.concatenate([pos, -pos]).astype(F32)
    per = 127  # values per block; the block's first element is 448
    nb = -(-v.size // per)
    x = np.zeros((nb, 128), F32)
    x[:, 0] = 448.0
    x.reshape(-1)[np.arange(v.size) // per * 128 + 1 + np.arange(v.size) % per] = v
    xd = torch.from_numpy(x).cuda()
    q, s_ = layer.quantize_fp8(xd, 1)
    torch.cuda.synchronize()
    rq, rs = fp8.quantize_blocks(x, 1, 128)
    assert np.all(rs == 1.0)
    np.testing.assert_array_equal(q.cpu().numpy(), rq)
    np.testing.assert_array_equal(s_.cpu().numpy().view(np.uint32), rs.view(np.uint32))


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_quantize_expert_tiles_bit_exact(dtype):
    rng = np.random.Generator(np.random.PCG64(2))
    W = (0.02 * rng.standard_normal((3, 384, 256))).astype(F32)
    W[1, :128, 128:] = 0.0
    W[2] *= 50.0
    Wd = torch.from_numpy(W).to(dtype).cuda()
    q, s = layer.quantize_fp8(Wd, 128)
    torch.cuda.synchronize()
    rq, rs = fp8.quantize_experts(Wd.float().cpu().numpy())
    np.testing.assert_array_equal(q.cpu().numpy(), rq)
    np.testing.assert_array_equal(s.cpu().numpy().view(np.uint32), rs.view(np.uint32))


def test_quantize_ragged_row_tiles():
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.standard_normal((300, 256)).astype(F32)
    q, s = layer.quantize_fp8(torch.from_numpy(x).cuda(), 128)
    torch.cuda.synchronize()
    rq, rs = fp8.quantize_blocks(x, 128, 128)
    assert tuple(s.shape) == (3, 2)
    np.testing.assert_array_equal(q.cpu().numpy(), rq)
    np.testing.assert_array_equal(s.cpu().numpy(), rs)


FP8_SMALL = synth.MoEShape("fp8-small", T=700, d=256, E=8, k=2, f=256, zipf=1.2, act="bf16",
                           w="fp8")
FP8_WIDE = synth.MoEShape("fp8-wide", T=1300, d=512, E=8, k=2, f=384, zipf=1.2, act="bf16",
                          w="fp8")
# T not a multiple of the 4 rows a quantising block handles, an odd number
# of experts, top-3, one 128-wide K block in GEMM 2
FP8_ODD = synth.MoEShape("fp8-odd", T=333, d=256, E=5, k=3, f=128, zipf=1.1, act="bf16", w="fp8")
# d % 256 != 0: the second product on 256 x 128 tiles instead of 128 x 256,
# top-8 (the compile-time slot count of the combine)
FP8_D384 = synth.MoEShape("fp8-d384", T=500, d=384, E=12, k=8, f=256, zipf=1.2, act="bf16",
                          w="fp8")


def _fp8_case(shape, config):
    inp = synth.make_inputs(shape, config)
    d, h = device_inputs(dataclass_bf16(shape), inp)
    cfg = cfg_for(shape)
    W13d = torch.from_numpy(inp["W13"]).to(torch.bfloat16).cuda()
    W2d = torch.from_numpy(inp["W2"]).to(torch.bfloat16).cuda()
    q13, s13 = layer.quantize_fp8(W13d, 128)
    q2, s2 = layer.quantize_fp8(W2d, 128)
    return cfg, inp, d, h, W13d, W2d, q13, s13, q2, s2


def dataclass_bf16(shape):
    import dataclasses
    return dataclasses.replace(shape, w="bf16")


@pytest.mark.parametrize("shape,config", [(FP8_SMALL, 31), (FP8_WIDE, 32), (FP8_ODD, 33),
                                          (FP8_D384, 34)])
def test_fp8_layer_matches_emulating_oracle(shape, config):
    cfg, inp, d, h, W13d, W2d, q13, s13, q2, s2 = _fp8_case(shape, config)
    r = layer.forward(cfg, d["X"], d["Wr"], d["br"], q13, q2, W13_scale=s13, W2_scale=s2)
    torch.cuda.synchronize()
    assert int(r["info"][L.INFO_STATUS]) == 0
    sel = r["idx"].cpu().numpy()
    offsets, row_map, inv_map = ffn.dispatch_maps(sel, shape.E)
    np.testing.assert_array_equal(r["offsets"].cpu().numpy(), offsets)
    np.testing.assert_array_equal(r["row_map"].cpu().numpy(), row_map)
    # the oracle quantises the same BF16 weights itself
    W13v = W13d.float().cpu().numpy()
    W2v = W2d.float().cpu().numpy()
    oq13, os13 = fp8.quantize_experts(W13v)
    oq2, os2 = fp8.quantize_experts(W2v)
    np.testing.assert_array_equal(q13.cpu().numpy(), oq13)
    np.testing.assert_array_equal(s2.cpu().numpy(), os2)
    ref = fp8.slots_forward_fp8(h["X"], row_map, offsets, oq13, os13, oq2, os2)
    # token codes and scales (quantised once per token, gathered by GEMM 1):
    # bit-exact
    assert r["X_perm"] is None
    np.testing.assert_array_equal(r["X_codes"].cpu().numpy(), ref["Xq"])
    np.testing.assert_array_equal(r["X_scale"].cpu().numpy(), ref["Xs"])
    Y = r["Y"].float().cpu().numpy()
    # the unfused path (slot-ordered codes written by the dispatch, then
    # the expert products) gives the same codes and the same Y bit for bit
    u = layer.forward(cfg, d["X"], d["Wr"], d["br"], q13, q2, W13_scale=s13, W2_scale=s2,
                      fuse=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u["X_perm"].cpu().numpy(), ref["Xq"][row_map])
    np.testing.assert_array_equal(u["X_perm_scale"].cpu().numpy(), ref["Xs"][row_map])
    np.testing.assert_array_equal(u["Y"].view(torch.int16).cpu().numpy(),
                                  r["Y"].view(torch.int16).cpu().numpy())
    assert_close(Y, ref["Y"], 1e-2, "Y", row_tol=1e-1, max_tol=3e-2)
    w = r["w"].cpu().numpy()
    out_ref = ffn.combine(ref["Y"], inv_map, w)
    assert_close(r["out"].float().cpu().numpy(), out_ref, 1e-2, "out", row_tol=1e-1,
                 max_tol=3e-2)
    # against the unquantised FP64 layer on the same BF16 tokens and weights
    _, _, Y64 = ffn.slots_forward(h["X"], row_map, offsets, W13v, W2v)
    assert rel_fro(Y, Y64) <= 8e-2


def test_fp8_gather_ffn_rejects_bad_arguments():
    shape = synth.MoEShape("fp8-bad", T=64, d=192, E=4, k=2, f=256, zipf=1.0, act="bf16", w="fp8")
    x = torch.zeros(128, 256, dtype=torch.uint8, device="cuda")
    p = x.data_ptr()
    with pytest.raises(L.MoEError) as e:  # d % 128 != 0
        L.moe_expert_ffn_gather_fp8(cfg_for(shape), p, p, p, p, p, p, p, p, p, p, 1 << 30, 0)
    assert e.value.status == L.MOE_EUNSUPPORTED
    ok = synth.MoEShape("fp8-ok", T=64, d=256, E=4, k=2, f=256, zipf=1.0, act="bf16", w="fp8")
    with pytest.raises(L.MoEError) as e:  # no scales for the token codes
        L.moe_expert_ffn_gather_fp8(cfg_for(ok), p, None, p, p, p, p, p, p, p, p, 1 << 30, 0)
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:  # BF16 experts take moe_expert_ffn_gather
        L.moe_expert_ffn_gather_fp8(cfg_for(dataclass_bf16(ok)), p, p, p, p, p, p, p, p, p, p,
                                    1 << 30, 0)
    assert e.value.status == L.MOE_EUNSUPPORTED


def test_fp8_ffn_rejects_unaligned_widths():
    shape = synth.MoEShape("fp8-bad", T=64, d=192, E=4, k=2, f=256, zipf=1.0, act="bf16", w="fp8")
    cfg = cfg_for(shape)
    x = torch.zeros(128, 192, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.MoEError) as e:
        L.moe_expert_ffn(cfg, x.data_ptr(), x.data_ptr(), x.data_ptr(), x.data_ptr(),
                         x.data_ptr(), x.data_ptr(), x.data_ptr(), x.data_ptr(), x.data_ptr(),
                         1 << 30, 0)
    assert e.value.status == L.MOE_EUNSUPPORTED


def test_fp8_experts_config_sampled():
    """The FP8-expert workload at full size (T=65536, d=4096, E=64, top-8,
    d_ff=1408) in the configuration the benchmark times; two tokens are
    checked against the FP8-emulating oracle on two of their experts each
    (the oracle quantises those experts' BF16 weights itself)."""
    shape = synth.SHAPES[3]
    inp = synth.make_inputs(shape, 3)
    X = torch.from_numpy(inp["X"]).to(torch.bfloat16).cuda()
    Wr = torch.from_numpy(inp["Wr"]).cuda()
    br = torch.from_numpy(inp["br"]).cuda()
    W13 = torch.from_numpy(inp["W13"]).to(torch.bfloat16).cuda()
    W2 = torch.from_numpy(inp["W2"]).to(torch.bfloat16).cuda()
    del inp
    q13, s13 = layer.quantize_fp8(W13, 128)
    q2, s2 = layer.quantize_fp8(W2, 128)
    cfg = cfg_for(shape)
    r = layer.forward(cfg, X, Wr, br, q13, q2, W13_scale=s13, W2_scale=s2)
    torch.cuda.synchronize()
    info = r["info"].cpu().numpy()
    assert int(info[L.INFO_STATUS]) == 0
    assert int(r["load"].max()) <= cfg.capacity
    # routing of the full batch (65536 tokens: each selection block streams
    # its margin column) bit-exact against the FP32 replica
    assert_route_matches(cfg, r, replica_route(cfg, r["logits"].cpu().numpy()))
    sel = r["idx"].cpu().numpy()
    inv = r["inv_map"].cpu().numpy()
    Y = r["Y"]
    for t in (0, shape.T - 1):
        xt = X[t:t + 1].float().cpu().numpy()
        xq, xs = fp8.quantize_blocks(xt, 1, 128)
        np.testing.assert_array_equal(r["X_codes"][t].cpu().numpy(), xq[0])
        np.testing.assert_array_equal(r["X_scale"][t].cpu().numpy(), xs[0])
        xd = fp8.dequantize_blocks(xq, xs, 1, 128)
        for j in (0, shape.k - 1):
            e = int(sel[t, j])
            w13q, w13s = fp8.quantize_blocks(W13[e].float().cpu().numpy(), 128, 128)
            np.testing.assert_array_equal(q13[e].cpu().numpy(), w13q)
            w2q, w2s = fp8.quantize_blocks(W2[e].float().cpu().numpy(), 128, 128)
            Wd = fp8.dequantize_blocks(w13q, w13s, 128, 128)
            A = xd @ Wd[:shape.f].T
            B = xd @ Wd[shape.f:].T
            h = fp8.round_bf16(A / (1.0 + np.exp(-A)) * B)
            hq, hs = fp8.quantize_blocks(h.astype(np.float32), 1, 128)
            y = fp8.dequantize_blocks(hq, hs, 1, 128) @ fp8.dequantize_blocks(w2q, w2s, 128, 128).T
            got = Y[int(inv[t, j])].float().cpu().numpy()
            assert_close(got[None], y, 1e-2, f"Y of token {t}, choice {j}", row_tol=1e-1,
                         max_tol=3e-2)
