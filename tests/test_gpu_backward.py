"""GPU parity of the layer backward against the FP64 oracle gradient
(oracle.grad, itself pinned by central differences), through the C ABI.

Tolerances (relative Frobenius against FP64): BF16 activations, weights and
stored intermediates (h, dA, dB, dY) give about 2^-8 per element, so
gradients are held to 2e-2; the FP32 dot products of the combine backward
(dw) to 1e-5 given the GPU's own Y.  Every gradient bar holds for the
relative Frobenius error and for max |diff| / max |ref|, and (at twice the
bar) for the worst row of each matrix of at least 64 columns; an FP64
emulation of the BF16 roundings gives at most 2.9e-3, 4.4e-3 and 7.6e-3 on
the three measures at these shapes.
"""
import numpy as np
import pytest
import torch

from oracle import grad, routing as R
from paper_2606_17065_amd import layer, synth

from _helpers import assert_close, assert_route_matches, cfg_for, device_inputs, replica_route

pytestmark = pytest.mark.gpu

# d % 256 == 0 and f % 128 == 0 (the backward GEMM tiling); ragged experts
BWD = synth.MoEShape("bf16-bwd", T=1500, d=256, E=8, k=2, f=256, zipf=1.2, act="bf16", w="bf16")
BWD2 = synth.MoEShape("bf16-bwd-k4", T=1100, d=512, E=16, k=4, f=384, zipf=1.3, act="bf16", w="bf16")
# top-1 over an odd number of experts (the gate gradient vanishes: one
# softmax weight is identically 1) and top-3 over seven experts
BWD_K1 = synth.MoEShape("bf16-bwd-k1", T=333, d=256, E=5, k=1, f=128, zipf=1.1, act="bf16", w="bf16")
BWD_K3 = synth.MoEShape("bf16-bwd-k3", T=250, d=256, E=7, k=3, f=256, zipf=1.2, act="bf16", w="bf16")
# top-8 (the slot count the combine and dispatch backward kernels unroll)
BWD_K8 = synth.MoEShape("bf16-bwd-k8", T=600, d=512, E=16, k=8, f=128, zipf=1.2, act="bf16", w="bf16")


def _setup(shape, config):
    inp = synth.make_inputs(shape, config)
    d, h = device_inputs(shape, inp)
    cfg = cfg_for(shape)
    fw = layer.forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"])
    dOut = torch.from_numpy(synth.make_upstream(shape.T, shape.d, config)).to(torch.bfloat16).cuda()
    torch.cuda.synchronize()
    return cfg, d, h, fw, dOut


@pytest.mark.parametrize("shape,config", [(BWD, 31), (BWD2, 32), (BWD_K1, 34), (BWD_K3, 35),
                                          (BWD_K8, 36)])
def test_backward_pieces_match_oracle(shape, config):
    cfg, d, h, fw, dOut = _setup(shape, config)
    dY, dw = layer.combine_bwd(cfg, dOut, fw["Y"], fw["inv_map"], fw["w"])
    dXp, dW13, dW2 = layer.expert_ffn_bwd(cfg, d["X"], fw["row_map"], fw["offsets"], dY, d["W13"],
                                          d["W2"])
    dX, dWr, dbr = layer.route_bwd(cfg, d["X"], d["Wr"], fw["idx"], fw["w"], dw, fw["row_map"],
                                   fw["offsets"], fw["inv_map"], dXp)
    torch.cuda.synchronize()
    sel = fw["idx"].cpu().numpy()
    dO = dOut.float().cpu().double().numpy()
    ref = grad.layer_backward(h["X"], h["Wr"], h["br"], h["W13"], h["W2"], sel, dO)
    # combine backward: dw against the GPU's own Y (FP32 dot products)
    Yg = fw["Y"].float().cpu().double().numpy()
    inv = fw["inv_map"].cpu().numpy()
    dw_exact = np.einsum("tkd,td->tk", Yg[inv], dO)
    assert_close(dw.cpu().numpy(), dw_exact, 1e-5, "dw (exact)")
    # dY = w * dOut in slot order, BF16-rounded
    wg = fw["w"].cpu().numpy().astype(np.float64)
    dY_exact = np.zeros_like(Yg)
    for j in range(shape.k):
        dY_exact[inv[:, j]] = wg[:, j:j + 1] * dO
    assert_close(dY.float().cpu().numpy(), dY_exact, 4e-3, "dY")
    # against the FP64 oracle
    assert_close(dw.cpu().numpy(), ref["dw"], 2e-2, "dw")
    assert_close(dXp.float().cpu().numpy(), ref["dXp"], 2e-2, "dXp")
    assert_close(dW13.cpu().numpy().reshape(-1, shape.d), ref["dW13"].reshape(-1, shape.d), 2e-2,
                 "dW13")
    assert_close(dW2.cpu().numpy().reshape(-1, shape.f), ref["dW2"].reshape(-1, shape.f), 2e-2,
                 "dW2")
    assert_close(dX.cpu().numpy(), ref["dX"], 2e-2, "dX")
    if shape.k == 1:
        # a single softmax weight is 1 whatever the logit: no router gradient
        assert np.abs(ref["dWr"]).max() == 0.0 and np.abs(ref["dbr"]).max() == 0.0
        assert np.abs(dWr.cpu().numpy()).max() == 0.0 and np.abs(dbr.cpu().numpy()).max() == 0.0
        return
    assert_close(dWr.cpu().numpy(), ref["dWr"], 2e-2, "dWr")
    assert_close(dbr.cpu().numpy(), ref["dbr"], 2e-2, "dbr")


@pytest.mark.parametrize("shape,config", [(BWD, 36), (BWD2, 37)])
def test_backward_bf16_outputs_are_the_rounded_fp32_results(shape, config):
    """Weight and token gradients stored as BF16 are the FP32 results rounded
    to nearest even, bit for bit (same accumulation, rounding at the store;
    the 256-wide weight-gradient tile at d_ff = 256 and the 128-wide one at
    d_ff = 384)."""
    cfg, d, h, fw, dOut = _setup(shape, config)
    dY, dw = layer.combine_bwd(cfg, dOut, fw["Y"], fw["inv_map"], fw["w"])
    outs = {}
    for dt in (torch.float32, torch.bfloat16):
        dXp, dW13, dW2 = layer.expert_ffn_bwd(cfg, d["X"], fw["row_map"], fw["offsets"], dY,
                                              d["W13"], d["W2"], grad_dtype=dt)
        dX, _, _ = layer.route_bwd(cfg, d["X"], d["Wr"], fw["idx"], fw["w"], dw, fw["row_map"],
                                   fw["offsets"], fw["inv_map"], dXp, dx_dtype=dt)
        outs[dt] = (dW13, dW2, dX)
    torch.cuda.synchronize()
    for name, a, b in zip(("dW13", "dW2", "dX"), outs[torch.float32], outs[torch.bfloat16]):
        np.testing.assert_array_equal(a.to(torch.bfloat16).view(torch.int16).cpu().numpy(),
                                      b.view(torch.int16).cpu().numpy(), err_msg=name)


@pytest.mark.parametrize("shape,config", [(BWD, 36), (BWD2, 37), (BWD_K1, 38)])
def test_saved_preactivations(shape, config):
    """The training forward (moe_expert_ffn_gather_save) stores [A|B]: Y and
    the layer output are bit-identical to the plain forward's; A and B are
    the FP64 products Xp W1^T, Xp W3^T within BF16 rounding (element-wise);
    and the backward that reads them (moe_expert_ffn_bwd_saved) returns the
    recomputing backward's gradients bit for bit, FP32 and BF16."""
    cfg, d, h, fw, dOut = _setup(shape, config)
    fs = layer.forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"], save_ab=True)
    torch.cuda.synchronize()
    assert fs["AB"] is not None and fs["AB"].shape == (cfg.T * cfg.k, 2 * cfg.d_ff)
    for key in ("Y", "out"):
        np.testing.assert_array_equal(fs[key].view(torch.int16).cpu().numpy(),
                                      fw[key].view(torch.int16).cpu().numpy(), err_msg=key)
    off = fw["offsets"].cpu().numpy()
    Xp = h["X"][fw["row_map"].cpu().numpy()]
    f = cfg.d_ff
    AB64 = np.zeros((cfg.T * cfg.k, 2 * f))
    for e in range(cfg.E):
        a, b = int(off[e]), int(off[e + 1])
        AB64[a:b] = Xp[a:b] @ h["W13"][e].T
    assert_close(fs["AB"].float().cpu().numpy(), AB64, 4e-3, "AB", max_tol=8e-3)
    dY, dw = layer.combine_bwd(cfg, dOut, fw["Y"], fw["inv_map"], fw["w"])
    for dt in (torch.float32, torch.bfloat16):
        ref = layer.expert_ffn_bwd(cfg, d["X"], fw["row_map"], fw["offsets"], dY, d["W13"],
                                   d["W2"], grad_dtype=dt)
        got = layer.expert_ffn_bwd(cfg, d["X"], fw["row_map"], fw["offsets"], dY, d["W13"],
                                   d["W2"], grad_dtype=dt, AB=fs["AB"])
        torch.cuda.synchronize()
        for name, a, b in zip(("dX_perm", "dW13", "dW2"), ref, got):
            assert torch.equal(a, b), (name, dt)


def test_autograd_with_and_without_saved_preactivations_agree():
    cfg, d, h, fw, dOut = _setup(BWD2, 39)
    grads = []
    for save in (False, True):
        leaves = [d[k].clone().requires_grad_(True) for k in ("X", "Wr", "br", "W13", "W2")]
        out = layer.moe_layer(cfg, *leaves, save_ab=save)
        out.backward(dOut)
        torch.cuda.synchronize()
        grads.append([t.grad for t in leaves])
    for name, a, b in zip(("X", "Wr", "br", "W13", "W2"), *grads):
        assert torch.equal(a, b), name


def test_dispatch_backward_is_a_gather_sum():
    cfg, d, h, fw, dOut = _setup(BWD, 33)
    dY, dw = layer.combine_bwd(cfg, dOut, fw["Y"], fw["inv_map"], fw["w"])
    dXp, _, _ = layer.expert_ffn_bwd(cfg, d["X"], fw["row_map"], fw["offsets"], dY, d["W13"], d["W2"])
    dX = layer.dispatch_bwd(cfg, dXp, fw["inv_map"])
    torch.cuda.synchronize()
    inv = fw["inv_map"].cpu().numpy()
    g = dXp.float().cpu().double().numpy()
    exp = sum(g[inv[:, j]] for j in range(cfg.k))
    assert_close(dX.cpu().numpy(), exp, 1e-6, "dX")


@pytest.mark.parametrize("act", ["f32", "bf16"])
@pytest.mark.parametrize("k", [3, 8])
def test_dispatch_backward_sums_in_slot_order_exactly(act, k):
    """moe_dispatch_bwd: dX[t] = sum over j in order of dX_perm[inv_map[t, j]],
    FP32 additions, bit for bit against the same additions on the host (FP32
    and BF16 slot gradients; d = 136 is not a multiple of 64 lanes x 8; top-8
    runs the kernel with the slot count fixed at compile time)."""
    T, d, E = 333, 136, 9
    shape = synth.MoEShape("dbwd", T=T, d=d, E=E, k=k, f=128, zipf=1.1, act=act, w=act)
    cfg = cfg_for(shape)
    rng = np.random.Generator(np.random.PCG64(77))
    g = rng.standard_normal((T * k, d)).astype(np.float32)
    inv = rng.permutation(T * k).astype(np.int32).reshape(T, k)
    dt = torch.float32 if act == "f32" else torch.bfloat16
    dXp = torch.from_numpy(g).to(dt).cuda()
    dX = layer.dispatch_bwd(cfg, dXp, torch.from_numpy(inv).cuda())
    torch.cuda.synchronize()
    gv = dXp.float().cpu().numpy()
    ref = np.zeros((T, d), np.float32)
    for j in range(k):
        ref = (ref + gv[inv[:, j]]).astype(np.float32)
    np.testing.assert_array_equal(dX.cpu().numpy(), ref)


def test_autograd_function_matches_oracle():
    shape = BWD
    inp = synth.make_inputs(shape, 34)
    d, h = device_inputs(shape, inp)
    cfg = cfg_for(shape)
    X = d["X"].clone().requires_grad_(True)
    Wr = d["Wr"].clone().requires_grad_(True)
    br = d["br"].clone().requires_grad_(True)
    W13 = d["W13"].clone().requires_grad_(True)
    W2 = d["W2"].clone().requires_grad_(True)
    out = layer.moe_layer(cfg, X, Wr, br, W13, W2)
    dOut = torch.from_numpy(synth.make_upstream(shape.T, shape.d, 34)).to(torch.bfloat16).cuda()
    out.backward(dOut)
    torch.cuda.synchronize()
    r = layer.route(cfg, d["X"], d["Wr"], d["br"])
    sel = r["idx"].cpu().numpy()
    ref = grad.layer_backward(h["X"], h["Wr"], h["br"], h["W13"], h["W2"], sel,
                              dOut.float().cpu().double().numpy())
    for name, t, key in [("X", X, "dX"), ("Wr", Wr, "dWr"), ("br", br, "dbr"), ("W13", W13, "dW13"),
                         ("W2", W2, "dW2")]:
        g, r_ = t.grad.float().cpu().numpy(), ref[key]
        if g.ndim == 3:
            g, r_ = g.reshape(-1, g.shape[-1]), r_.reshape(-1, r_.shape[-1])
        assert_close(g, r_, 2e-2, name)


def test_backward_is_deterministic():
    cfg, d, h, fw, dOut = _setup(BWD2, 35)
    res = []
    for _ in range(2):
        dY, dw = layer.combine_bwd(cfg, dOut, fw["Y"], fw["inv_map"], fw["w"])
        dXp, dW13, dW2 = layer.expert_ffn_bwd(cfg, d["X"], fw["row_map"], fw["offsets"], dY,
                                              d["W13"], d["W2"])
        dX, dWr, dbr = layer.route_bwd(cfg, d["X"], d["Wr"], fw["idx"], fw["w"], dw, fw["row_map"],
                                       fw["offsets"], fw["inv_map"], dXp)
        res.append([x.clone() for x in (dY, dw, dXp, dW13, dW2, dX, dWr, dbr)])
    torch.cuda.synchronize()
    for a, b in zip(*res):
        assert torch.equal(a, b)


def test_backward_fwd_bwd_config_sampled():
    """Workload 4 (T=32768, d=2048, E=128, top-8, f=1024): weight gradients of
    two experts and dX of 24 tokens against FP64 computed from those slots."""
    shape = synth.SHAPES[4]
    inp = synth.make_inputs(shape, 4)
    d, h = device_inputs(shape, inp, host_weights=False)
    del inp
    cfg = cfg_for(shape)
    fw = layer.forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"])
    torch.cuda.synchronize()
    # routing of the full batch (32768 tokens: each selection block streams
    # its margin column) bit-exact against the FP32 replica
    assert_route_matches(cfg, fw, replica_route(cfg, fw["logits"].cpu().numpy()))
    dOut = torch.from_numpy(synth.make_upstream(shape.T, shape.d, 4)).to(torch.bfloat16).cuda()
    dY, dw = layer.combine_bwd(cfg, dOut, fw["Y"], fw["inv_map"], fw["w"])
    dXp, dW13, dW2 = layer.expert_ffn_bwd(cfg, d["X"], fw["row_map"], fw["offsets"], dY, d["W13"],
                                          d["W2"])
    torch.cuda.synchronize()
    off = fw["offsets"].cpu().numpy()
    row_map = fw["row_map"].cpu().numpy()
    Xh = h["X"]
    dYh = dY.float().cpu().double().numpy()
    import scipy.special
    for e in (0, int(np.argmax(np.diff(off)))):
        a, b = int(off[e]), int(off[e + 1])
        x = Xh[row_map[a:b]]
        W13e = d["W13"][e].float().cpu().double().numpy()
        W2e = d["W2"][e].float().cpu().double().numpy()
        f = shape.f
        A = x @ W13e[:f].T
        B = x @ W13e[f:].T
        g = scipy.special.expit(A)
        hh = A * g * B
        U = dYh[a:b] @ W2e
        dA = U * B * (g + A * g * (1 - g))
        dB = U * A * g
        assert_close(dW2[e].cpu().numpy(), dYh[a:b].T @ hh, 2e-2, "dW2")
        assert_close(dW13[e, :f].cpu().numpy(), dA.T @ x, 2e-2, "dW1")
        assert_close(dW13[e, f:].cpu().numpy(), dB.T @ x, 2e-2, "dW3")
        dxp = dA @ W13e[:f] + dB @ W13e[f:]
        assert_close(dXp[a:b].float().cpu().numpy(), dxp, 2e-2, "dXp")
