"""Pins of the FFN, backward, FP8 and MLP oracles against library routines,
closed forms, special cases and finite differences."""
import math

import numpy as np
import scipy.special
import pytest
import torch
import torch.nn.functional as Fnn

from oracle import ffn, fp8, grad, mlp, routing as R
from paper_2606_17065_amd import synth

F32 = np.float32


def _small_layer(T=24, d=16, E=4, k=2, f=8, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((T, d))
    Wr = 0.3 * rng.standard_normal((E, d))
    br = synth.zipf_bias(rng, E, 1.0).astype(np.float64)
    W13 = 0.3 * rng.standard_normal((E, 2 * f, d))
    W2 = 0.3 * rng.standard_normal((E, d, f))
    return X, Wr, br, W13, W2


def test_single_expert_is_a_dense_swiglu():
    X, _, _, W13, W2 = _small_layer(E=1, k=1)
    T = X.shape[0]
    sel = np.zeros((T, 1), np.int32)
    w = np.ones((T, 1))
    out = ffn.layer_forward(X, sel, w, W13, W2)["out"]
    x = torch.tensor(X)
    f = W13.shape[1] // 2
    ref = Fnn.linear(Fnn.silu(Fnn.linear(x, torch.tensor(W13[0, :f]))) * Fnn.linear(x, torch.tensor(W13[0, f:])),
                     torch.tensor(W2[0]))
    np.testing.assert_allclose(out, ref.numpy(), rtol=1e-12, atol=1e-14)


def test_identical_experts_combine_to_one_ffn():
    X, Wr, br, W13, W2 = _small_layer()
    W13[:] = W13[0]
    W2[:] = W2[0]
    s = R.logits_fp64(X, Wr, br).astype(F32)
    r = R.route(s, 2, X.shape[0])
    out = ffn.layer_forward(X, r["sel"], r["w"], W13, W2)["out"]
    _, _, _, y = ffn.expert_forward(X, W13[0], W2[0])
    np.testing.assert_allclose(out, y, rtol=1e-12, atol=1e-14)


def test_silu_closed_forms():
    # silu(ln 3) = ln 3 * 3/4 ; silu(0) = 0 ; silu(-ln 3) = -ln 3 / 4
    z = np.array([math.log(3.0), 0.0, -math.log(3.0)])
    np.testing.assert_allclose(ffn.silu(z), [math.log(3) * 0.75, 0.0, -math.log(3) * 0.25], rtol=1e-15)


def test_dispatch_maps_are_a_stable_sort():
    s = synth.tiny_logits(37, 5, 1)
    r = R.route(s, 2, 37)
    off, row_map, inv = ffn.dispatch_maps(r["sel"], 5)
    T, k = r["sel"].shape
    assert off[0] == 0 and off[-1] == T * k
    np.testing.assert_array_equal(np.diff(off), np.bincount(r["sel"].ravel(), minlength=5))
    for e in range(5):
        rows = row_map[off[e]:off[e + 1]]
        assert np.all(np.diff(rows) > 0)  # token ascending within an expert
        assert np.all((r["sel"][rows] == e).any(axis=1))
    for t in range(T):
        for j in range(k):
            slot = inv[t, j]
            assert row_map[slot] == t
            assert off[r["sel"][t, j]] <= slot < off[r["sel"][t, j] + 1]


def test_combine_with_one_hot_weights_picks_one_expert():
    X, Wr, br, W13, W2 = _small_layer()
    T = X.shape[0]
    s = R.logits_fp64(X, Wr, br).astype(F32)
    r = R.route(s, 2, T)
    w = np.zeros((T, 2))
    w[:, 1] = 1.0
    out = ffn.layer_forward(X, r["sel"], w, W13, W2)["out"]
    for t in range(0, T, 5):
        e = r["sel"][t, 1]
        _, _, _, y = ffn.expert_forward(X[t:t + 1], W13[e], W2[e])
        np.testing.assert_allclose(out[t], y[0], rtol=1e-13, atol=1e-15)


def test_backward_matches_central_differences():
    X, Wr, br, W13, W2 = _small_layer(T=12, d=6, E=4, k=2, f=5, seed=3)
    rng = np.random.default_rng(7)
    dOut = rng.standard_normal((12, 6))
    s = R.logits_fp64(X, Wr, br).astype(F32)
    sel = R.route(s, 2, 12)["sel"]
    g = grad.layer_backward(X, Wr, br, W13, W2, sel, dOut)
    params = dict(X=X, Wr=Wr, br=br, W13=W13, W2=W2)
    names = dict(X="dX", Wr="dWr", br="dbr", W13="dW13", W2="dW2")
    for name, arr in params.items():
        flat = arr.reshape(-1)
        idxs = rng.choice(flat.shape[0], size=min(12, flat.shape[0]), replace=False)
        for i in idxs:
            h = 1e-6 * max(1.0, abs(flat[i]))
            old = flat[i]
            flat[i] = old + h
            lp = grad.layer_loss(X, Wr, br, W13, W2, sel, dOut)
            flat[i] = old - h
            lm = grad.layer_loss(X, Wr, br, W13, W2, sel, dOut)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[names[name]].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, i, fd, an)


def test_gate_backward_is_the_softmax_jacobian():
    rng = np.random.default_rng(2)
    z = rng.standard_normal(5)
    w = np.exp(z - z.max()) / np.exp(z - z.max()).sum()
    dw = rng.standard_normal(5)
    zt = torch.tensor(z, requires_grad=True)
    torch.softmax(zt, 0).backward(torch.tensor(dw))
    np.testing.assert_allclose(w * (dw - np.sum(w * dw)), zt.grad.numpy(), rtol=1e-13)


# ---------------------------------------------------------------- FP8 e4m3

def test_fp8_decode_matches_torch_for_all_codes():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    ours = fp8.decode(codes)
    np.testing.assert_array_equal(np.isnan(ours), np.isnan(ref))
    m = ~np.isnan(ref)
    np.testing.assert_array_equal(ours[m], ref[m])


def test_fp8_format_constants():
    assert fp8.decode(np.array([0x7E]))[0] == 448.0
    assert fp8.decode(np.array([0x08]))[0] == 2.0 ** -6
    assert fp8.decode(np.array([0x01]))[0] == 2.0 ** -9
    assert np.isnan(fp8.decode(np.array([0x7F, 0xFF]))).all()
    assert np.sum(~np.isnan(fp8.decode(np.arange(256, dtype=np.uint8)))) == 254


def test_fp8_encode_roundtrip_midpoints_and_saturation():
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    np.testing.assert_array_equal(fp8.encode(fp8.decode(codes)), codes)
    pos = np.sort(fp8.decode(np.arange(127, dtype=np.uint8)))
    mids = 0.5 * (pos[:-1] + pos[1:])
    got = fp8.encode(mids)
    lo = np.arange(126)
    # ties go to the code with the even mantissa (code parity = mantissa parity)
    expect = np.where(lo % 2 == 0, lo, lo + 1)
    np.testing.assert_array_equal(got, expect)
    assert fp8.round_rne_sat(np.array([1e6, -1e6, 464.0, 449.0]))[0] == 448.0
    np.testing.assert_array_equal(fp8.round_rne_sat(np.array([-1e6, 464.0, 449.0])), [-448.0, 448.0, 448.0])


def test_fp8_rounding_matches_torch_cast_in_range():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 30, rng.standard_normal(5000) * 1e-2]).astype(F32)
    x = np.clip(x, -448, 448)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(fp8.round_rne_sat(x), ref)


def test_fp8_block_quantisation_bounds():
    rng = np.random.default_rng(1)
    x = (rng.standard_normal((130, 256)) * np.exp(rng.standard_normal((130, 1)))).astype(F32)
    x[5, :128] = 0.0
    q, sc = fp8.quantize_blocks(x, 1, 128)
    deq = fp8.dequantize_blocks(q, sc, 1, 128)
    assert np.all(q[5, :128] == 0) and sc[5, 0] == 1.0
    # relative error of e4m3 RNE is at most 2^-4 of the value for normals
    big = np.abs(x) >= (2.0 ** -6) * np.repeat(sc, 128, axis=1)
    err = np.abs(deq - x)
    assert np.all(err[big] <= 2.0 ** -4 * np.abs(x[big]) * 1.0001)
    # the block maximum maps to +-448 codes
    amax_pos = np.abs(x[:, :128]).argmax(axis=1)
    assert np.all(np.abs(fp8.decode(q[np.arange(130), amax_pos])[np.arange(130) != 5]) == 448.0)


def test_round_bf16_is_nearest_even_and_matches_torch_on_float32_inputs():
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(50000) * np.exp(rng.uniform(-30, 30, 50000))).astype(F32)
    ref = torch.from_numpy(x).to(torch.bfloat16).double().numpy()
    np.testing.assert_array_equal(fp8.round_bf16(x.astype(np.float64)), ref)
    # ties between 1 and 1 + 2^-7 go to the even significand
    t = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 0.0])
    np.testing.assert_array_equal(fp8.round_bf16(t), [1.0, 1 + 2 * 2.0 ** -7, -1.0, 0.0])


def _fp8_layer_case(T=96, d=256, E=4, k=2, f=256, seed=3, grid=False):
    rng = np.random.default_rng(seed)
    if grid:
        # every value on the e4m3 grid and every block holding a 448, so all
        # scales are 1 and quantisation is exact
        vals = fp8.decode(np.arange(0x20, 0x48, dtype=np.uint8))  # 2^-4 .. 3.75
        X = rng.choice(vals, (T, d)) * rng.choice([-1.0, 1.0], (T, d))
        X[:, ::128] = 448.0
        W13 = rng.choice(vals, (E, 2 * f, d)) * rng.choice([-1.0, 1.0], (E, 2 * f, d))
        W13[:, ::128, ::128] = 448.0
        W2 = rng.choice(vals, (E, d, f))
        W2[:, ::128, ::128] = 448.0
    else:
        X = rng.standard_normal((T, d))
        W13 = 0.05 * rng.standard_normal((E, 2 * f, d))
        W2 = 0.05 * rng.standard_normal((E, d, f))
    X, W13, W2 = (a.astype(F32) for a in (X, W13, W2))
    sel = np.stack([rng.permutation(E)[:k] for _ in range(T)])
    offsets, row_map, inv_map = ffn.dispatch_maps(sel, E)
    W13q, W13s = fp8.quantize_experts(W13)
    W2q, W2s = fp8.quantize_experts(W2)
    return X, W13, W2, offsets, row_map, W13q, W13s, W2q, W2s


def test_fp8_layer_is_exact_on_the_grid():
    X, W13, W2, offsets, row_map, W13q, W13s, W2q, W2s = _fp8_layer_case(grid=True)
    assert np.all(W13s == 1.0) and np.all(W2s == 1.0)
    r = fp8.slots_forward_fp8(X, row_map, offsets, W13q, W13s, W2q, W2s)
    assert np.all(r["Xs"] == 1.0)
    Xp = X.astype(np.float64)[row_map]
    f = W13.shape[1] // 2
    for e in range(W13.shape[0]):
        a, b = offsets[e], offsets[e + 1]
        A = Xp[a:b] @ W13[e, :f].astype(np.float64).T
        B = Xp[a:b] @ W13[e, f:].astype(np.float64).T
        h = fp8.round_bf16(A * scipy.special.expit(A) * B)
        np.testing.assert_array_equal(r["h"][a:b], h)


def test_fp8_layer_power_of_two_weight_scaling_is_exact():
    X, W13, W2, offsets, row_map, W13q, W13s, W2q, W2s = _fp8_layer_case(seed=4)
    r1 = fp8.slots_forward_fp8(X, row_map, offsets, W13q, W13s, W2q, W2s)
    W2q8, W2s8 = fp8.quantize_experts(W2 * np.float32(8.0))
    np.testing.assert_array_equal(W2q8, W2q)
    np.testing.assert_array_equal(W2s8, W2s * 8)
    r8 = fp8.slots_forward_fp8(X, row_map, offsets, W13q, W13s, W2q8, W2s8)
    np.testing.assert_array_equal(r8["Y"], 8.0 * r1["Y"])


def test_fp8_layer_close_to_the_fp64_layer():
    X, W13, W2, offsets, row_map, W13q, W13s, W2q, W2s = _fp8_layer_case(seed=5)
    r = fp8.slots_forward_fp8(X, row_map, offsets, W13q, W13s, W2q, W2s)
    _, _, Y64 = ffn.slots_forward(X, row_map, offsets, W13, W2)
    rel = np.linalg.norm(r["Y"] - Y64) / np.linalg.norm(Y64)
    assert 1e-4 < rel <= 8e-2, rel


# ---------------------------------------------------------------- price MLP

def test_gelu_matches_torch_exact_gelu():
    z = np.linspace(-6, 6, 1001)
    np.testing.assert_allclose(mlp.gelu(z), Fnn.gelu(torch.tensor(z)).numpy(), rtol=1e-13, atol=1e-15)


def test_mlp_gradient_matches_torch_autograd():
    theta = mlp.init_params(1).astype(np.float64)
    rng = np.random.default_rng(4)
    F = rng.standard_normal((33, 8))
    y = np.abs(rng.standard_normal(33))
    loss, g = mlp.loss_and_grad(theta, F, y)
    th = torch.tensor(theta, requires_grad=True)
    P, o = {}, 0
    for name, shp in mlp.SIZES:
        n = int(np.prod(shp))
        P[name] = th[o:o + n].reshape(shp)
        o += n
    Ft = torch.tensor(F)
    a1 = Fnn.gelu(Ft @ P["W1"].T + P["b1"])
    a2 = Fnn.gelu(a1 @ P["W2"].T + P["b2"])
    z = a2 @ P["w3"] + P["b3"][0]
    lt = torch.mean((Fnn.softplus(z) - torch.tensor(y)) ** 2)
    lt.backward()
    assert abs(loss - lt.item()) < 1e-12
    np.testing.assert_allclose(g, th.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_mlp_gradient_matches_central_differences():
    theta = mlp.init_params(2).astype(np.float64)
    rng = np.random.default_rng(5)
    F = rng.standard_normal((9, 8))
    y = np.abs(rng.standard_normal(9))
    _, g = mlp.loss_and_grad(theta, F, y)
    for i in rng.choice(theta.shape[0], 25, replace=False):
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, F, y)[0] - mlp.loss_and_grad(tm, F, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))


def test_adam_matches_torch_adam():
    rng = np.random.default_rng(6)
    theta = rng.standard_normal(50)
    tt = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([tt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for step in range(1, 6):
        gr = rng.standard_normal(50)
        theta, m, v = mlp.adam_step(theta, gr, m, v, step, 1e-2)
        opt.zero_grad()
        tt.grad = torch.tensor(gr)
        opt.step()
    np.testing.assert_allclose(theta, tt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_feature_seven_is_the_first_clearing_price():
    s = synth.make_logits(500, 8, 1.2, seed=13)
    k, C = 2, synth.capacity(500, 2, 8)
    Fm = mlp.features(s, k, C)
    sig = float(np.std(s.astype(np.float64)))
    r1 = R.acp_prices(s, k, C, max_iters=1)
    over = R.acp_prices(s, k, C, max_iters=0)["load"] > C
    # first update: p = nextafter(q) + eps, eps = 1e-3 sigma
    p1 = r1["p"].astype(np.float64)
    np.testing.assert_allclose(Fm[over, 6] * sig, p1[over] - float(r1["eps"]), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(Fm[:, 4] * C, R.acp_prices(s, k, C, max_iters=0)["load"])


def test_feature_loads_follow_the_ranking_rule_on_ties():
    """On logits with exact ties and signed zeros, the zero-price loads behind
    f4 are those of a brute-force ranking by (total-order key desc, expert
    asc), and those of the routing oracle's first ranking."""
    rng = np.random.default_rng(17)
    T, E, k = 40, 6, 2
    s = (np.round(rng.standard_normal((T, E)) * 2.0) / 2.0).astype(np.float32)
    s[0, :2] = [-0.0, 0.0]
    s[1, :3] = [0.0, -0.0, 0.0]
    C = synth.capacity(T, k, E)
    Fm = mlp.features(s, k, C)
    key = R.f32_key(s)
    load = np.zeros(E, np.int64)
    for t in range(T):
        for _, e in sorted((-int(key[t, e]), e) for e in range(E))[:k]:
            load[e] += 1
    np.testing.assert_array_equal(np.rint(Fm[:, 4] * C).astype(np.int64), load)
    np.testing.assert_array_equal(load, R.acp_prices(s, k, C, max_iters=0)["load"])


@pytest.mark.slow
def test_backward_matches_central_differences_on_a_c4_slice():
    """The oracle's gradient against central differences on a 64-token slice
    of the forward+backward workload (d=2048, E=128, top-8, d_ff=1024,
    Zipf 1.3, upstream N(0,1)): the slice is routed by the workload's router
    (capacity for 64 tokens), and only the experts it uses take part, so the
    router rows, biases and expert weights are restricted to those experts
    (an unused expert's logit never enters the softmax over the chosen
    ones).  Expert weights N(0, 0.02^2) from a seeded generator; h = 1e-6
    max(1, |theta|); agreement <= 1e-6 relative."""
    from paper_2606_17065_amd import synth
    shape = synth.SHAPES[4]
    inp = synth.make_inputs(shape, 4, experts=False)
    T, k, E = 64, shape.k, shape.E
    X = inp["X"][:T].astype(np.float64)
    Wr = inp["Wr"].astype(np.float64)
    br = inp["br"].astype(np.float64)
    s = R.logits_fp64(X, Wr, br).astype(F32)
    r = R.route(s, k, synth.capacity(T, k, E), 50)
    assert r["status"] == R.OK
    used = np.unique(r["sel"])
    remap = np.full(E, -1)
    remap[used] = np.arange(used.shape[0])
    sel = remap[r["sel"]].astype(np.int32)
    rng = np.random.default_rng(4064)
    U, d, f = used.shape[0], shape.d, shape.f
    W13 = 0.02 * rng.standard_normal((U, 2 * f, d))
    W2 = 0.02 * rng.standard_normal((U, d, f))
    Wr_u, br_u = Wr[used].copy(), br[used].copy()
    dOut = synth.make_upstream(T, d, 4).astype(np.float64)
    g = grad.layer_backward(X, Wr_u, br_u, W13, W2, sel, dOut)
    params = dict(X=X, Wr=Wr_u, br=br_u, W13=W13, W2=W2)
    names = dict(X="dX", Wr="dWr", br="dbr", W13="dW13", W2="dW2")
    for name, arr in params.items():
        flat = arr.reshape(-1)
        # every compacted expert holds slots, so any coordinate is live
        for i in rng.choice(flat.shape[0], size=3, replace=False):
            h = 1e-6 * max(1.0, abs(flat[i]))
            old = flat[i]
            flat[i] = old + h
            lp = grad.layer_loss(X, Wr_u, br_u, W13, W2, sel, dOut)
            flat[i] = old - h
            lm = grad.layer_loss(X, Wr_u, br_u, W13, W2, sel, dOut)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[names[name]].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, i, fd, an)
