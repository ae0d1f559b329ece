"""Shared helpers of the GPU parity tests (inputs, conversions, comparisons)."""
from __future__ import annotations

import numpy as np
import torch

from oracle import routing as R
from paper_2606_17065_amd import _lib as L
from paper_2606_17065_amd import synth

F32 = np.float32

MODE_NAME = {L.MOE_PRICE_NONE: "none", L.MOE_PRICE_ACP: "acp", L.MOE_PRICE_GIVEN: "given",
             L.MOE_PRICE_WARM: "acp", L.MOE_PRICE_SUBGRAD: "subgrad"}


def cfg_for(shape: synth.MoEShape, price_mode=L.MOE_PRICE_ACP, max_iters=None, capacity=None,
            warm_gamma=0.9):
    act = L.MOE_F32 if shape.act == "f32" else L.MOE_BF16
    w = {"f32": L.MOE_F32, "bf16": L.MOE_BF16, "fp8": L.MOE_FP8E4M3}[shape.w]
    return L.make_cfg(shape.T, shape.d, shape.E, shape.k, shape.f,
                      shape.capacity if capacity is None else capacity,
                      shape.max_iters if max_iters is None else max_iters, act, w, price_mode,
                      warm_gamma)


def device_inputs(shape, inp, dev="cuda", host_weights=True):
    """Device tensors in the storage types of the shape, plus the FP64 host
    copies of exactly those stored values (what the oracle must see)."""
    act = torch.float32 if shape.act == "f32" else torch.bfloat16
    wdt = torch.float32 if shape.w == "f32" else torch.bfloat16
    d = {}
    h = {}
    d["X"] = torch.from_numpy(inp["X"]).to(act).to(dev).contiguous()
    h["X"] = d["X"].float().cpu().double().numpy()
    d["Wr"] = torch.from_numpy(inp["Wr"]).to(dev)
    h["Wr"] = inp["Wr"].astype(np.float64)
    d["br"] = torch.from_numpy(inp["br"]).to(dev)
    h["br"] = inp["br"].astype(np.float64)
    if "W13" in inp:
        d["W13"] = torch.from_numpy(inp["W13"]).to(wdt).to(dev).contiguous()
        d["W2"] = torch.from_numpy(inp["W2"]).to(wdt).to(dev).contiguous()
        if host_weights:
            h["W13"] = d["W13"].float().cpu().double().numpy()
            h["W2"] = d["W2"].float().cpu().double().numpy()
    return d, h


def rel_fro(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def max_abs_rel(a, b) -> float:
    """max |a - b| / max |b| (0 for empty arrays)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if b.size == 0:
        return 0.0
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def row_rel_max(a, b) -> float:
    """Worst row of a 2-D result: ||a_r - b_r|| / max(||b_r||, 1e-3 max_r ||b_r||).
    A single wrong, stale or zeroed row shows up here at its own size even
    when the norm of the whole matrix hides it."""
    a = np.asarray(a, np.float64).reshape(np.shape(a)[0], -1)
    b = np.asarray(b, np.float64).reshape(np.shape(b)[0], -1)
    if b.size == 0:
        return 0.0
    nb = np.linalg.norm(b, axis=1)
    floor = 1e-3 * nb.max() if nb.max() > 0 else 1.0
    return float((np.linalg.norm(a - b, axis=1) / np.maximum(nb, floor)).max())


def assert_close(got, ref, tol, what="", row_tol=None, max_tol=None):
    """Relative Frobenius error <= tol, max |diff| / max |ref| <= max_tol
    (tol unless given) and, for matrices of at least 64 columns, every row's
    relative error <= row_tol (2 * tol unless given)."""
    fro, mx = rel_fro(got, ref), max_abs_rel(got, ref)
    row = 0.0
    if np.ndim(ref) == 2 and np.shape(ref)[1] >= 64:
        row = row_rel_max(got, ref)
    row_tol = 2.0 * tol if row_tol is None else row_tol
    max_tol = tol if max_tol is None else max_tol
    assert fro <= tol and mx <= max_tol and row <= row_tol, (what, fro, mx, row)
    return fro, mx, row


def replica_route(cfg, logits32, price_in=None):
    """The FP32-replica routing the GPU must reproduce bit for bit."""
    mode = cfg.price_mode
    p0 = None
    if mode == L.MOE_PRICE_GIVEN:
        p0 = np.asarray(price_in, F32)
    elif mode == L.MOE_PRICE_WARM:
        p0 = (F32(cfg.warm_gamma) * np.asarray(price_in, F32)).astype(F32)
    iters = cfg.max_iters if mode in (L.MOE_PRICE_ACP, L.MOE_PRICE_WARM,
                                      L.MOE_PRICE_SUBGRAD) else 0
    stages = cfg.price_stages if mode != L.MOE_PRICE_SUBGRAD else 0
    return R.route(logits32, cfg.k, cfg.capacity, iters, p0, MODE_NAME[mode], stages)


def assert_route_matches(cfg, r_gpu, ref):
    info = r_gpu["info"].cpu().numpy()
    assert int(info[L.INFO_STATUS]) == ref["status"], (info, ref["status"])
    if ref["status"] != R.OK:
        return
    np.testing.assert_array_equal(r_gpu["idx"].cpu().numpy(), ref["sel"])
    np.testing.assert_array_equal(r_gpu["load"].cpu().numpy(), ref["load"])
    p = r_gpu["price"].cpu().numpy().astype(F32)
    np.testing.assert_array_equal(p.view(np.uint32), np.asarray(ref["p"], F32).view(np.uint32))
    assert int(info[L.INFO_ITERS]) == ref["iters"]
    assert bool(info[L.INFO_CONVERGED]) == bool(ref["converged"])
    assert bool(info[L.INFO_REPAIRED]) == bool(ref["enforced"])
    assert np.int32(info[L.INFO_SIGMA]).view(F32) == ref["sigma"]
    assert np.int32(info[L.INFO_EPS]).view(F32) == ref["eps"]
    np.testing.assert_allclose(r_gpu["w"].cpu().numpy(), ref["w"], rtol=0, atol=2e-6)
