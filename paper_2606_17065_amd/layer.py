"""Torch-facing wrappers over the C ABI: allocate outputs, pass pointers and
the current stream, raise on a bad status.  Every step of the layer runs in
libmoe's HIP kernels; torch only supplies device memory and the stream.
"""
from __future__ import annotations

import torch

from . import _lib as L

_DT = {L.MOE_F32: torch.float32, L.MOE_BF16: torch.bfloat16, L.MOE_FP8E4M3: torch.uint8}


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _p(t):
    return None if t is None else t.data_ptr()


def _need(t, name, dtype, shape=None):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Workspace:
    """One device buffer of moe_workspace_bytes(cfg), grown on demand."""

    def __init__(self):
        self.buf = None

    def get(self, cfg, device) -> torch.Tensor:
        n = max(L.moe_workspace_bytes(cfg), 256)
        if self.buf is None or self.buf.numel() < n or self.buf.device != device:
            self.buf = torch.empty(n, dtype=torch.uint8, device=device)
        return self.buf


_WS = Workspace()


def _fresh_price(cfg, dev):
    """Price buffer when the caller gives none: the clearing-price and the
    no-price modes start from p = 0 inside the routing kernels, so the
    buffer needs no fill; given and warm-started prices read it (zeros)."""
    if cfg.price_mode in (L.MOE_PRICE_ACP, L.MOE_PRICE_NONE, L.MOE_PRICE_SUBGRAD):
        return torch.empty(cfg.E, dtype=torch.float32, device=dev)
    return torch.zeros(cfg.E, dtype=torch.float32, device=dev)


def route(cfg, X, Wr, br, price=None, ws=None):
    T, d, E, k = cfg.T, cfg.d, cfg.E, cfg.k
    _need(X, "X", _DT[cfg.act], (T, d))
    _need(Wr, "Wr", torch.float32, (E, d))
    _need(br, "br", torch.float32, (E,))
    dev = X.device
    if price is None:
        price = _fresh_price(cfg, dev)
    else:
        _need(price, "price", torch.float32, (E,))
    # info is written in full by the routing kernels
    out = dict(
        logits=torch.empty(T, E, dtype=torch.float32, device=dev), price=price,
        idx=torch.empty(T, k, dtype=torch.int32, device=dev),
        w=torch.empty(T, k, dtype=torch.float32, device=dev),
        load=torch.empty(E, dtype=torch.int32, device=dev),
        info=torch.empty(L.INFO_LEN, dtype=torch.int32, device=dev))
    ws = _WS.get(cfg, dev) if ws is None else ws
    L.moe_route(cfg, _p(X), _p(Wr), _p(br), _p(out["logits"]), _p(price), _p(out["idx"]),
                _p(out["w"]), _p(out["load"]), _p(out["info"]), _p(ws), ws.numel(), _stream())
    return out


def router_logits(cfg, X, Wr, br, ws=None):
    """logits [T,E] f32 = X W_r^T + b_r (the router of moe_route alone)."""
    T, d, E = cfg.T, cfg.d, cfg.E
    _need(X, "X", _DT[cfg.act], (T, d))
    _need(Wr, "Wr", torch.float32, (E, d))
    _need(br, "br", torch.float32, (E,))
    logits = torch.empty(T, E, dtype=torch.float32, device=X.device)
    ws = _WS.get(cfg, X.device) if ws is None else ws
    L.moe_router_logits(cfg, _p(X), _p(Wr), _p(br), _p(logits), _p(ws), ws.numel(), _stream())
    return logits


def dispatch(cfg, X, idx, ws=None, permute=True):
    """Slot maps and permuted tokens; with FP8 experts X_perm holds e4m3
    codes (uint8) and X_perm_scale the per-1x128-block scales.  With
    permute=False (not FP8) only the maps are produced (X_perm is None)."""
    T, d, E, k = cfg.T, cfg.d, cfg.E, cfg.k
    _need(X, "X", _DT[cfg.act], (T, d))
    _need(idx, "topk_idx", torch.int32, (T, k))
    dev = X.device
    fp8 = cfg.w == L.MOE_FP8E4M3
    out = dict(offsets=torch.empty(E + 1, dtype=torch.int32, device=dev),
               row_map=torch.empty(T * k, dtype=torch.int32, device=dev),
               inv_map=torch.empty(T, k, dtype=torch.int32, device=dev),
               X_perm=(torch.empty(T * k, d, dtype=torch.uint8 if fp8 else X.dtype, device=dev)
                       if permute else None),
               X_perm_scale=(torch.empty(T * k, d // 128, dtype=torch.float32, device=dev)
                             if fp8 else None))
    ws = _WS.get(cfg, dev) if ws is None else ws
    L.moe_dispatch(cfg, _p(X), _p(idx), _p(out["offsets"]), _p(out["row_map"]),
                   _p(out["inv_map"]), _p(out["X_perm"]), _p(out["X_perm_scale"]), _p(ws),
                   ws.numel(), _stream())
    return out


def expert_ffn(cfg, X_perm, offsets, W13, W2, W13_scale=None, W2_scale=None, ws=None,
               X_perm_scale=None):
    N, d, E, f = cfg.T * cfg.k, cfg.d, cfg.E, cfg.d_ff
    fp8 = cfg.w == L.MOE_FP8E4M3
    _need(X_perm, "X_perm", torch.uint8 if fp8 else _DT[cfg.act], (N, d))
    _need(offsets, "offsets", torch.int32, (E + 1,))
    _need(W13, "W13", _DT[cfg.w], (E, 2 * f, d))
    _need(W2, "W2", _DT[cfg.w], (E, d, f))
    if fp8:
        _need(X_perm_scale, "X_perm_scale", torch.float32, (N, d // 128))
        _need(W13_scale, "W13_scale", torch.float32, (E, 2 * f // 128, d // 128))
        _need(W2_scale, "W2_scale", torch.float32, (E, d // 128, f // 128))
    Y = torch.empty(N, d, dtype=_DT[cfg.act], device=X_perm.device)
    ws = _WS.get(cfg, X_perm.device) if ws is None else ws
    L.moe_expert_ffn(cfg, _p(X_perm), _p(X_perm_scale), _p(offsets), _p(W13), _p(W13_scale),
                     _p(W2), _p(W2_scale), _p(Y), _p(ws), ws.numel(), _stream())
    return Y


def quantize_fp8(x, block_rows):
    """(codes uint8, scales f32) of a [rows, cols] f32/bf16 matrix (or a
    stack of expert matrices, quantised as rows = E * R) in block_rows x 128
    blocks."""
    if x.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("quantize_fp8 takes float32 or bfloat16")
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("quantize_fp8 takes a contiguous device tensor")
    cols = x.shape[-1]
    rows = x.numel() // max(cols, 1)
    lead = tuple(x.shape[:-1])
    codes = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    if block_rows == 1:
        sshape = lead + (cols // 128,)
    else:
        R = x.shape[-2]
        if x.dim() > 2 and R % block_rows != 0:
            raise ValueError("expert matrices need a multiple of 128 rows")
        sshape = tuple(x.shape[:-2]) + ((R + block_rows - 1) // block_rows, cols // 128)
    scales = torch.empty(sshape, dtype=torch.float32, device=x.device)
    L.moe_quantize_fp8(rows, cols, block_rows, L.MOE_BF16 if x.dtype == torch.bfloat16 else L.MOE_F32,
                       _p(x), _p(codes), _p(scales), _stream())
    return codes, scales


MX_DTYPES = (L.MOE_MXFP8E4M3, L.MOE_MXFP6E2M3, L.MOE_MXFP4E2M1)


def mx_row_bytes(fmt, K):
    """Bytes of an MX code row of K elements (e2m1: two codes per byte;
    e4m3 and the padded e2m3 layout: one byte per element)."""
    return K // 2 if fmt == L.MOE_MXFP4E2M1 else K


def quantize_mx(x, fmt):
    """(codes uint8 [..., row bytes], scale bytes uint8 [..., K/32]) of a
    contiguous f32/bf16 device tensor, quantised along its last dimension
    in OCP MX blocks of 32."""
    if x.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("quantize_mx takes float32 or bfloat16")
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("quantize_mx takes a contiguous device tensor")
    if fmt not in MX_DTYPES:
        raise ValueError(f"not an MX format: {fmt}")
    K = x.shape[-1]
    rows = x.numel() // max(K, 1)
    codes = torch.empty(tuple(x.shape[:-1]) + (mx_row_bytes(fmt, K),), dtype=torch.uint8,
                        device=x.device)
    scales = torch.empty(tuple(x.shape[:-1]) + (K // 32,), dtype=torch.uint8, device=x.device)
    L.moe_quantize_mx(rows, K, fmt, L.MOE_BF16 if x.dtype == torch.bfloat16 else L.MOE_F32,
                      _p(x), _p(codes), _p(scales), _stream())
    return codes, scales


def expert_ffn_mx(cfg, X_codes, X_scale, row_map, offsets, W13, W13_scale, W2, W2_scale, ws=None):
    N, d, E, f = cfg.T * cfg.k, cfg.d, cfg.E, cfg.d_ff
    fmt = cfg.w
    _need(X_codes, "X_codes", torch.uint8, (cfg.T, mx_row_bytes(fmt, d)))
    _need(X_scale, "X_scale", torch.uint8, (cfg.T, d // 32))
    _need(row_map, "row_map", torch.int32, (N,))
    _need(offsets, "offsets", torch.int32, (E + 1,))
    _need(W13, "W13", torch.uint8, (E, 2 * f, mx_row_bytes(fmt, d)))
    _need(W13_scale, "W13_scale", torch.uint8, (E, 2 * f, d // 32))
    _need(W2, "W2", torch.uint8, (E, d, mx_row_bytes(fmt, f)))
    _need(W2_scale, "W2_scale", torch.uint8, (E, d, f // 32))
    Y = torch.empty(N, d, dtype=torch.bfloat16, device=X_codes.device)
    ws = _WS.get(cfg, X_codes.device) if ws is None else ws
    L.moe_expert_ffn_mx(cfg, _p(X_codes), _p(X_scale), _p(row_map), _p(offsets), _p(W13),
                        _p(W13_scale), _p(W2), _p(W2_scale), _p(Y), _p(ws), ws.numel(), _stream())
    return Y


def combine(cfg, Y, inv_map, w):
    T, d, k = cfg.T, cfg.d, cfg.k
    _need(Y, "Y", _DT[cfg.act], (T * k, d))
    _need(inv_map, "inv_map", torch.int32, (T, k))
    _need(w, "topk_w", torch.float32, (T, k))
    out = torch.empty(T, d, dtype=Y.dtype, device=Y.device)
    L.moe_combine(cfg, _p(Y), _p(inv_map), _p(w), _p(out), _stream())
    return out


def gather_fused(cfg) -> bool:
    """True when the first expert product can read X through row_map."""
    return (cfg.act == L.MOE_BF16 and cfg.w == L.MOE_BF16 and cfg.d_ff % 128 == 0
            and cfg.d % 256 == 0)


def expert_ffn_gather(cfg, X, row_map, offsets, W13, W2, ws=None, save_ab=False):
    """Y [N,d]; with save_ab, (Y, AB) where AB [N, 2f] holds the first
    product's pre-activations [A|B] for expert_ffn_bwd."""
    N, d, E, f = cfg.T * cfg.k, cfg.d, cfg.E, cfg.d_ff
    _need(X, "X", _DT[cfg.act], (cfg.T, d))
    _need(row_map, "row_map", torch.int32, (N,))
    _need(offsets, "offsets", torch.int32, (E + 1,))
    _need(W13, "W13", _DT[cfg.w], (E, 2 * f, d))
    _need(W2, "W2", _DT[cfg.w], (E, d, f))
    Y = torch.empty(N, d, dtype=X.dtype, device=X.device)
    ws = _WS.get(cfg, X.device) if ws is None else ws
    if not save_ab:
        L.moe_expert_ffn_gather(cfg, _p(X), _p(row_map), _p(offsets), _p(W13), _p(W2), _p(Y),
                                _p(ws), ws.numel(), _stream())
        return Y
    AB = torch.empty(N, 2 * f, dtype=X.dtype, device=X.device)
    L.moe_expert_ffn_gather_save(cfg, _p(X), _p(row_map), _p(offsets), _p(W13), _p(W2), _p(Y),
                                 _p(AB), _p(ws), ws.numel(), _stream())
    return Y, AB


def gather_fused_fp8(cfg) -> bool:
    """True when the FP8 expert products can read per-token codes through
    row_map."""
    return (cfg.act == L.MOE_BF16 and cfg.w == L.MOE_FP8E4M3 and cfg.d_ff % 128 == 0
            and cfg.d % 128 == 0)


def expert_ffn_gather_fp8(cfg, X_codes, X_scale, row_map, offsets, W13, W2, W13_scale, W2_scale,
                          ws=None):
    N, d, E, f = cfg.T * cfg.k, cfg.d, cfg.E, cfg.d_ff
    _need(X_codes, "X_codes", torch.uint8, (cfg.T, d))
    _need(X_scale, "X_scale", torch.float32, (cfg.T, d // 128))
    _need(row_map, "row_map", torch.int32, (N,))
    _need(offsets, "offsets", torch.int32, (E + 1,))
    _need(W13, "W13", torch.uint8, (E, 2 * f, d))
    _need(W2, "W2", torch.uint8, (E, d, f))
    _need(W13_scale, "W13_scale", torch.float32, (E, 2 * f // 128, d // 128))
    _need(W2_scale, "W2_scale", torch.float32, (E, d // 128, f // 128))
    Y = torch.empty(N, d, dtype=torch.bfloat16, device=X_codes.device)
    ws = _WS.get(cfg, X_codes.device) if ws is None else ws
    L.moe_expert_ffn_gather_fp8(cfg, _p(X_codes), _p(X_scale), _p(row_map), _p(offsets), _p(W13),
                                _p(W13_scale), _p(W2), _p(W2_scale), _p(Y), _p(ws), ws.numel(),
                                _stream())
    return Y


def check_status(info, where="moe_route"):
    """Raise MoEError if a routing's device status (info[MOE_INFO_STATUS]) is
    not MOE_OK.  Reads the value on the host, so it waits for the stream."""
    st = int(info[L.INFO_STATUS].item())
    if st != L.MOE_OK:
        raise L.MoEError(st, where)


def forward(cfg, X, Wr, br, W13, W2, price=None, W13_scale=None, W2_scale=None, fuse=True,
            check=True, save_ab=False):
    """The whole layer forward; returns every intermediate (X_perm is None
    when the permute is fused into the first expert product).  save_ab: on
    the gather-fused BF16 path, also keep the first product's
    pre-activations as r["AB"] (for the backward; None on other paths).

    check: after enqueueing every stage, wait for the stream and raise
    MoEError if the routing failed on the device (a non-finite logit, or a
    capacity repair that could not place every slot).  With check=False
    nothing waits; a failed routing then carries NaN gate weights, so the
    layer output is NaN rather than a plausible-looking value."""
    r = route(cfg, X, Wr, br, price)
    r["AB"] = None
    if fuse and gather_fused(cfg):
        dsp = dispatch(cfg, X, r["idx"], permute=False)
        if save_ab:
            Y, r["AB"] = expert_ffn_gather(cfg, X, dsp["row_map"], dsp["offsets"], W13, W2,
                                           save_ab=True)
        else:
            Y = expert_ffn_gather(cfg, X, dsp["row_map"], dsp["offsets"], W13, W2)
    elif cfg.w in MX_DTYPES:
        # tokens MX-quantised once, gathered by the first product
        Xq, Xs = quantize_mx(X, cfg.w)
        dsp = dispatch(cfg, X, r["idx"], permute=False)
        Y = expert_ffn_mx(cfg, Xq, Xs, dsp["row_map"], dsp["offsets"], W13, W13_scale, W2,
                          W2_scale)
        r["X_codes"], r["X_scale"] = Xq, Xs
    elif fuse and gather_fused_fp8(cfg):
        # tokens quantised once (1 x 128 blocks), gathered by the first product
        Xq, Xs = quantize_fp8(X, 1)
        dsp = dispatch(cfg, X, r["idx"], permute=False)
        Y = expert_ffn_gather_fp8(cfg, Xq, Xs, dsp["row_map"], dsp["offsets"], W13, W2,
                                  W13_scale, W2_scale)
        r["X_codes"], r["X_scale"] = Xq, Xs
    else:
        dsp = dispatch(cfg, X, r["idx"])
        Y = expert_ffn(cfg, dsp["X_perm"], dsp["offsets"], W13, W2, W13_scale, W2_scale,
                       X_perm_scale=dsp["X_perm_scale"])
    out = combine(cfg, Y, dsp["inv_map"], r["w"])
    r.update(dsp)
    r["Y"] = Y
    r["out"] = out
    if check:
        check_status(r["info"])
    return r


# ----------------------------------------------------------------- backward

def combine_bwd(cfg, dOut, Y, inv_map, w):
    T, d, k = cfg.T, cfg.d, cfg.k
    _need(dOut, "dOut", _DT[cfg.act], (T, d))
    _need(Y, "Y", _DT[cfg.act], (T * k, d))
    dY = torch.empty_like(Y)
    dw = torch.empty(T, k, dtype=torch.float32, device=Y.device)
    L.moe_combine_bwd(cfg, _p(dOut), _p(Y), _p(inv_map), _p(w), _p(dY), _p(dw), _stream())
    return dY, dw


_GRAD_DT = {torch.float32: L.MOE_F32, torch.bfloat16: L.MOE_BF16}


def expert_ffn_bwd(cfg, X, row_map, offsets, dY, W13, W2, ws=None, grad_dtype=torch.float32,
                   AB=None):
    """dX_perm [N,d] (act dtype) and the weight gradients dW13, dW2 stored in
    grad_dtype (float32 or bfloat16; FP32 accumulation either way).  AB: the
    pre-activations expert_ffn_gather(save_ab=True) stored, read instead of
    recomputed (same results)."""
    N, d, E, f = cfg.T * cfg.k, cfg.d, cfg.E, cfg.d_ff
    _need(X, "X", _DT[cfg.act], (cfg.T, d))
    _need(dY, "dY", _DT[cfg.act], (N, d))
    dev = X.device
    dXp = torch.empty(N, d, dtype=X.dtype, device=dev)
    dW13 = torch.empty(E, 2 * f, d, dtype=grad_dtype, device=dev)
    dW2 = torch.empty(E, d, f, dtype=grad_dtype, device=dev)
    ws = _WS.get(cfg, dev) if ws is None else ws
    if AB is None:
        L.moe_expert_ffn_bwd(cfg, _p(X), _p(row_map), _p(offsets), _p(dY), _p(W13), _p(W2),
                             _p(dXp), _p(dW13), _p(dW2), _GRAD_DT[grad_dtype], _p(ws), ws.numel(),
                             _stream())
    else:
        _need(AB, "AB", _DT[cfg.act], (N, 2 * f))
        L.moe_expert_ffn_bwd_saved(cfg, _p(X), _p(row_map), _p(offsets), _p(dY), _p(W13),
                                   _p(W2), _p(AB), _p(dXp), _p(dW13), _p(dW2),
                                   _GRAD_DT[grad_dtype], _p(ws), ws.numel(), _stream())
    return dXp, dW13, dW2


def dispatch_bwd(cfg, dXp, inv_map):
    dX = torch.empty(cfg.T, cfg.d, dtype=torch.float32, device=dXp.device)
    L.moe_dispatch_bwd(cfg, _p(dXp), _p(inv_map), _p(dX), _stream())
    return dX


def route_bwd(cfg, X, Wr, idx, w, dw, row_map, offsets, inv_map, dXp, ws=None,
              dx_dtype=torch.float32):
    dev = X.device
    dX = torch.empty(cfg.T, cfg.d, dtype=dx_dtype, device=dev)
    dWr = torch.empty(cfg.E, cfg.d, dtype=torch.float32, device=dev)
    dbr = torch.empty(cfg.E, dtype=torch.float32, device=dev)
    ws = _WS.get(cfg, dev) if ws is None else ws
    L.moe_route_bwd(cfg, _p(X), _p(Wr), _p(idx), _p(w), _p(dw), _p(row_map), _p(offsets),
                    _p(inv_map), _p(dXp), _p(dX), _GRAD_DT[dx_dtype], _p(dWr), _p(dbr), _p(ws),
                    ws.numel(), _stream())
    return dX, dWr, dbr


class MoEFunction(torch.autograd.Function):
    """The layer as one differentiable op.  Saves X, the routing (indices,
    gate weights, slot maps), Y and, with save_ab on the gather-fused BF16
    path, the first expert product's pre-activations [A|B] (N x 2 d_ff
    values, kept instead of recomputing that product in the backward; the
    gradients are the same either way).  The permuted tokens are recomputed
    through row_map.  Gradients flow to X, W_r, b_r, W13 and W2; none flows
    into the prices or through the expert selection."""

    @staticmethod
    def forward(ctx, X, Wr, br, W13, W2, cfg, check=True, save_ab=True):
        r = forward(cfg, X, Wr, br, W13, W2, check=check, save_ab=save_ab)
        ctx.cfg = cfg
        ctx.save_for_backward(X, Wr, W13, W2, r["idx"], r["w"], r["row_map"], r["offsets"],
                              r["inv_map"], r["Y"], r["AB"])
        return r["out"]

    @staticmethod
    def backward(ctx, dOut):
        X, Wr, W13, W2, idx, w, row_map, offsets, inv_map, Y, AB = ctx.saved_tensors
        cfg = ctx.cfg
        dOut = dOut.to(Y.dtype).contiguous()
        dY, dw = combine_bwd(cfg, dOut, Y, inv_map, w)
        # gradients stored directly in their parameters' dtypes (FP32 sums)
        dXp, dW13, dW2 = expert_ffn_bwd(cfg, X, row_map, offsets, dY, W13, W2,
                                        grad_dtype=W13.dtype, AB=AB)
        dX, dWr, dbr = route_bwd(cfg, X, Wr, idx, w, dw, row_map, offsets, inv_map, dXp,
                                 dx_dtype=X.dtype)
        return (dX, dWr, dbr, dW13, dW2, None, None, None)


def moe_layer(cfg, X, Wr, br, W13, W2, check=True, save_ab=True):
    """Differentiable layer forward (see MoEFunction; check as in forward)."""
    return MoEFunction.apply(X, Wr, br, W13, W2, cfg, check, save_ab)
