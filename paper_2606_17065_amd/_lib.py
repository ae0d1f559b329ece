"""ctypes binding of libmoe.so: the C ABI of include/moe.h, name for name.

Argument marshalling only.  Pointers are passed as Python ints (device
addresses, e.g. ``tensor.data_ptr()``), the stream as an int handle.  A
missing library raises at load time: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmoe.so")

MOE_OK = 0
MOE_EINVAL = -1
MOE_EINFEASIBLE = -2
MOE_EUNSUPPORTED = -3
MOE_EWORKSPACE = -4
MOE_EHIP = -5
MOE_ENAN = -6
MOE_ECAPACITY = -7

MOE_F32, MOE_BF16, MOE_FP8E4M3 = 0, 1, 2
MOE_MXFP8E4M3, MOE_MXFP6E2M3, MOE_MXFP4E2M1 = 3, 4, 5
MOE_PRICE_NONE, MOE_PRICE_ACP, MOE_PRICE_GIVEN, MOE_PRICE_WARM, MOE_PRICE_SUBGRAD = 0, 1, 2, 3, 4

INFO_ITERS, INFO_CONVERGED, INFO_OVERFLOW, INFO_STATUS = 0, 1, 2, 3
INFO_ROUNDS, INFO_SIGMA, INFO_EPS, INFO_REPAIRED = 4, 5, 6, 7
INFO_LEN = 8


class MoeCfg(ctypes.Structure):
    _fields_ = [
        ("T", ctypes.c_int32), ("d", ctypes.c_int32), ("E", ctypes.c_int32),
        ("k", ctypes.c_int32), ("d_ff", ctypes.c_int32), ("capacity", ctypes.c_int32),
        ("max_iters", ctypes.c_int32), ("act", ctypes.c_int32), ("w", ctypes.c_int32),
        ("price_mode", ctypes.c_int32), ("warm_gamma", ctypes.c_float),
        ("price_stages", ctypes.c_int32),
    ]


class MoEError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} (status {status})")


_P = ctypes.c_void_p
_S = ctypes.c_size_t
_CFG = ctypes.POINTER(MoeCfg)

# name -> argtypes (every function returns int32 status unless noted)
SIGNATURES = {
    "moe_workspace_bytes": [_CFG, ctypes.POINTER(ctypes.c_size_t)],
    "moe_route": [_CFG, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _S, _P],
    "moe_router_logits": [_CFG, _P, _P, _P, _P, _P, _S, _P],
    "moe_dispatch": [_CFG, _P, _P, _P, _P, _P, _P, _P, _P, _S, _P],
    "moe_dispatch_noalloc": [_CFG, _P, _P, _P, _P, _P, _P, _P, _P],
    "moe_expert_ffn": [_CFG, _P, _P, _P, _P, _P, _P, _P, _P, _P, _S, _P],
    "moe_expert_ffn_gather": [_CFG, _P, _P, _P, _P, _P, _P, _P, _S, _P],
    "moe_expert_ffn_gather_save": [_CFG, _P, _P, _P, _P, _P, _P, _P, _P, _S, _P],
    "moe_expert_ffn_gather_fp8": [_CFG, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _S, _P],
    "moe_quantize_mx": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P],
    "moe_expert_ffn_mx": [_CFG, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _S, _P],
    "moe_quantize_fp8": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P],
    "moe_combine": [_CFG, _P, _P, _P, _P, _P],
    "moe_combine_bwd": [_CFG, _P, _P, _P, _P, _P, _P, _P],
    "moe_expert_ffn_bwd": [_CFG, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_int, _P, _S, _P],
    "moe_expert_ffn_bwd_saved": [_CFG, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_int, _P,
                                 _S, _P],
    "moe_dispatch_bwd": [_CFG, _P, _P, _P, _P],
    "moe_route_bwd": [_CFG, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_int, _P, _P, _P, _S,
                      _P],
    "moe_route_logits": [_CFG, _P, _P, _P, _P, _P, _P, _P, _S, _P],
    "moe_price_update": [_CFG, _P, _P, _P, _P, _S, _P],
    "moe_route_certify": [_CFG, _P, _P, _P, _P, _P, _S, _P],
    "moe_route_judged": [_CFG, _P, _P, ctypes.c_float, _P, _P, _P, _P, _P, _P, _P, _S, _P],
    "moe_route_learned": [_CFG, _P, _P, ctypes.c_float, _P, _P, _P, _P, _P, _P, _P, _S, _P],
    "moe_logit_stats": [_CFG, _P, _P, _P, _P, _S, _P],
    "moe_price_mlp_sizes": [ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                            ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
    "moe_price_mlp_forward": [ctypes.c_int, _P, _P, _P, _P, _P, _P],
    "moe_price_mlp_backward": [ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _S, _P],
    "moe_price_mse": [ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P, _P],
    "moe_adam_step": [ctypes.c_int, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float,
                      ctypes.c_float, ctypes.c_float, ctypes.c_int, _P],
    "moe_prof_enable": [ctypes.c_int],
    "moe_prof_reset": [],
    "moe_prof_lds_copy": [_P, _P, _S, _P],
    "moe_prof_get": [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)],
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libmoe.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2606_17065_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        L.moe_strerror.argtypes = [ctypes.c_int]
        L.moe_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().moe_strerror(int(status)).decode()


def _check(status: int, where: str) -> None:
    if status != MOE_OK:
        raise MoEError(status, where)


def make_cfg(T, d, E, k, d_ff, capacity, max_iters=50, act=MOE_BF16, w=MOE_BF16,
             price_mode=MOE_PRICE_ACP, warm_gamma=0.9, price_stages=0) -> MoeCfg:
    return MoeCfg(T, d, E, k, d_ff, capacity, max_iters, act, w, price_mode, warm_gamma,
                  price_stages)


def moe_workspace_bytes(cfg: MoeCfg) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().moe_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)), "moe_workspace_bytes")
    return int(out.value)


def moe_route(cfg, X, Wr, br, logits, price, topk_idx, topk_w, load, info, ws, ws_bytes, stream):
    _check(lib().moe_route(ctypes.byref(cfg), X, Wr, br, logits, price, topk_idx, topk_w, load,
                           info, ws, ws_bytes, stream), "moe_route")


def moe_router_logits(cfg, X, Wr, br, logits, ws, ws_bytes, stream):
    _check(lib().moe_router_logits(ctypes.byref(cfg), X, Wr, br, logits, ws, ws_bytes, stream),
           "moe_router_logits")


def moe_dispatch(cfg, X, topk_idx, offsets, row_map, inv_map, X_perm, X_perm_scale, ws, ws_bytes,
                 stream):
    _check(lib().moe_dispatch(ctypes.byref(cfg), X, topk_idx, offsets, row_map, inv_map, X_perm,
                              X_perm_scale, ws, ws_bytes, stream), "moe_dispatch")


def moe_expert_ffn(cfg, X_perm, X_perm_scale, offsets, W13, W13_scale, W2, W2_scale, Y, ws,
                   ws_bytes, stream):
    _check(lib().moe_expert_ffn(ctypes.byref(cfg), X_perm, X_perm_scale, offsets, W13, W13_scale,
                                W2, W2_scale, Y, ws, ws_bytes, stream), "moe_expert_ffn")


def moe_expert_ffn_gather_fp8(cfg, X_codes, X_scale, row_map, offsets, W13, W13_scale, W2,
                              W2_scale, Y, ws, ws_bytes, stream):
    _check(lib().moe_expert_ffn_gather_fp8(ctypes.byref(cfg), X_codes, X_scale, row_map, offsets,
                                           W13, W13_scale, W2, W2_scale, Y, ws, ws_bytes, stream),
           "moe_expert_ffn_gather_fp8")


def moe_quantize_mx(rows, cols, fmt, src_dtype, src, codes, scales, stream):
    _check(lib().moe_quantize_mx(rows, cols, fmt, src_dtype, src, codes, scales, stream),
           "moe_quantize_mx")


def moe_expert_ffn_mx(cfg, X_codes, X_scale, row_map, offsets, W13, W13_scale, W2, W2_scale, Y,
                      ws, ws_bytes, stream):
    _check(lib().moe_expert_ffn_mx(ctypes.byref(cfg), X_codes, X_scale, row_map, offsets, W13,
                                   W13_scale, W2, W2_scale, Y, ws, ws_bytes, stream),
           "moe_expert_ffn_mx")


def moe_expert_ffn_gather(cfg, X, row_map, offsets, W13, W2, Y, ws, ws_bytes, stream):
    _check(lib().moe_expert_ffn_gather(ctypes.byref(cfg), X, row_map, offsets, W13, W2, Y, ws,
                                       ws_bytes, stream), "moe_expert_ffn_gather")


def moe_expert_ffn_gather_save(cfg, X, row_map, offsets, W13, W2, Y, AB, ws, ws_bytes, stream):
    _check(lib().moe_expert_ffn_gather_save(ctypes.byref(cfg), X, row_map, offsets, W13, W2, Y,
                                            AB, ws, ws_bytes, stream),
           "moe_expert_ffn_gather_save")


def moe_quantize_fp8(rows, cols, block_rows, src_dtype, src, codes, scales, stream):
    _check(lib().moe_quantize_fp8(int(rows), int(cols), int(block_rows), int(src_dtype), src, codes,
                                  scales, stream), "moe_quantize_fp8")


def moe_combine(cfg, Y, inv_map, topk_w, out, stream):
    _check(lib().moe_combine(ctypes.byref(cfg), Y, inv_map, topk_w, out, stream), "moe_combine")


def moe_combine_bwd(cfg, dOut, Y, inv_map, topk_w, dY, dtopk_w, stream):
    _check(lib().moe_combine_bwd(ctypes.byref(cfg), dOut, Y, inv_map, topk_w, dY, dtopk_w, stream),
           "moe_combine_bwd")


def moe_expert_ffn_bwd(cfg, X, row_map, offsets, dY, W13, W2, dX_perm, dW13, dW2, grad_dtype, ws,
                       ws_bytes, stream):
    _check(lib().moe_expert_ffn_bwd(ctypes.byref(cfg), X, row_map, offsets, dY, W13, W2, dX_perm,
                                    dW13, dW2, grad_dtype, ws, ws_bytes, stream),
           "moe_expert_ffn_bwd")


def moe_expert_ffn_bwd_saved(cfg, X, row_map, offsets, dY, W13, W2, AB, dX_perm, dW13, dW2,
                             grad_dtype, ws, ws_bytes, stream):
    _check(lib().moe_expert_ffn_bwd_saved(ctypes.byref(cfg), X, row_map, offsets, dY, W13, W2,
                                          AB, dX_perm, dW13, dW2, grad_dtype, ws, ws_bytes,
                                          stream),
           "moe_expert_ffn_bwd_saved")


def moe_dispatch_noalloc(cfg, X, topk_idx, offsets, row_map, inv_map, X_perm, X_perm_scale,
                         stream):
    _check(lib().moe_dispatch_noalloc(ctypes.byref(cfg), X, topk_idx, offsets, row_map, inv_map,
                                      X_perm, X_perm_scale, stream), "moe_dispatch_noalloc")


def moe_dispatch_bwd(cfg, dX_perm, inv_map, dX, stream):
    _check(lib().moe_dispatch_bwd(ctypes.byref(cfg), dX_perm, inv_map, dX, stream), "moe_dispatch_bwd")


def moe_route_bwd(cfg, X, Wr, topk_idx, topk_w, dtopk_w, row_map, offsets, inv_map, dX_perm, dX,
                  dx_dtype, dWr, dbr, ws, ws_bytes, stream):
    _check(lib().moe_route_bwd(ctypes.byref(cfg), X, Wr, topk_idx, topk_w, dtopk_w, row_map,
                               offsets, inv_map, dX_perm, dX, dx_dtype, dWr, dbr, ws, ws_bytes,
                               stream), "moe_route_bwd")


def moe_route_logits(cfg, logits, price, topk_idx, topk_w, load, info, ws, ws_bytes, stream):
    _check(lib().moe_route_logits(ctypes.byref(cfg), logits, price, topk_idx, topk_w, load, info,
                                  ws, ws_bytes, stream), "moe_route_logits")


def moe_price_update(cfg, logits, price, info, ws, ws_bytes, stream):
    _check(lib().moe_price_update(ctypes.byref(cfg), logits, price, info, ws, ws_bytes, stream),
           "moe_price_update")


def moe_route_certify(cfg, logits, price, topk_idx, cert, ws, ws_bytes, stream):
    _check(lib().moe_route_certify(ctypes.byref(cfg), logits, price, topk_idx, cert, ws, ws_bytes,
                                   stream), "moe_route_certify")


def moe_route_judged(cfg, logits, price_hat, gap_tol, price, topk_idx, topk_w, load, info,
                     verdict, ws, ws_bytes, stream):
    _check(lib().moe_route_judged(ctypes.byref(cfg), logits, price_hat, float(gap_tol), price,
                                  topk_idx, topk_w, load, info, verdict, ws, ws_bytes, stream),
           "moe_route_judged")


def moe_route_learned(cfg, logits, price_hat, gap_tol, price, topk_idx, topk_w, load, info,
                     verdict, ws, ws_bytes, stream):
    _check(lib().moe_route_learned(ctypes.byref(cfg), logits, price_hat, float(gap_tol), price,
                                  topk_idx, topk_w, load, info, verdict, ws, ws_bytes, stream),
           "moe_route_learned")


def moe_logit_stats(cfg, logits, feats, sigma, ws, ws_bytes, stream):
    _check(lib().moe_logit_stats(ctypes.byref(cfg), logits, feats, sigma, ws, ws_bytes, stream),
           "moe_logit_stats")


def moe_price_mlp_sizes(rows: int):
    """(n_params, acts_floats, bwd_ws_bytes) for `rows` feature rows."""
    n = ctypes.c_int32(0)
    a = ctypes.c_size_t(0)
    w = ctypes.c_size_t(0)
    _check(lib().moe_price_mlp_sizes(int(rows), ctypes.byref(n), ctypes.byref(a), ctypes.byref(w)),
           "moe_price_mlp_sizes")
    return int(n.value), int(a.value), int(w.value)


def moe_price_mlp_forward(rows, feats, params, sigma, price_hat, acts, stream):
    _check(lib().moe_price_mlp_forward(int(rows), feats, params, sigma, price_hat, acts, stream),
           "moe_price_mlp_forward")


def moe_price_mlp_backward(rows, feats, params, sigma, acts, dprice, dparams, ws, ws_bytes,
                           stream):
    _check(lib().moe_price_mlp_backward(int(rows), feats, params, sigma, acts, dprice, dparams, ws,
                                        ws_bytes, stream), "moe_price_mlp_backward")


def moe_price_mse(rows, group, price_hat, target, sigma, dprice, loss, stream):
    _check(lib().moe_price_mse(int(rows), int(group), price_hat, target, sigma, dprice, loss,
                               stream), "moe_price_mse")


def moe_adam_step(n, params, grads, m, v, lr, beta1, beta2, eps, step, stream):
    _check(lib().moe_adam_step(int(n), params, grads, m, v, float(lr), float(beta1), float(beta2),
                               float(eps), int(step), stream), "moe_adam_step")


def moe_prof_enable(on: bool) -> None:
    _check(lib().moe_prof_enable(1 if on else 0), "moe_prof_enable")


def moe_prof_lds_copy(src, dst, nbytes, stream) -> None:
    _check(lib().moe_prof_lds_copy(src, dst, nbytes, stream), "moe_prof_lds_copy")


def moe_prof_reset() -> None:
    _check(lib().moe_prof_reset(), "moe_prof_reset")


def moe_prof_get(kernel: str):
    """(total milliseconds, launches) recorded for one instrumented kernel."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int32(0)
    _check(lib().moe_prof_get(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)), "moe_prof_get")
    return float(ms.value), int(n.value)
