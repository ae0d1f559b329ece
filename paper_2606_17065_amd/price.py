"""Learned starting prices: batch logit statistics, the price network, its
training, and routing that starts from (or replaces) the clearing-price
update with the exact update as fallback and judge.

Every computation runs in libmoe's kernels; this module allocates device
tensors and passes pointers and streams.  The judge's decision (keep the
learned routing or route again from zero prices) is made on the device by
moe_route_judged.
"""
from __future__ import annotations

import dataclasses

import torch

from . import _lib as L
from .layer import _WS, _fresh_price, _need, _p, _stream

GAP_TOL = 5e-3  # relative duality gap the judge accepts (the update's own level)


def route_logits(cfg, logits, price=None, ws=None):
    """moe_route from given logits [T,E] f32; returns the routing dict."""
    T, E, k = cfg.T, cfg.E, cfg.k
    _need(logits, "logits", torch.float32, (T, E))
    dev = logits.device
    if price is None:
        price = _fresh_price(cfg, dev)
    else:
        _need(price, "price", torch.float32, (E,))
    out = dict(price=price, idx=torch.empty(T, k, dtype=torch.int32, device=dev),
               w=torch.empty(T, k, dtype=torch.float32, device=dev),
               load=torch.empty(E, dtype=torch.int32, device=dev),
               info=torch.empty(L.INFO_LEN, dtype=torch.int32, device=dev))
    ws = _WS.get(cfg, dev) if ws is None else ws
    L.moe_route_logits(cfg, _p(logits), _p(price), _p(out["idx"]), _p(out["w"]), _p(out["load"]),
                       _p(out["info"]), _p(ws), ws.numel(), _stream())
    return out


def price_update(cfg, logits, price=None, ws=None):
    """moe_price_update: (price [E], info) after the price update on logits."""
    _need(logits, "logits", torch.float32, (cfg.T, cfg.E))
    dev = logits.device
    if price is None:
        price = _fresh_price(cfg, dev)
    else:
        _need(price, "price", torch.float32, (cfg.E,))
    info = torch.empty(L.INFO_LEN, dtype=torch.int32, device=dev)
    ws = _WS.get(cfg, dev) if ws is None else ws
    L.moe_price_update(cfg, _p(logits), _p(price), _p(info), _p(ws), ws.numel(), _stream())
    return price, info


def certify(cfg, logits, price, idx, ws=None):
    """[primal, dual, gap_rel] (f64 device tensor) of a routing under prices."""
    _need(logits, "logits", torch.float32, (cfg.T, cfg.E))
    _need(idx, "topk_idx", torch.int32, (cfg.T, cfg.k))
    cert = torch.empty(3, dtype=torch.float64, device=logits.device)
    ws = _WS.get(cfg, logits.device) if ws is None else ws
    L.moe_route_certify(cfg, _p(logits), _p(price), _p(idx), _p(cert), _p(ws), ws.numel(),
                        _stream())
    return cert


def logit_stats(cfg, logits, ws=None):
    """(features [E,8] f32, sigma [1] f32) of a batch of logits."""
    _need(logits, "logits", torch.float32, (cfg.T, cfg.E))
    dev = logits.device
    feats = torch.empty(cfg.E, 8, dtype=torch.float32, device=dev)
    sigma = torch.empty(1, dtype=torch.float32, device=dev)
    ws = _WS.get(cfg, dev) if ws is None else ws
    L.moe_logit_stats(cfg, _p(logits), _p(feats), _p(sigma), _p(ws), ws.numel(), _stream())
    return feats, sigma


def n_params() -> int:
    return L.moe_price_mlp_sizes(0)[0]


def mlp_forward(params, feats, sigma=None):
    """(p_hat [rows], acts) for features [rows,8]; sigma None = sigma units."""
    rows = feats.shape[0]
    _need(feats, "feats", torch.float32, (rows, 8))
    _need(params, "params", torch.float32, (n_params(),))
    _, nacts, _ = L.moe_price_mlp_sizes(rows)
    acts = torch.empty(max(nacts, 1), dtype=torch.float32, device=feats.device)
    phat = torch.empty(rows, dtype=torch.float32, device=feats.device)
    L.moe_price_mlp_forward(rows, _p(feats), _p(params), _p(sigma), _p(phat), _p(acts), _stream())
    return phat, acts


def mlp_backward(params, feats, acts, dprice, sigma=None, ws=None):
    rows = feats.shape[0]
    _, _, nws = L.moe_price_mlp_sizes(rows)
    if ws is None or ws.numel() < nws:
        ws = torch.empty(max(nws, 256), dtype=torch.uint8, device=feats.device)
    dparams = torch.empty_like(params)
    L.moe_price_mlp_backward(rows, _p(feats), _p(params), _p(sigma), _p(acts), _p(dprice),
                             _p(dparams), _p(ws), ws.numel(), _stream())
    return dparams


def mse(phat, target, sigma=None, group=None):
    """(loss [1], dprice [rows]) of p_hat against target / sigma[r // group]."""
    rows = phat.shape[0]
    group = rows if group is None else group
    loss = torch.empty(1, dtype=torch.float32, device=phat.device)
    dprice = torch.empty(rows, dtype=torch.float32, device=phat.device)
    L.moe_price_mse(rows, group, _p(phat), _p(target), _p(sigma), _p(dprice), _p(loss), _stream())
    return loss, dprice


class Adam:
    """Adam state over one parameter vector; step() runs moe_adam_step."""

    def __init__(self, params, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        self.params, self.lr, self.betas, self.eps = params, lr, betas, eps
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.t = 0

    def step(self, grads):
        self.t += 1
        L.moe_adam_step(self.params.numel(), _p(self.params), _p(grads), _p(self.m), _p(self.v),
                        self.lr, self.betas[0], self.betas[1], self.eps, self.t, _stream())


@dataclasses.dataclass
class PriceDataset:
    """Rows of (features, target price, sigma) for B batches of E experts;
    row r belongs to batch r // E."""

    feats: torch.Tensor  # [B*E, 8]
    target: torch.Tensor  # [B*E] clearing prices p*
    sigma: torch.Tensor  # [B]
    iters: torch.Tensor  # [B] int32: price updates the exact update needed
    E: int


def build_dataset(batches, E, k, max_iters=50):
    """batches: iterable of (logits [T,E] f32 device tensor, C).  Features
    and sigma from moe_logit_stats, targets from the exact clearing-price
    update (moe_route_logits, MOE_PRICE_ACP, starting at p = 0)."""
    feats, target, sigma, iters = [], [], [], []
    for s, C in batches:
        cfg = L.make_cfg(s.shape[0], 8, E, k, 1, C, max_iters, L.MOE_F32, L.MOE_F32,
                         L.MOE_PRICE_ACP)
        f, sg = logit_stats(cfg, s)
        r = route_logits(cfg, s)
        feats.append(f)
        sigma.append(sg)
        target.append(r["price"])
        iters.append(r["info"][L.INFO_ITERS:L.INFO_ITERS + 1])
    return PriceDataset(torch.cat(feats), torch.cat(target), torch.cat(sigma),
                        torch.cat(iters), E)


def init_params(seed: int, device) -> torch.Tensor:
    """He-normal weights, zero biases (the network's starting point)."""
    g = torch.Generator().manual_seed(seed)
    H, NF = 256, 8
    parts = [torch.randn(H * NF, generator=g, dtype=torch.float64) * (2.0 / NF) ** 0.5,
             torch.zeros(H, dtype=torch.float64),
             torch.randn(H * H, generator=g, dtype=torch.float64) * (2.0 / H) ** 0.5,
             torch.zeros(H, dtype=torch.float64),
             torch.randn(H, generator=g, dtype=torch.float64) * (1.0 / H) ** 0.5,
             torch.zeros(1, dtype=torch.float64)]
    return torch.cat(parts).to(torch.float32).to(device)


def train(ds: PriceDataset, steps=2000, batches_per_step=32, lr=1e-3, seed=0, params=None,
          log_every=0):
    """Adam on the mean squared error of softplus(z) against p*/sigma over
    minibatches of whole batches (consecutive in a fixed seeded order of
    the dataset).  Returns (params, list of (step, loss))."""
    dev = ds.feats.device
    B, E = ds.sigma.numel(), ds.E
    params = init_params(seed, dev) if params is None else params
    opt = Adam(params, lr=lr)
    perm = torch.randperm(B, generator=torch.Generator().manual_seed(seed + 1))
    rows_idx = (perm[:, None] * E + torch.arange(E)[None, :]).reshape(-1).to(dev)
    feats = ds.feats.index_select(0, rows_idx).contiguous()
    target = ds.target.index_select(0, rows_idx).contiguous()
    sigma = ds.sigma.index_select(0, perm.to(dev)).contiguous()
    mb = min(batches_per_step, B)
    rows = mb * E
    _, _, nws = L.moe_price_mlp_sizes(rows)
    ws = torch.empty(max(nws, 256), dtype=torch.uint8, device=dev)
    hist = []
    for step in range(steps):
        b0 = (step * mb) % (B - mb + 1) if B > mb else 0
        F = feats[b0 * E:(b0 + mb) * E]
        y = target[b0 * E:(b0 + mb) * E]
        sg = sigma[b0:b0 + mb]
        phat, acts = mlp_forward(params, F)
        loss, dprice = mse(phat, y, sg, group=E)
        grads = mlp_backward(params, F, acts, dprice, ws=ws)
        opt.step(grads)
        if log_every and (step % log_every == 0 or step == steps - 1):
            hist.append((step, float(loss.item())))
    return params, hist


def predict(cfg, logits, params):
    """p_hat [E] for one batch of logits: statistics, then the network."""
    feats, sigma = logit_stats(cfg, logits)
    phat, _ = mlp_forward(params, feats, sigma)
    return phat


VERDICT_V, VERDICT_GAP, VERDICT_KEPT, VERDICT_GAP_FINAL, VERDICT_ITERS = range(5)


def judged_route(cfg, logits, phat, mode="warm", gamma=0.9, gap_tol=GAP_TOL, ws=None,
                 fallback="device"):
    """moe_route_judged: the routing from learned prices p_hat, kept when the
    certificate's relative gap is <= gap_tol, else the exact update from
    p = 0.  fallback="device" decides on the device (the fallback pass is
    always enqueued and exits at once when it is not needed); "host" calls
    moe_route_learned, reads the verdict (one wait for the stream) and runs
    the update from p = 0 only when the judge rejected the learned routing.
    Returns the routing dict plus the verdict tensor [5] f64 (V, learned
    gap, kept, final gap, learned-pass updates)."""
    T, E, k = cfg.T, cfg.E, cfg.k
    _need(logits, "logits", torch.float32, (T, E))
    _need(phat, "price_hat", torch.float32, (E,))
    if mode not in ("warm", "replace"):
        raise ValueError(f"unknown mode {mode!r}")
    pm = L.MOE_PRICE_WARM if mode == "warm" else L.MOE_PRICE_GIVEN
    c = L.make_cfg(T, cfg.d, E, k, cfg.d_ff, cfg.capacity, cfg.max_iters, cfg.act, cfg.w, pm, gamma,
                   cfg.price_stages)
    dev = logits.device
    out = dict(price=torch.empty(E, dtype=torch.float32, device=dev),
               idx=torch.empty(T, k, dtype=torch.int32, device=dev),
               w=torch.empty(T, k, dtype=torch.float32, device=dev),
               load=torch.empty(E, dtype=torch.int32, device=dev),
               info=torch.empty(L.INFO_LEN, dtype=torch.int32, device=dev),
               verdict=torch.empty(5, dtype=torch.float64, device=dev))
    ws = _WS.get(c, dev) if ws is None else ws
    if fallback == "device":
        L.moe_route_judged(c, _p(logits), _p(phat), gap_tol, _p(out["price"]), _p(out["idx"]),
                           _p(out["w"]), _p(out["load"]), _p(out["info"]), _p(out["verdict"]),
                           _p(ws), ws.numel(), _stream())
        return out
    if fallback != "host":
        raise ValueError(f"unknown fallback {fallback!r}")
    L.moe_route_learned(c, _p(logits), _p(phat), gap_tol, _p(out["price"]), _p(out["idx"]),
                        _p(out["w"]), _p(out["load"]), _p(out["info"]), _p(out["verdict"]),
                        _p(ws), ws.numel(), _stream())
    if float(out["verdict"][VERDICT_KEPT].item()) != 1.0 and \
            int(out["info"][L.INFO_STATUS].item()) != L.MOE_ENAN:
        c0 = L.make_cfg(T, cfg.d, E, k, cfg.d_ff, cfg.capacity, cfg.max_iters, cfg.act, cfg.w,
                        L.MOE_PRICE_ACP, gamma, cfg.price_stages)
        r0 = route_logits(c0, logits, out["price"], ws=ws)
        cert = certify(c0, logits, r0["price"], r0["idx"], ws=ws)
        out.update({key: r0[key] for key in ("price", "idx", "w", "load", "info")})
        out["verdict"][VERDICT_GAP_FINAL] = cert[2]
    return out


def learned_route(cfg, logits, params, mode="warm", gamma=0.9, gap_tol=GAP_TOL,
                  fallback="device"):
    """Route one batch with learned prices (statistics, network, then
    moe_route_judged; no host synchronisation).

    warm:    p0 = gamma * p_hat, then the exact clearing-price update.
    replace: route under p_hat alone (the capacity repair places any
             overflow).
    Either routing is kept when its certificate gap is <= gap_tol, else the
    batch is routed again by the exact update from p = 0.  Returns the
    routing dict plus p_hat and the verdict tensor."""
    phat = predict(cfg, logits, params)
    r = judged_route(cfg, logits, phat, mode, gamma, gap_tol, fallback=fallback)
    r["p_hat"] = phat
    return r


def verdict_dict(r):
    """Host copy of a judged routing's verdict (waits for the stream)."""
    v = r["verdict"].cpu().numpy()
    return {"V": float(v[VERDICT_V]), "gap_learned": float(v[VERDICT_GAP]),
            "kept": bool(v[VERDICT_KEPT] == 1.0), "gap": float(v[VERDICT_GAP_FINAL]),
            "learned_iters": int(v[VERDICT_ITERS])}


def learned_layer_forward(cfg, X, Wr, br, W13, W2, params, mode="warm", gamma=0.9,
                          gap_tol=GAP_TOL, fallback="device"):
    """The layer forward with learned prices (BF16 experts): router logits,
    statistics and the price network, the judged routing (warm start or
    replacement, the exact update as judge and fallback), dispatch maps, the
    gather-fused expert products and the combine.  No host synchronisation.
    Returns the routing dict plus Y and out."""
    from . import layer
    logits = layer.router_logits(cfg, X, Wr, br)
    r = learned_route(cfg, logits, params, mode, gamma, gap_tol, fallback)
    dsp = layer.dispatch(cfg, X, r["idx"], permute=False)
    Y = layer.expert_ffn_gather(cfg, X, dsp["row_map"], dsp["offsets"], W13, W2)
    r.update(dsp)
    r["logits"] = logits
    r["Y"] = Y
    r["out"] = layer.combine(cfg, Y, dsp["inv_map"], r["w"])
    return r
