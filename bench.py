#!/usr/bin/env python3
"""Routed tokens/s of one mixture-of-experts layer on one MI355X.

Timed workload (the value of the JSON line): T=16384 tokens, d_model=1024,
E=64 experts, top-8, SwiGLU d_ff=2048, capacity factor 1.25, Zipf(1.2)
router bias, BF16 tokens and expert weights, FP32 router and prices; seeded
synthetic inputs already resident in HBM.  One step = router logits +
clearing-price loop + top-k + capacity check + dispatch + both grouped
expert GEMMs + combine.

Also measured (extra fields): forward+backward at T=32768, d=2048, E=128,
top-8, d_ff=1024 (Zipf 1.3); the FP8-expert forward at T=65536, d=4096,
E=64, top-8, d_ff=1408 (e4m3 weights and activations with per-block FP32
scales); the learned starting prices (E=256, d=2048: network trained on the
GPU on clearing prices of synthetic logit batches, then cold vs warm-started
routing of fresh batches and the judge's verdict on learned prices alone);
the per-stage kernel times (HIP events on the launch stream), the roofline
of the dominant kernel, and the CPU oracle on the same forward batch.

Prints ONE JSON line.  `--profile-only fwd|copy|copylds|fp8` runs a few
steps without output for hardware-counter runs (copy = a plain device copy
of 1 GiB, copylds = the same bytes read by direct-to-LDS loads, both used to
calibrate the byte counters).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP8_PEAK_TFLOPS = 5000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gemm1_bf16_scale.json")
GEMM_SRC = os.path.join(ROOT, "paper_2606_17065_amd", "csrc", "gemm.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2, help="forward workload number (1, 2, 4)")
    ap.add_argument("--bwd-config", type=int, default=4, help="fwd+bwd workload (0 = skip)")
    ap.add_argument("--cpu-tokens", type=int, default=-1,
                    help="tokens in the oracle's timed sample (-1 = the whole batch, 0 = skip)")
    ap.add_argument("--fp8", type=int, default=1, help="also time the FP8-expert workload")
    ap.add_argument("--forms", type=int, default=1,
                    help="compare every precision form (tokens/s, error vs FP64) at one shape")
    ap.add_argument("--mx", type=int, default=1,
                    help="also time the MX-expert forms (e4m3, e2m3, e2m1) at the FP8 shape")
    ap.add_argument("--rules", type=int, default=1,
                    help="compare the price rules (clearing price, restarts, subgradient)")
    ap.add_argument("--price-batches", type=int, default=10000,
                    help="training batches of the price network (0 = skip that part)")
    ap.add_argument("--price-steps", type=int, default=4000)
    ap.add_argument("--profile-only", choices=["fwd", "copy", "copylds", "fp8"], default=None)
    return ap.parse_args()


def gemm_src_hash() -> str:
    return hashlib.sha256(open(GEMM_SRC, "rb").read()).hexdigest()[:16]


def load_inputs(shape, config, dev, torch):
    from paper_2606_17065_amd import synth
    act = torch.float32 if shape.act == "f32" else torch.bfloat16
    inp = synth.make_inputs(shape, config)
    d = dict(X=torch.from_numpy(inp["X"]).to(act).to(dev),
             Wr=torch.from_numpy(inp["Wr"]).to(dev), br=torch.from_numpy(inp["br"]).to(dev),
             W13=torch.from_numpy(inp["W13"]).to(act).to(dev),
             W2=torch.from_numpy(inp["W2"]).to(act).to(dev))
    return inp, d


def make_cfg(shape, L):
    return L.make_cfg(shape.T, shape.d, shape.E, shape.k, shape.f, shape.capacity, shape.max_iters,
                      L.MOE_F32 if shape.act == "f32" else L.MOE_BF16,
                      L.MOE_F32 if shape.w == "f32" else L.MOE_BF16, L.MOE_PRICE_ACP)


def timed(fn, steps, warmup, torch, L):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    L.moe_prof_reset()
    L.moe_prof_enable(True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    L.moe_prof_enable(False)
    return ev0.elapsed_time(ev1), wall


def stage_times(L, names):
    out = {}
    for name in names:
        tot, n = L.moe_prof_get(name)
        if n:
            out[name] = {"ms": tot / n, "launches": n}
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2606_17065_amd import _lib as L
    from paper_2606_17065_amd import layer, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")

    if args.profile_only == "copy":
        a = torch.empty(1 << 29, dtype=torch.int16, device=dev).fill_(1)  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copied 1 GiB x3")
        return

    if args.profile_only == "copylds":
        a = torch.empty(1 << 29, dtype=torch.int16, device=dev).fill_(1)  # 1 GiB
        b = torch.empty_like(a)
        stream = torch.cuda.current_stream().cuda_stream
        for _ in range(3):
            L.moe_prof_lds_copy(a.data_ptr(), b.data_ptr(), a.numel() * 2, stream)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        print("copied 1 GiB x3 through LDS")
        return

    if args.profile_only == "fp8":
        args.steps = max(args.steps, 8)
        args.warmup = 0
        fp8_forward(args, dev, torch, L, layer, synth)
        torch.cuda.synchronize()
        print("fp8 forward steps done")
        return

    shape = synth.SHAPES[args.config]
    inp, D = load_inputs(shape, args.config, dev, torch)
    cfg = make_cfg(shape, L)

    def fwd():
        return layer.forward(cfg, D["X"], D["Wr"], D["br"], D["W13"], D["W2"], check=False)

    if args.profile_only == "fwd":
        for _ in range(max(args.steps, 1)):
            fwd()
        torch.cuda.synchronize()
        print("forward steps done")
        return

    gpu_ms, wall = timed(fwd, args.steps, args.warmup, torch, L)
    out = fwd()
    torch.cuda.synchronize()
    info = out["info"].cpu().numpy()
    ms_per_step = gpu_ms / args.steps
    value = shape.T * args.steps / (gpu_ms / 1e3)

    N, d, f, E, T = shape.N, shape.d, shape.f, shape.E, shape.T
    b = 4 if shape.act == "f32" else 2
    stages = stage_times(L, ("router_logits", "price_loop", "dispatch", "gemm1_swiglu", "gemm2",
                             "combine"))
    gemm1_flop = 4.0 * N * d * f
    gemm2_flop = 2.0 * N * d * f
    stages["gemm1_swiglu"].update(flop=gemm1_flop,
                                  tflops=gemm1_flop / (stages["gemm1_swiglu"]["ms"] * 1e9))
    stages["gemm2"].update(flop=gemm2_flop, tflops=gemm2_flop / (stages["gemm2"]["ms"] * 1e9))
    # with the permute fused into GEMM 1 the dispatch stage only builds the
    # slot maps (idx read, row_map and inv_map written)
    fused = layer.gather_fused(cfg)
    disp_bytes = 4.0 * (T * shape.k * 3 + E + 1) + (0.0 if fused else T * d * b + N * d * b)
    comb_bytes = N * d * b + T * d * b + 8.0 * N
    stages["dispatch"].update(bytes=disp_bytes, gbs=disp_bytes / (stages["dispatch"]["ms"] * 1e6))
    stages["combine"].update(bytes=comb_bytes, gbs=comb_bytes / (stages["combine"]["ms"] * 1e6))
    route_bytes = T * d * b + 4.0 * d * E + 8.0 * T * E
    stages["router_logits"].update(bytes=route_bytes,
                                   gbs=route_bytes / (stages["router_logits"]["ms"] * 1e6))
    dom = "gemm1_swiglu"
    ach = stages[dom]["tflops"]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("gemm_src_sha256_16") == gemm_src_hash() and tr.get("workload") == shape.name:
            traffic = tr.get("hbm_bytes_per_launch")
    roof = {"kernel": dom, "bound": "mfma", "achieved": ach, "peak": BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / BF16_PEAK_TFLOPS, "traffic": traffic,
            "algorithmic_flop_per_launch": gemm1_flop}

    rules = price_rules(args, cfg, out["logits"], torch, L) if args.rules else None
    fb = None
    if args.bwd_config:
        fb = fwd_bwd(args.bwd_config, args, dev, torch, L, layer, synth)
    f8 = fp8_forward(args, dev, torch, L, layer, synth) if args.fp8 else None
    mxr = mx_forward(args, dev, torch, L, layer, synth) if args.mx else None
    forms = forms_comparison(args, dev, torch, L, layer, synth) if args.forms else None
    lp = None
    if args.price_batches:
        from paper_2606_17065_amd import price
        lp = learned_prices(args, dev, torch, L, price, layer, synth)

    cpu = None
    if args.cpu_tokens != 0:
        T_s = T if args.cpu_tokens < 0 else min(args.cpu_tokens, T)
        cpu = cpu_baseline(shape, inp, T_s)

    rec = {
        "metric": "routed tokens/s per MoE layer (forward)",
        "value": value, "unit": "tokens/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if shape.act == "bf16" else "f32", "data": "synthetic",
        "config": {"workload": f"moe-{shape.name}", "T": T, "d_model": d, "E": E, "top_k": shape.k,
                   "d_ff": f, "capacity": shape.capacity, "zipf": shape.zipf,
                   "router": "fp32", "price": "acp", "permute": "fused into GEMM 1" if fused
                   else "explicit", "global_batch": T, "seq_len": 1,
                   "parallelism": "single-gpu"},
        "price_iters": int(info[0]), "converged": bool(info[1]),
        "slots_per_s": value * shape.k, "wall_s": wall,
        "roofline": roof, "stages": stages, "price_rules": rules, "fwd_bwd": fb, "fp8": f8,
        "mx": mxr, "forms": forms,
        "learned_price": lp,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


def fwd_bwd(config, args, dev, torch, L, layer, synth):
    """Forward + backward through the autograd Function (upstream ~N(0,1))."""
    shape = synth.SHAPES[config]
    inp, D = load_inputs(shape, config, dev, torch)
    del inp
    cfg = make_cfg(shape, L)
    params = {k: D[k].clone().requires_grad_(True) for k in ("X", "Wr", "br", "W13", "W2")}
    dOut = torch.from_numpy(synth.make_upstream(shape.T, shape.d, config)).to(torch.bfloat16).to(dev)

    def step():
        for p in params.values():
            p.grad = None
        out = layer.moe_layer(cfg, params["X"], params["Wr"], params["br"], params["W13"],
                              params["W2"], check=False)
        out.backward(dOut)

    steps = max(2, args.steps // 2)
    gpu_ms, wall = timed(step, steps, max(1, args.warmup // 2), torch, L)
    ms = gpu_ms / steps
    st = stage_times(L, ("router_logits", "price_loop", "dispatch", "gemm1_swiglu", "gemm2",
                         "combine", "combine_bwd", "ffn_bwd", "route_bwd"))
    N, d, f = shape.N, shape.d, shape.f
    if "ffn_bwd" in st:
        # the autograd layer keeps GEMM 1's pre-activations, so the expert
        # backward multiplies U = dY W2, dX_perm, dW13 and dW2: 12 N d f
        st["ffn_bwd"].update(flop=12.0 * N * d * f,
                             tflops=12.0 * N * d * f / (st["ffn_bwd"]["ms"] * 1e9))
    return {"workload": f"moe-{shape.name}", "T": shape.T, "d_model": d, "E": shape.E,
            "top_k": shape.k, "d_ff": f, "steps": steps, "ms_per_step": ms,
            "tokens_per_s": shape.T / (ms / 1e3), "stages": st}


MX_PEAK_TFLOPS = {"e4m3": 5000.0, "e2m3": 10100.0, "e2m1": 10100.0}


def price_rules(args, cfg, logits, torch, L):
    """The price rules on the forward workload's own logits: the ascending
    clearing price, the same with three epsilon-scaled restarts, and the
    projected dual subgradient (all with at most 50 updates per run).  Per
    rule: routing time (logits to routing, the repair included), updates,
    whether the last ranking met every capacity, whether the repair ran,
    and the certificate's relative gap (D(p) - sum s x) / |D(p)|."""
    from paper_2606_17065_amd import price as P
    res = {}
    for name, mode, stages in (("clearing_price", L.MOE_PRICE_ACP, 0),
                               ("clearing_price_3_restarts", L.MOE_PRICE_ACP, 3),
                               ("subgradient", L.MOE_PRICE_SUBGRAD, 0)):
        c = L.make_cfg(cfg.T, cfg.d, cfg.E, cfg.k, cfg.d_ff, cfg.capacity, 50, cfg.act, cfg.w,
                       mode, 0.9, stages)
        holder = {}

        def run():
            holder["r"] = P.route_logits(c, logits)

        ms, _ = timed(run, 10, 2, torch, L)
        r = holder["r"]
        cert = P.certify(c, logits, r["price"], r["idx"]).cpu().numpy()
        info = r["info"].cpu().numpy()
        res[name] = {"ms": ms / 10, "iters": int(info[L.INFO_ITERS]),
                     "converged": bool(info[L.INFO_CONVERGED]),
                     "repaired": bool(info[L.INFO_REPAIRED]), "gap_rel": float(cert[2])}
    return res


def forms_comparison(args, dev, torch, L, layer, synth):
    """Every precision form of the layer forward on the BF16 workload's shape
    (T=16384, d=1024, E=64, top-8, d_ff=2048, same FP32 inputs): tokens/s
    and the error of each form against the FP64 layer on the FP32 inputs
    (router logits of all tokens; Y and out of 64 sampled tokens on the
    routing each form chose, with FP64 gate weights)."""
    from oracle import ffn, routing as R
    shape = synth.SHAPES[2]
    inp = synth.make_inputs(shape, 2)
    T, d, E, k, f = shape.T, shape.d, shape.E, shape.k, shape.f
    sample = np.linspace(0, T - 1, 64).astype(np.int64)
    X64 = inp["X"].astype(np.float64)
    s64 = R.logits_fp64(X64, inp["Wr"], inp["br"])
    W13_64 = inp["W13"].astype(np.float64)
    W2_64 = inp["W2"].astype(np.float64)
    Wr = torch.from_numpy(inp["Wr"]).to(dev)
    br = torch.from_numpy(inp["br"]).to(dev)
    res = {"workload": "moe-bf16-scale shape, every form", "T": T, "d_model": d, "E": E,
           "top_k": k, "d_ff": f, "error_sample_tokens": len(sample), "forms": {}}
    forms = [("f32", L.MOE_F32, L.MOE_F32), ("bf16", L.MOE_BF16, L.MOE_BF16),
             ("fp8-e4m3 (1x128 / 128x128 FP32 scales)", L.MOE_BF16, L.MOE_FP8E4M3),
             ("mx-e4m3", L.MOE_BF16, L.MOE_MXFP8E4M3), ("mx-e2m3", L.MOE_BF16, L.MOE_MXFP6E2M3),
             ("mx-e2m1", L.MOE_BF16, L.MOE_MXFP4E2M1)]
    for name, act, w in forms:
        adt = torch.float32 if act == L.MOE_F32 else torch.bfloat16
        X = torch.from_numpy(inp["X"]).to(adt).to(dev)
        W13 = torch.from_numpy(inp["W13"]).to(dev)
        W2 = torch.from_numpy(inp["W2"]).to(dev)
        s13 = s2 = None
        if w == L.MOE_BF16:
            W13, W2 = W13.to(torch.bfloat16), W2.to(torch.bfloat16)
        elif w == L.MOE_FP8E4M3:
            (W13, s13), (W2, s2) = layer.quantize_fp8(W13, 128), layer.quantize_fp8(W2, 128)
        elif w != L.MOE_F32:
            (W13, s13), (W2, s2) = layer.quantize_mx(W13, w), layer.quantize_mx(W2, w)
        cfg = L.make_cfg(T, d, E, k, f, shape.capacity, shape.max_iters, act, w, L.MOE_PRICE_ACP)

        def fwd():
            return layer.forward(cfg, X, Wr, br, W13, W2, W13_scale=s13, W2_scale=s2,
                                 check=False)

        steps = 5
        gpu_ms, _ = timed(fwd, steps, 2, torch, L)
        r = fwd()
        torch.cuda.synchronize()
        sel = r["idx"].cpu().numpy()
        inv = r["inv_map"].cpu().numpy()
        Yg = r["Y"].float()
        s_gpu = r["logits"].cpu().numpy().astype(np.float64)
        errs = {"logits": float(np.abs(s_gpu - s64).max() / np.abs(s64).max())}
        w64 = R.gate_weights(s64[sample], sel[sample])
        y_ref = np.zeros((len(sample), k, d))
        y_got = np.zeros((len(sample), k, d))
        for a, t in enumerate(sample):
            for j in range(k):
                e = int(sel[t, j])
                x = X64[t]
                A = W13_64[e, :f] @ x
                B = W13_64[e, f:] @ x
                y_ref[a, j] = W2_64[e] @ (A / (1.0 + np.exp(-A)) * B)
                y_got[a, j] = Yg[int(inv[t, j])].cpu().numpy()
        o_ref = np.einsum("tj,tjd->td", w64, y_ref)
        o_got = r["out"][torch.from_numpy(sample).to(dev)].float().cpu().numpy()
        for key, got, ref in (("Y", y_got, y_ref), ("out", o_got, o_ref)):
            errs[key] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            errs[key + "_max_abs"] = float(np.abs(got - ref).max() / np.abs(ref).max())
        res["forms"][name] = {"ms_per_step": gpu_ms / steps,
                              "tokens_per_s": T / (gpu_ms / steps / 1e3),
                              "rel_err_vs_fp64": errs, "price_iters": int(r["info"][0])}
        del X, W13, W2, s13, s2, r, Yg
    return res


def mx_forward(args, dev, torch, L, layer, synth):
    """Forward of the FP8-expert workload's shape with OCP MX experts (e4m3,
    e2m3 and e2m1 codes, E8M0 scales per 32 along K; weights quantised once
    outside the timed region, tokens and h inside the layer)."""
    shape = synth.SHAPES[3]
    inp = synth.make_inputs(shape, 3)
    X = torch.from_numpy(inp["X"]).to(torch.bfloat16).to(dev)
    Wr = torch.from_numpy(inp["Wr"]).to(dev)
    br = torch.from_numpy(inp["br"]).to(dev)
    W13 = torch.from_numpy(inp["W13"]).to(torch.bfloat16).to(dev)
    W2 = torch.from_numpy(inp["W2"]).to(torch.bfloat16).to(dev)
    del inp
    N, d, f = shape.N, shape.d, shape.f
    res = {"workload": f"moe-{shape.name}-mx", "T": shape.T, "d_model": d, "E": shape.E,
           "top_k": shape.k, "d_ff": f, "formats": {}}
    for fmt, name in ((L.MOE_MXFP8E4M3, "e4m3"), (L.MOE_MXFP6E2M3, "e2m3"),
                      (L.MOE_MXFP4E2M1, "e2m1")):
        q13, s13 = layer.quantize_mx(W13, fmt)
        q2, s2 = layer.quantize_mx(W2, fmt)
        cfg = L.make_cfg(shape.T, d, shape.E, shape.k, f, shape.capacity, shape.max_iters,
                         L.MOE_BF16, fmt, L.MOE_PRICE_ACP)

        def fwd():
            return layer.forward(cfg, X, Wr, br, q13, q2, W13_scale=s13, W2_scale=s2, check=False)

        steps = max(2, args.steps // 4)
        gpu_ms, wall = timed(fwd, steps, max(1, args.warmup // 2), torch, L)
        ms = gpu_ms / steps
        st = stage_times(L, ("router_logits", "price_loop", "quant_mx", "dispatch", "gemm1_swiglu",
                             "gemm2", "combine"))
        st["gemm1_swiglu"].update(flop=4.0 * N * d * f,
                                  tflops=4.0 * N * d * f / (st["gemm1_swiglu"]["ms"] * 1e9))
        st["gemm2"].update(flop=2.0 * N * d * f,
                           tflops=2.0 * N * d * f / (st["gemm2"]["ms"] * 1e9))
        ach = st["gemm1_swiglu"]["tflops"]
        res["formats"][name] = {
            "steps": steps, "ms_per_step": ms, "tokens_per_s": shape.T / (ms / 1e3),
            "roofline": {"kernel": f"gemm1_swiglu (mx {name})", "bound": "mfma", "achieved": ach,
                         "peak": MX_PEAK_TFLOPS[name], "unit": "TFLOP/s",
                         "frac": ach / MX_PEAK_TFLOPS[name]},
            "stages": st}
        del q13, s13, q2, s2
    return res


def fp8_forward(args, dev, torch, L, layer, synth):
    """Forward of the FP8-expert workload: BF16 tokens, e4m3 expert weights
    with 128x128 block scales (quantised once on the GPU, outside the timed
    region), tokens (once per token, gathered by the first product) and h
    quantised per 1x128 block by the first product's epilogue."""
    shape = synth.SHAPES[3]
    inp = synth.make_inputs(shape, 3)
    X = torch.from_numpy(inp["X"]).to(torch.bfloat16).to(dev)
    Wr = torch.from_numpy(inp["Wr"]).to(dev)
    br = torch.from_numpy(inp["br"]).to(dev)
    W13 = torch.from_numpy(inp["W13"]).to(torch.bfloat16).to(dev)
    q13, s13 = layer.quantize_fp8(W13, 128)
    del W13
    W2 = torch.from_numpy(inp["W2"]).to(torch.bfloat16).to(dev)
    q2, s2 = layer.quantize_fp8(W2, 128)
    del W2, inp
    cfg = L.make_cfg(shape.T, shape.d, shape.E, shape.k, shape.f, shape.capacity, shape.max_iters,
                     L.MOE_BF16, L.MOE_FP8E4M3, L.MOE_PRICE_ACP)

    def fwd():
        return layer.forward(cfg, X, Wr, br, q13, q2, W13_scale=s13, W2_scale=s2, check=False)

    steps = max(2, args.steps // 4)
    gpu_ms, wall = timed(fwd, steps, max(1, args.warmup // 2), torch, L)
    ms = gpu_ms / steps
    st = stage_times(L, ("router_logits", "price_loop", "quant_rows", "dispatch", "gemm1_swiglu",
                         "gemm2", "combine"))
    N, d, f = shape.N, shape.d, shape.f
    st["gemm1_swiglu"].update(flop=4.0 * N * d * f,
                              tflops=4.0 * N * d * f / (st["gemm1_swiglu"]["ms"] * 1e9))
    st["gemm2"].update(flop=2.0 * N * d * f, tflops=2.0 * N * d * f / (st["gemm2"]["ms"] * 1e9))
    ach = st["gemm1_swiglu"]["tflops"]
    return {"workload": f"moe-{shape.name}", "T": shape.T, "d_model": d, "E": shape.E,
            "top_k": shape.k, "d_ff": f, "dtype": "fp8-e4m3 experts, bf16 tokens",
            "steps": steps, "ms_per_step": ms, "tokens_per_s": shape.T / (ms / 1e3),
            "roofline": {"kernel": "gemm1_swiglu (fp8)", "bound": "mfma", "achieved": ach,
                         "peak": FP8_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": ach / FP8_PEAK_TFLOPS},
            "stages": st}


def learned_prices(args, dev, torch, L, price, layer, synth):
    """Train the price network on clearing prices of synthetic logit
    batches, then route fresh batches (real tokens through the router) cold
    and from learned prices; report updates, routing time and the judge."""
    import math
    E, d, k = 256, 2048, 8
    Wr = synth.router_weights(5, E, d)
    Lc = torch.from_numpy(np.linalg.cholesky(Wr.astype(np.float64) @ Wr.astype(np.float64).T)
                          .astype(np.float32)).to(dev)
    rng = np.random.Generator(np.random.PCG64(5_000_000))
    gen = torch.Generator(device=dev)
    gen.manual_seed(5_000_001)

    def batches(n):
        for _ in range(n):
            T = int(min(65536, max(4096, math.floor(math.exp(rng.uniform(math.log(4096),
                                                                          math.log(65537)))))))
            b = torch.from_numpy(synth.zipf_bias(rng, E, float(rng.uniform(1.0, 1.5)))).to(dev)
            z = torch.randn(T, E, generator=gen, device=dev, dtype=torch.float32)
            yield (z @ Lc.T + b).contiguous(), synth.capacity(T, k, E)

    t0 = time.perf_counter()
    ds = price.build_dataset(batches(args.price_batches), E, k)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    params, hist = price.train(ds, steps=args.price_steps, batches_per_step=32, lr=1e-3, seed=0,
                               log_every=max(1, args.price_steps // 4))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    it_train = ds.iters.float()
    evals = []
    # expert weights of the layer timings: N(0, 0.02^2) drawn on the device
    # from a seeded generator (only their shape matters for the timing)
    f = synth.SHAPES[5].f
    wg = torch.Generator(device=dev)
    wg.manual_seed(5_000_002)
    W13 = (0.02 * torch.randn(E, 2 * f, d, generator=wg, device=dev)).to(torch.bfloat16)
    W2 = (0.02 * torch.randn(E, d, f, generator=wg, device=dev)).to(torch.bfloat16)
    # uneven batch lengths over the training range (none a multiple of a tile)
    for T in (4133, 11587, 30011, 65521):
        shape = synth.SHAPES[5].with_tokens(T)
        inp = synth.make_inputs(shape, 5, rep=1, experts=False)
        X = torch.from_numpy(inp["X"]).to(torch.bfloat16).to(dev)
        Wr_d = torch.from_numpy(inp["Wr"]).to(dev)
        br_d = torch.from_numpy(inp["br"]).to(dev)
        cfg = L.make_cfg(T, d, E, k, shape.f, shape.capacity, 50, L.MOE_BF16, L.MOE_BF16,
                         L.MOE_PRICE_ACP)
        logits = layer.router_logits(cfg, X, Wr_d, br_d)

        def cold():
            return price.route_logits(cfg, logits)

        def warm():
            return price.learned_route(cfg, logits, params, mode="warm", fallback="host")

        def replace():
            return price.learned_route(cfg, logits, params, mode="replace", fallback="host")

        res = {}
        for name, fn in (("cold", cold), ("warm", warm), ("replace", replace)):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            reps = 5
            for _ in range(reps):
                r = fn()
            e1.record()
            torch.cuda.synchronize()
            res[name] = {"ms": e0.elapsed_time(e1) / reps,
                         "iters": int(r["info"][L.INFO_ITERS]),
                         "converged": bool(r["info"][L.INFO_CONVERGED])}
            if name != "cold":
                res[name].update(price.verdict_dict(r))

        def layer_cold():
            return layer.forward(cfg, X, Wr_d, br_d, W13, W2, check=False)

        def layer_warm():
            return price.learned_layer_forward(cfg, X, Wr_d, br_d, W13, W2, params, mode="warm",
                                               fallback="host")

        for name, fn in (("layer_cold", layer_cold), ("layer_learned_warm", layer_warm)):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 5
            res[name] = {"ms": ms, "tokens_per_s": T / (ms / 1e3)}
        evals.append({"T": T, **res})
    return {"workload": "moe-learned-price", "E": E, "d_model": d, "top_k": k,
            "train_batches": args.price_batches, "train_steps": args.price_steps,
            "train_rows_per_step": 32 * E,
            "target_iters_mean": float(it_train.mean()), "data_s": t_data, "train_s": t_train,
            "loss": hist, "eval": evals}


def cpu_baseline(shape, inp, T_s):
    """The oracle, untuned, on the first T_s tokens of the same batch (same
    weights, capacity rescaled to T_s)."""
    import torch

    from oracle import ffn, routing as R
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    sub = shape.with_tokens(T_s)

    def stored(a):
        if shape.act == "f32":
            return np.asarray(a, np.float64)
        return torch.from_numpy(a).to(torch.bfloat16).float().double().numpy()

    Xb = stored(inp["X"][:T_s])
    W13 = stored(inp["W13"])
    W2 = stored(inp["W2"])
    reps = 0
    t0 = time.perf_counter()
    while reps < 5 and (reps == 0 or time.perf_counter() - t0 < 10.0):
        s64 = R.logits_fp64(Xb, inp["Wr"], inp["br"])
        r = R.route(s64.astype(np.float32), sub.k, sub.capacity, sub.max_iters)
        ffn.layer_forward(Xb, r["sel"], r["w"], W13, W2)
        reps += 1
    dt = time.perf_counter() - t0
    return {"value": T_s * reps / dt, "unit": "tokens/s", "cores": cores, "kind": "oracle",
            "sample": f"{'the whole batch' if T_s == shape.T else f'first {T_s} tokens'} "
                      f"({T_s} tokens, capacity {sub.capacity}) of the timed workload, same "
                      f"weights, {reps} repetition(s): full layer forward in FP64 NumPy "
                      f"(logits, price loop, top-k, dispatch, experts, combine)",
            "seconds": dt}


if __name__ == "__main__":
    main()
