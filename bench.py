#!/usr/bin/env python3
"""Routed tokens/s of one mixture-of-experts layer on one MI355X.

Workload (default): T=16384 tokens, d_model=1024, E=64 experts, top-8,
SwiGLU d_ff=2048, capacity factor 1.25, Zipf(1.2) router bias, BF16 tokens
and expert weights, FP32 router and prices; seeded synthetic inputs already
resident in HBM.  One step = router logits + clearing-price loop + top-k +
capacity check + dispatch + both grouped expert GEMMs + combine.

Prints ONE JSON line (rank 0) with the throughput, the roofline of the
dominant kernel (timed live with HIP events on the launch stream) and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2, help="workload number (1..5)")
    ap.add_argument("--cpu-tokens", type=int, default=4096,
                    help="tokens in the oracle's timed sample (0 = skip)")
    ap.add_argument("--traffic", type=str, default=None,
                    help="JSON file with counter-derived HBM bytes per launch of the dominant kernel")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2606_17065_amd import _lib as L
    from paper_2606_17065_amd import layer, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    shape = synth.SHAPES[args.config]
    if shape.w == "fp8":
        print("FP8 experts are not built yet", file=sys.stderr)
        sys.exit(2)
    act = torch.float32 if shape.act == "f32" else torch.bfloat16
    inp = synth.make_inputs(shape, args.config)
    X = torch.from_numpy(inp["X"]).to(act).to(dev)
    Wr = torch.from_numpy(inp["Wr"]).to(dev)
    br = torch.from_numpy(inp["br"]).to(dev)
    W13 = torch.from_numpy(inp["W13"]).to(act).to(dev)
    W2 = torch.from_numpy(inp["W2"]).to(act).to(dev)
    cfg = L.make_cfg(shape.T, shape.d, shape.E, shape.k, shape.f, shape.capacity, shape.max_iters,
                     L.MOE_F32 if shape.act == "f32" else L.MOE_BF16,
                     L.MOE_F32 if shape.w == "f32" else L.MOE_BF16, L.MOE_PRICE_ACP)

    def step():
        return layer.forward(cfg, X, Wr, br, W13, W2)

    for _ in range(args.warmup):
        out = step()
    torch.cuda.synchronize()
    info = out["info"].cpu().numpy()

    L.moe_prof_reset()
    L.moe_prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        out = step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    L.moe_prof_enable(False)
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    value = shape.T * args.steps / (gpu_ms / 1e3)

    N, d, f, E, T = shape.N, shape.d, shape.f, shape.E, shape.T
    b = 4 if shape.act == "f32" else 2
    stages = {}
    for name in ("router_logits", "price_loop", "dispatch", "gemm1_swiglu", "gemm2", "combine"):
        tot, n = L.moe_prof_get(name)
        stages[name] = {"ms": tot / max(n, 1), "launches": n}
    # algorithmic work per launch
    gemm1_flop = 4.0 * N * d * f
    gemm2_flop = 2.0 * N * d * f
    stages["gemm1_swiglu"].update(flop=gemm1_flop, tflops=gemm1_flop / (stages["gemm1_swiglu"]["ms"] * 1e9))
    stages["gemm2"].update(flop=gemm2_flop, tflops=gemm2_flop / (stages["gemm2"]["ms"] * 1e9))
    disp_bytes = T * d * b + N * d * b + 4.0 * (T * shape.k * 3 + E + 1)
    comb_bytes = N * d * b + T * d * b + 8.0 * N
    stages["dispatch"].update(bytes=disp_bytes, gbs=disp_bytes / (stages["dispatch"]["ms"] * 1e6))
    stages["combine"].update(bytes=comb_bytes, gbs=comb_bytes / (stages["combine"]["ms"] * 1e6))
    dom = max(("gemm1_swiglu", "gemm2"), key=lambda k: stages[k]["ms"])
    ach = stages[dom]["tflops"]
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        traffic = json.load(open(args.traffic)).get(dom)
    roof = {"kernel": dom, "bound": "mfma", "achieved": ach, "peak": BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / BF16_PEAK_TFLOPS, "traffic": traffic}

    cpu = None
    if args.cpu_tokens > 0:
        cpu = cpu_baseline(shape, inp, args.cpu_tokens)

    rec = {
        "metric": "routed tokens/s per MoE layer (forward)",
        "value": value, "unit": "tokens/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if shape.act == "bf16" else "f32", "data": "synthetic",
        "config": {"workload": f"moe-{shape.name}", "T": T, "d_model": d, "E": E, "top_k": shape.k,
                   "d_ff": f, "capacity": shape.capacity, "zipf": shape.zipf,
                   "router": "fp32", "price": "acp", "global_batch": T, "seq_len": 1,
                   "parallelism": "single-gpu"},
        "price_iters": int(info[0]), "converged": bool(info[1]),
        "slots_per_s": value * shape.k, "wall_s": wall,
        "roofline": roof, "stages": stages, "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


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
    t0 = time.perf_counter()
    s64 = R.logits_fp64(Xb, inp["Wr"], inp["br"])
    r = R.route(s64.astype(np.float32), sub.k, sub.capacity, sub.max_iters)
    ffn.layer_forward(Xb, r["sel"], r["w"], W13, W2)
    dt = time.perf_counter() - t0
    return {"value": T_s / dt, "unit": "tokens/s", "cores": cores, "kind": "oracle",
            "sample": f"first {T_s} tokens of the timed batch, same weights, capacity "
                      f"{sub.capacity}: full layer forward in FP64 NumPy (logits, price loop, "
                      f"top-k, dispatch, experts, combine)",
            "seconds": dt}


if __name__ == "__main__":
    main()
