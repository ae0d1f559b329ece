"""Seeded synthetic inputs for the mixture-of-experts layer.

This module holds no arithmetic of the layer itself: it only draws random
numbers and reports shapes.  Both the HIP path and the CPU oracle consume
what it returns, so it must not import either of them.

Recipe (stated once here, used everywhere):

* generator: NumPy PCG64, ``seed = 1000 * config_number + rep``;
* tokens X ~ N(0, 1), float32 draws;
* router weights W_r ~ N(0, 0.02^2), expert weights W1, W3, W2 ~ N(0, 0.02^2);
* router bias b_e = -s_z * ln(r_e) with r a seeded permutation of 1..E
  (Zipf(s_z) expert popularity);
* capacity C = ceil(1.25 * T * k / E) for every expert;
* upstream gradients dOut ~ N(0, 1).

Expert weights are laid out K-contiguous: W13 is [E, 2f, d] (rows 0..f-1
hold W1, rows f..2f-1 hold W3) and W2 is [E, d, f].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class MoEShape:
    """One workload: T tokens of width d, E experts, top-k, SwiGLU width f."""

    name: str
    T: int
    d: int
    E: int
    k: int
    f: int
    zipf: float
    act: str  # "f32" or "bf16": token / activation storage type
    w: str  # "f32", "bf16" or "fp8": expert weight type
    cap_factor: float = 1.25
    max_iters: int = 50

    @property
    def N(self) -> int:
        return self.T * self.k

    @property
    def capacity(self) -> int:
        return capacity(self.T, self.k, self.E, self.cap_factor)

    def with_tokens(self, T: int) -> "MoEShape":
        return dataclasses.replace(self, T=T)


def capacity(T: int, k: int, E: int, cap_factor: float = 1.25) -> int:
    """C = ceil(cap_factor * T * k / E), computed exactly for factor 1.25."""
    if cap_factor == 1.25:
        return (5 * T * k + 4 * E - 1) // (4 * E)
    return int(math.ceil(cap_factor * T * k / E))


# The five workloads of the benchmark, by number.
SHAPES = {
    1: MoEShape("fp32-small", T=512, d=128, E=8, k=2, f=256, zipf=1.1, act="f32", w="f32"),
    2: MoEShape("bf16-scale", T=16384, d=1024, E=64, k=8, f=2048, zipf=1.2, act="bf16", w="bf16"),
    3: MoEShape("fp8-experts", T=65536, d=4096, E=64, k=8, f=1408, zipf=1.2, act="bf16", w="fp8"),
    4: MoEShape("bf16-fwd-bwd", T=32768, d=2048, E=128, k=8, f=1024, zipf=1.3, act="bf16", w="bf16"),
    5: MoEShape("learned-price", T=16384, d=2048, E=256, k=8, f=768, zipf=1.25, act="bf16", w="bf16"),
}


def rng_for(config: int, rep: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * config + rep))


def zipf_bias(rng: np.random.Generator, E: int, s_z: float) -> np.ndarray:
    """b_e = -s_z * ln(r_e), r a random permutation of 1..E (float32)."""
    ranks = rng.permutation(E) + 1
    return (-s_z * np.log(ranks.astype(np.float64))).astype(np.float32)


def make_inputs(shape: MoEShape, config: int, rep: int = 0, experts: bool = True) -> dict:
    """Draw one batch: X [T,d], Wr [E,d], br [E], and (if ``experts``)
    W13 [E,2f,d], W2 [E,d,f].  All float32; storage rounding (BF16/FP8) is
    the caller's business."""
    rng = rng_for(config, rep)
    T, d, E, f = shape.T, shape.d, shape.E, shape.f
    out = {}
    out["X"] = rng.standard_normal((T, d), dtype=np.float32)
    out["Wr"] = (0.02 * rng.standard_normal((E, d), dtype=np.float32)).astype(np.float32)
    out["br"] = zipf_bias(rng, E, shape.zipf)
    if experts:
        out["W13"] = (0.02 * rng.standard_normal((E, 2 * f, d), dtype=np.float32)).astype(np.float32)
        out["W2"] = (0.02 * rng.standard_normal((E, d, f), dtype=np.float32)).astype(np.float32)
    return out


def make_upstream(T: int, d: int, config: int, rep: int = 0) -> np.ndarray:
    """dOut ~ N(0,1), from a stream separate from make_inputs'."""
    rng = np.random.Generator(np.random.PCG64(1000 * config + rep + 500))
    return rng.standard_normal((T, d), dtype=np.float32)


def make_logits(T: int, E: int, s_z: float, seed: int, scale: float = 0.64) -> np.ndarray:
    """Router-logit-shaped scores without a router GEMM: s = scale * Z + b,
    Z ~ N(0,1) [T,E], b the Zipf bias.  Distributionally what X W_r^T + b
    gives for X ~ N(0,1) and independent rows of W_r with norm ``scale``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = zipf_bias(rng, E, s_z)
    z = rng.standard_normal((T, E), dtype=np.float32)
    return (np.float32(scale) * z + b[None, :]).astype(np.float32)


def tiny_logits(T: int, E: int, seed: int) -> np.ndarray:
    """Small score matrices for exhaustive checks: N(0,1) plus a mild skew."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = zipf_bias(rng, E, 1.0)
    return (rng.standard_normal((T, E), dtype=np.float32) + b[None, :]).astype(np.float32)


def price_batch_logits(i: int, E: int = 256, d: int = 2048, k: int = 8,
                       t_min: int = 4096, t_max: int = 65536, Wr: np.ndarray | None = None):
    """Training batch ``i`` of the learned-price workload: router logits
    drawn without tokens, s = Z L^T + b with L = chol(W_r W_r^T) (rows of
    X W_r^T for X ~ N(0, 1) have exactly this law), Z ~ N(0, 1) [T, E].

    T is log-uniform over the integers [t_min, t_max]; the Zipf exponent is
    U[1.0, 1.5] per batch.  ``Wr`` defaults to the learned-price workload's
    router weights (workload 5, rep 0).  Returns (logits [T,E] float32, C)."""
    if Wr is None:
        Wr = router_weights(5, E, d)
    L = np.linalg.cholesky(Wr.astype(np.float64) @ Wr.astype(np.float64).T).astype(np.float32)
    rng = np.random.Generator(np.random.PCG64(5_000_000 + i))
    T = int(math.floor(math.exp(rng.uniform(math.log(t_min), math.log(t_max + 1)))))
    T = min(max(T, t_min), t_max)
    s_z = float(rng.uniform(1.0, 1.5))
    b = zipf_bias(rng, E, s_z)
    z = rng.standard_normal((T, E), dtype=np.float32)
    s = (z @ L.T + b[None, :]).astype(np.float32)
    return s, capacity(T, k, E)


def router_weights(config: int, E: int, d: int, rep: int = 0) -> np.ndarray:
    """The W_r that make_inputs(config, rep) draws (same stream position)."""
    rng = rng_for(config, rep)
    shape = SHAPES[config]
    rng.standard_normal((shape.T, shape.d), dtype=np.float32)  # X
    assert shape.d == d and shape.E == E
    return (0.02 * rng.standard_normal((E, d), dtype=np.float32)).astype(np.float32)
