"""FP64 price MLP, its features and Adam -- TEST INFRASTRUCTURE ONLY.

Parity unpinned by the paper (it has no learned price).  The reading:

Features.  For logits s [T,E] with mean mu and population std sigma_s (over
all entries), capacity C and top-k size k, expert e gets eight numbers:
  1. (mean_t s_te - mu) / sigma_s        2. std_t s_te / sigma_s
  3. (max_t s_te - mu) / sigma_s         4. (q_{C+1}(s_.e) - mu) / sigma_s
  5. load0_e / C                         6. mean_t m0_te / sigma_s
  7. q_{C+1}(m0_.e) / sigma_s            8. std_t m0_te / sigma_s
where q_{C+1} is the (C+1)-th largest value (or the smallest, when T <= C),
load0 the plain top-k load at zero prices and m0 the price margins at zero
prices: m0_te = s_te - (e chosen by t ? kappa2_t : kappa1_t), with kappa1_t,
kappa2_t the k-th and (k+1)-th largest scores of token t.

Network, shared by all experts: 8 -> 256 -> 256 -> 1 with exact (erf) GELU
after both hidden layers; z = output; p_hat_e = sigma_s * softplus(z_e).
Training loss over rows r of a minibatch: mean_r (softplus(z_r) - y_r)^2
with y = p_star / sigma_s.  Adam with bias correction:
  m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
  theta -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).

Parameter vector layout (float32 on the device, float64 here):
  W1 [256,8], b1 [256], W2 [256,256], b2 [256], w3 [256], b3 [1].
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special

from .routing import f32_key

H = 256
NF = 8
SIZES = [("W1", (H, NF)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], np.float64).ravel() for name, _ in SIZES])


def init_params(seed: int) -> np.ndarray:
    """He-style normal init of the weights, zero biases (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = {
        "W1": rng.standard_normal((H, NF)) * math.sqrt(2.0 / NF),
        "b1": np.zeros(H),
        "W2": rng.standard_normal((H, H)) * math.sqrt(2.0 / H),
        "b2": np.zeros(H),
        "w3": rng.standard_normal(H) * math.sqrt(1.0 / H),
        "b3": np.zeros(1),
    }
    return pack(parts).astype(np.float32)


def gelu(z):
    return 0.5 * z * (1.0 + scipy.special.erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + scipy.special.erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def softplus(z):
    return np.logaddexp(0.0, z)


def forward(theta, F):
    """z [R] and the cached activations for rows F [R,8] (FP64)."""
    P = unpack(theta)
    F = np.asarray(F, np.float64)
    u1 = F @ P["W1"].T + P["b1"]
    a1 = gelu(u1)
    u2 = a1 @ P["W2"].T + P["b2"]
    a2 = gelu(u2)
    z = a2 @ P["w3"] + P["b3"][0]
    return z, dict(F=F, u1=u1, a1=a1, u2=u2, a2=a2)


def loss_and_grad(theta, F, y):
    """Mean squared error of softplus(z) against y and its gradient."""
    P = unpack(theta)
    z, c = forward(theta, F)
    R = z.shape[0]
    r = softplus(z) - np.asarray(y, np.float64)
    loss = float(np.mean(r * r))
    dz = (2.0 / R) * r * scipy.special.expit(z)
    g = {}
    g["w3"] = c["a2"].T @ dz
    g["b3"] = np.array([dz.sum()])
    da2 = np.outer(dz, P["w3"])
    du2 = da2 * gelu_grad(c["u2"])
    g["W2"] = du2.T @ c["a1"]
    g["b2"] = du2.sum(axis=0)
    da1 = du2 @ P["W2"]
    du1 = da1 * gelu_grad(c["u1"])
    g["W1"] = du1.T @ c["F"]
    g["b1"] = du1.sum(axis=0)
    return loss, pack(g)


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (FP64); step counts from 1.  Returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def _qdesc(col: np.ndarray, r: int) -> float:
    """r-th largest entry of a column (1-based), or its minimum if r > len."""
    srt = np.sort(col)[::-1]
    return float(srt[min(r, col.shape[0]) - 1])


def features(s, k, C):
    """The eight per-expert statistics [E,8] of FP32 logits s (computed in
    FP64).  The plain top-k behind kappa and load0 ranks each token's
    experts by the total-order key of the FP32 logit, descending, ties to
    the lower expert (the ranking rule of the price update), so -0.0 ranks
    below +0.0."""
    key = f32_key(np.asarray(s, np.float32)).astype(np.int64)
    s = np.asarray(s, np.float64)
    T, E = s.shape
    mu = s.mean()
    sig = s.std()
    sig = sig if sig > 0 else 1.0
    order = np.lexsort((np.broadcast_to(np.arange(E), (T, E)), -key), axis=1)
    rows = np.arange(T)
    kap1 = s[rows, order[:, k - 1]]
    kap2 = s[rows, order[:, k]] if k < E else np.full(T, -np.inf)
    held = np.zeros((T, E), dtype=bool)
    held[rows[:, None], order[:, :k]] = True
    m0 = s - np.where(held, kap2[:, None], kap1[:, None])
    load0 = held.sum(axis=0)
    Fm = np.zeros((E, 8))
    for e in range(E):
        col = s[:, e]
        Fm[e, 0] = (col.mean() - mu) / sig
        Fm[e, 1] = col.std() / sig
        Fm[e, 2] = (col.max() - mu) / sig
        Fm[e, 3] = (_qdesc(col, C + 1) - mu) / sig
        Fm[e, 4] = load0[e] / C
        Fm[e, 5] = m0[:, e].mean() / sig
        Fm[e, 6] = _qdesc(m0[:, e], C + 1) / sig
        Fm[e, 7] = m0[:, e].std() / sig
    return Fm
