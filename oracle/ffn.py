"""FP64 dispatch, SwiGLU experts and weighted combine -- TEST INFRASTRUCTURE ONLY.

Parity unpinned by the paper (it defines no expert layer); the reading:

* dispatch: slots are ordered by expert, then by token (ascending);
  offsets[e] is the first slot of expert e (exclusive prefix sum of the
  loads), row_map[slot] the token of a slot, inv_map[t, j] the slot of the
  token's j-th chosen expert;
* expert e maps a token row x to y = (silu(x W1_e^T) * (x W3_e^T)) W2_e^T
  with silu(z) = z / (1 + exp(-z)), no biases; W13[e] stacks W1_e (rows
  0..f-1) over W3_e (rows f..2f-1), W2[e] is [d, f];
* combine: out_t = sum_j w[t, j] * y of the slot inv_map[t, j], summed in
  j order.
"""
from __future__ import annotations

import numpy as np
import scipy.special


def dispatch_maps(sel: np.ndarray, E: int):
    """(offsets [E+1], row_map [N], inv_map [T,k]) for slots in (expert,
    token) order."""
    T, k = sel.shape
    t_of = np.repeat(np.arange(T), k)
    e_of = sel.ravel().astype(np.int64)
    order = np.lexsort((t_of, e_of))  # expert major, token minor
    row_map = t_of[order].astype(np.int32)
    counts = np.bincount(e_of, minlength=E)
    offsets = np.zeros(E + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(counts)
    inv = np.empty(T * k, dtype=np.int64)
    inv[order] = np.arange(T * k)
    return offsets, row_map, inv.reshape(T, k).astype(np.int32)


def silu(z):
    return z * scipy.special.expit(z)


def expert_forward(x, W13e, W2e):
    """Returns (A, B, h, y) for rows x [n,d] through one expert, FP64."""
    x = np.asarray(x, np.float64)
    W13e = np.asarray(W13e, np.float64)
    f = W13e.shape[0] // 2
    A = x @ W13e[:f].T
    B = x @ W13e[f:].T
    h = silu(A) * B
    y = h @ np.asarray(W2e, np.float64).T
    return A, B, h, y


def slots_forward(X, row_map, offsets, W13, W2):
    """Per-slot FP64 tensors: X_perm [N,d], h [N,f], Y [N,d]."""
    X = np.asarray(X, np.float64)
    E = offsets.shape[0] - 1
    Xp = X[row_map]
    f = W13.shape[1] // 2
    N = row_map.shape[0]
    h = np.zeros((N, f))
    Y = np.zeros((N, X.shape[1]))
    for e in range(E):
        a, b = int(offsets[e]), int(offsets[e + 1])
        if a == b:
            continue
        _, _, h[a:b], Y[a:b] = expert_forward(Xp[a:b], W13[e], W2[e])
    return Xp, h, Y


def combine(Y, inv_map, w):
    """out_t = sum_j w[t,j] * Y[inv_map[t,j]] in j order (FP64)."""
    Y = np.asarray(Y, np.float64)
    w = np.asarray(w, np.float64)
    T, k = inv_map.shape
    out = np.zeros((T, Y.shape[1]))
    for j in range(k):
        out = out + w[:, j:j + 1] * Y[inv_map[:, j]]
    return out


def layer_forward(X, sel, w, W13, W2):
    """Whole expert part of the layer for a fixed routing: returns dict with
    offsets, row_map, inv_map, Xp, h, Y, out (FP64)."""
    E = W13.shape[0]
    offsets, row_map, inv_map = dispatch_maps(sel, E)
    Xp, h, Y = slots_forward(X, row_map, offsets, W13, W2)
    out = combine(Y, inv_map, w)
    return dict(offsets=offsets, row_map=row_map, inv_map=inv_map, Xp=Xp, h=h, Y=Y, out=out)


def token_outputs(X, tokens, sel, w, W13, W2):
    """out for a subset of tokens only (for spot checks at full size)."""
    X = np.asarray(X, np.float64)
    out = np.zeros((len(tokens), X.shape[1]))
    for i, t in enumerate(tokens):
        for j in range(sel.shape[1]):
            e = int(sel[t, j])
            _, _, _, y = expert_forward(X[t:t + 1], W13[e], W2[e])
            out[i] += float(w[t, j]) * y[0]
    return out
