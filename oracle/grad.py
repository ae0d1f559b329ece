"""FP64 backward of the layer with the routing held fixed -- TEST INFRASTRUCTURE ONLY.

Parity unpinned by the paper (it defines no expert layer).  The layer is
piecewise smooth: the chosen experts (and the prices that chose them) are
constants of each piece, so no gradient flows into the prices or through
the selection.  On a piece:

  s = X W_r^T + b_r;  w_t = softmax over the chosen experts of s_t;
  y_tj = expert e_j applied to x_t;  out_t = sum_j w_tj y_tj.

Backward, for an upstream dOut:
  dw_tj  = <dOut_t, y_tj>
  ds_te  = w_tj (dw_tj - sum_i w_ti dw_ti) if e = e_j, else 0
  dy_tj  = w_tj dOut_t
  dh     = dy W2_e;  dW2_e += dy^T h
  dA     = dh * B * silu'(A),  dB = dh * silu(A),  silu'(z) = g + z g (1-g),
           g = sigmoid(z)
  dx_tj  = dA W1_e + dB W3_e;  dW1_e += dA^T x;  dW3_e += dB^T x
  dX_t   = sum_j dx_tj + ds_t W_r;  dW_r = ds^T X;  db_r = sum_t ds_t.
"""
from __future__ import annotations

import numpy as np
import scipy.special

from . import ffn, routing


def layer_backward(X, Wr, br, W13, W2, sel, dOut):
    """Gradients of sum(out * dOut) for the fixed routing ``sel``.

    Returns dict(dX, dWr, dbr, dW13, dW2, dw [T,k], ds [T,E], and the
    per-slot tensors G (= dOut gathered to slots), dXp)."""
    X = np.asarray(X, np.float64)
    Wr = np.asarray(Wr, np.float64)
    W13 = np.asarray(W13, np.float64)
    W2 = np.asarray(W2, np.float64)
    dOut = np.asarray(dOut, np.float64)
    T, d = X.shape
    E = W13.shape[0]
    f = W13.shape[1] // 2
    k = sel.shape[1]
    s = routing.logits_fp64(X, Wr, br)
    w = routing.gate_weights(s, sel)
    offsets, row_map, inv_map = ffn.dispatch_maps(sel, E)
    N = T * k
    Xp = X[row_map]
    # slot-order gate weight and upstream gradient
    slot_t = row_map
    slot_j = np.empty(N, dtype=np.int64)
    for j in range(k):
        slot_j[inv_map[:, j]] = j
    w_slot = w[slot_t, slot_j]
    G = dOut[slot_t]
    dXp = np.zeros((N, d))
    dW13 = np.zeros_like(W13)
    dW2 = np.zeros_like(W2)
    dw_slot = np.zeros(N)
    for e in range(E):
        a, b = int(offsets[e]), int(offsets[e + 1])
        if a == b:
            continue
        x = Xp[a:b]
        A = x @ W13[e, :f].T
        B = x @ W13[e, f:].T
        g = scipy.special.expit(A)
        sA = A * g
        h = sA * B
        y = h @ W2[e].T
        dw_slot[a:b] = np.sum(G[a:b] * y, axis=1)
        dy = w_slot[a:b, None] * G[a:b]
        dh = dy @ W2[e]
        dW2[e] = dy.T @ h
        dA = dh * B * (g + A * g * (1.0 - g))
        dB = dh * sA
        dXp[a:b] = dA @ W13[e, :f] + dB @ W13[e, f:]
        dW13[e, :f] = dA.T @ x
        dW13[e, f:] = dB.T @ x
    dw = dw_slot[inv_map]
    dsel = w * (dw - np.sum(w * dw, axis=1, keepdims=True))
    ds = np.zeros((T, E))
    ds[np.arange(T)[:, None], sel] = dsel
    dX = np.zeros((T, d))
    for j in range(k):
        dX = dX + dXp[inv_map[:, j]]
    dX = dX + ds @ Wr
    dWr = ds.T @ X
    dbr = ds.sum(axis=0)
    return dict(dX=dX, dWr=dWr, dbr=dbr, dW13=dW13, dW2=dW2, dw=dw, ds=ds, G=G, dXp=dXp,
                w=w, offsets=offsets, row_map=row_map, inv_map=inv_map)


def layer_loss(X, Wr, br, W13, W2, sel, dOut) -> float:
    """sum(out * dOut) for the fixed routing (FP64), for finite differences."""
    s = routing.logits_fp64(X, Wr, br)
    w = routing.gate_weights(s, sel)
    out = ffn.layer_forward(X, sel, w, W13, W2)["out"]
    return float(np.sum(out * np.asarray(dOut, np.float64)))
