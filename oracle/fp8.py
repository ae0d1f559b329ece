"""OCP FP8 e4m3 emulator and per-128-block quantisation -- TEST INFRASTRUCTURE ONLY.

Format (OCP 8-bit floating point, E4M3 variant): 1 sign bit, 4 exponent bits
(bias 7), 3 mantissa bits; exponent field 0 encodes subnormals m/8 * 2^-6;
the all-ones exponent with mantissa 7 is NaN; there is no infinity, so the
largest finite magnitude is 1.75 * 2^8 = 448.

Encoding rule used by the layer: round to nearest, ties to even mantissa,
then saturate to +-448.

Block quantisation (reading; the paper defines none): for a block of
values (1 x 128 for activations, 128 x 128 for weights) with FP32 amax:
if amax == 0 the scale is 1 and every code is 0; otherwise
inv = fl32(448 / amax), q = encode(fl32(x * inv)), scale = fl32(amax / 448).
A block's dequantised value is decode(q) * scale; a matrix product over a
128-wide K block is accumulated as sum(qa * qb) * sa * sb in FP32.
"""
from __future__ import annotations

import numpy as np
import scipy.special

F32 = np.float32
FP8_MAX = 448.0


def decode(codes: np.ndarray) -> np.ndarray:
    """float64 value of each e4m3 code (NaN for 0x7F / 0xFF)."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    sign = np.where(c >> 7, -1.0, 1.0)
    ex = (c >> 3) & 15
    man = c & 7
    sub = man / 8.0 * 2.0 ** -6
    nrm = (1.0 + man / 8.0) * np.exp2(ex - 7.0)
    val = sign * np.where(ex == 0, sub, nrm)
    return np.where((ex == 15) & (man == 7), np.nan, val)


_TABLE = decode(np.arange(256, dtype=np.uint8))


def round_rne_sat(x: np.ndarray) -> np.ndarray:
    """Nearest e4m3 value (ties to even mantissa), saturated to +-448; float64."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    m, ex = np.frexp(np.where(a > 0, a, 1.0))  # a = m * 2^ex, m in [0.5, 1)
    e = ex - 1  # a in [2^e, 2^(e+1))
    quantum = np.where(a >= 2.0 ** -6, np.exp2(e - 3.0), 2.0 ** -9)
    r = np.rint(a / quantum) * quantum  # rint rounds half to even
    r = np.minimum(r, FP8_MAX)
    return np.where(a > 0, np.sign(x) * r, 0.0 * x)


def encode(x: np.ndarray) -> np.ndarray:
    """uint8 e4m3 codes of round_rne_sat(x).  Zero keeps its sign."""
    v = round_rne_sat(x)
    pos = np.abs(v)
    # positive codes 0..126 are increasing in value
    idx = np.searchsorted(_TABLE[:127], pos)
    neg = np.signbit(v)
    return (idx.astype(np.uint8) | np.where(neg, 0x80, 0).astype(np.uint8)).astype(np.uint8)


def quantize_blocks(x: np.ndarray, br: int, bc: int):
    """Quantise a float32 matrix [R, Ccols] in br x bc blocks.

    Returns (codes uint8 [R, Ccols], scales float32 [ceil(R/br), Ccols/bc]).
    Ccols must be a multiple of bc; a ragged last row block is allowed."""
    x = np.asarray(x, dtype=F32)
    R, Cc = x.shape
    assert Cc % bc == 0
    nbr = -(-R // br)
    nbc = Cc // bc
    codes = np.zeros((R, Cc), dtype=np.uint8)
    scales = np.ones((nbr, nbc), dtype=F32)
    for i in range(nbr):
        r0, r1 = i * br, min(R, (i + 1) * br)
        blk = x[r0:r1].reshape(r1 - r0, nbc, bc)
        amax = np.max(np.abs(blk), axis=(0, 2)).astype(F32)  # [nbc]
        nz = amax > 0
        inv = np.where(nz, F32(FP8_MAX) / np.where(nz, amax, F32(1)), F32(1)).astype(F32)
        scaled = (blk * inv[None, :, None]).astype(F32)
        q = encode(scaled)
        q = np.where(nz[None, :, None], q, 0).astype(np.uint8)
        codes[r0:r1] = q.reshape(r1 - r0, Cc)
        scales[i] = np.where(nz, (amax / F32(FP8_MAX)).astype(F32), F32(1))
    return codes, scales


def dequantize_blocks(codes: np.ndarray, scales: np.ndarray, br: int, bc: int) -> np.ndarray:
    """float64 values decode(q) * scale of a block-quantised matrix."""
    v = decode(codes)
    R, Cc = codes.shape
    sc = np.repeat(np.repeat(np.asarray(scales, np.float64), br, axis=0)[:R], bc, axis=1)
    return v * sc


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Nearest BF16 value (8 significant bits, ties to even) of float64
    values in BF16's normal range; float64 result."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    _, ex = np.frexp(np.where(a > 0, a, 1.0))
    quantum = np.exp2(ex - 1 - 7.0)
    r = np.rint(a / quantum) * quantum
    return np.where(a > 0, np.sign(x) * r, 0.0 * x)


def slots_forward_fp8(X, row_map, offsets, W13q, W13s, W2q, W2s):
    """FP8 expert path over the slots (reading; the paper defines none).

    X holds the stored token values (float64 of the BF16 activations).
    Tokens are quantised per 1 x 128 block of a row and gathered into
    slot order; weights come quantised per 128 x 128 block (codes and
    scales as quantize_blocks returns them, one expert per leading index).
    Per expert: [A|B] = Xd W13d^T with Xd, W13d the dequantised values
    decode(q) * scale -- exact in FP64, so this product equals the sum over
    128-wide K blocks of (sum qa qb) * sa * sb; h = silu(A) * B is stored
    as BF16 and quantised per 1 x 128 block; Y = hd W2d^T.

    Returns dict of Xq, Xs (token codes / scales, [T,d] / [T,d/128]), h
    (BF16 values, [N,f]), hq, hs, Y [N,d] (FP64)."""
    X = np.asarray(X, np.float32)
    Xq, Xs = quantize_blocks(X, 1, 128)
    Xd = dequantize_blocks(Xq, Xs, 1, 128)[row_map]
    E = offsets.shape[0] - 1
    f = W13q.shape[1] // 2
    N, d = Xd.shape
    h = np.zeros((N, f))
    for e in range(E):
        a, b = int(offsets[e]), int(offsets[e + 1])
        if a == b:
            continue
        W = dequantize_blocks(W13q[e], W13s[e], 128, 128)
        A = Xd[a:b] @ W[:f].T
        B = Xd[a:b] @ W[f:].T
        h[a:b] = round_bf16(A * scipy.special.expit(A) * B)
    hq, hs = quantize_blocks(h.astype(np.float32), 1, 128)
    hd = dequantize_blocks(hq, hs, 1, 128)
    Y = np.zeros((N, d))
    for e in range(E):
        a, b = int(offsets[e]), int(offsets[e + 1])
        if a == b:
            continue
        Y[a:b] = hd[a:b] @ dequantize_blocks(W2q[e], W2s[e], 128, 128).T
    return dict(Xq=Xq, Xs=Xs, h=h, hq=hq, hs=hs, Y=Y)


def quantize_experts(W, br=128, bc=128):
    """Per-expert block quantisation of W [E, R, C]: (codes [E,R,C] uint8,
    scales [E, ceil(R/br), C/bc] float32)."""
    W = np.asarray(W, np.float32)
    qs = [quantize_blocks(W[e], br, bc) for e in range(W.shape[0])]
    return np.stack([q for q, _ in qs]), np.stack([s for _, s in qs])
