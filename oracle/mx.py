"""OCP Microscaling (MX) block formats -- TEST INFRASTRUCTURE ONLY.

The paper defines no low-precision format; this module follows the
published OCP Microscaling Formats (MX) v1.0 specification, reading stated
here.  An MX block is 32 consecutive elements along the reduction dimension
sharing one scale X = 2^s stored as an E8M0 byte (s + 127); each element is
a code of a small floating-point format:

    format  sign/exp/mant  bias  largest normal  emax   subnormals  specials
    e4m3    1/4/3          7     448             8      yes         NaN only
    e2m3    1/2/3          1     7.5             2      yes         none
    e3m2    1/3/2          3     28              4      yes         none
    e2m1    1/2/1          1     6               2      yes         none

Quantisation of one block (the specification's conversion, reading):
  amax = max |x|; amax = 0 gives s = 0 (X = 1) and every code +0;
  otherwise s = floor(log2(amax)) - emax, clamped to [-127, 127];
  code_i = the element value nearest to x_i / X, ties to the even
  mantissa, magnitudes above the largest normal saturated to it (so the
  block's largest element never overflows: x / X < 2^(emax + 1)).
Decoding: value = decode(code) * X.  Products of two MX operands are
sum over blocks of X_a X_b sum_i decode(a_i) decode(b_i) -- exact in FP64.

Bit packing in memory (reading): e4m3 one code per byte; e2m1 two codes per
byte, the lower K index in the low nibble; e2m3 / e3m2 per 32-code block
24 bytes holding code i at bits 6i .. 6i+5 of the block's little-endian
bit string, then 8 zero bytes (32 bytes per block, so a block starts on a
32-byte boundary like the e4m3 rows).

Parity unpinned by the paper (it defines none of this); pinned in the tests
by an exhaustive decode of every code against the specification's value
tables, round-to-nearest-even midpoints, saturation, and block scales
against the specification's floor(log2) rule.
"""
from __future__ import annotations

import numpy as np

BLOCK = 32

# name -> (exponent bits, mantissa bits, bias, emax, has NaN code)
FORMATS = {
    "e4m3": (4, 3, 7, 8, True),
    "e2m3": (2, 3, 1, 2, False),
    "e3m2": (3, 2, 3, 4, False),
    "e2m1": (2, 1, 1, 2, False),
}
# the hardware format selectors of the scaled matrix instructions
HW_CODE = {"e4m3": 0, "e2m3": 2, "e3m2": 3, "e2m1": 4}
BITS = {"e4m3": 8, "e2m3": 6, "e3m2": 6, "e2m1": 4}


def decode(codes, fmt: str) -> np.ndarray:
    """FP64 values of element codes (unsigned ints below 2^bits)."""
    eb, mb, bias, _, nan = FORMATS[fmt]
    c = np.asarray(codes, dtype=np.int64)
    sign = np.where((c >> (eb + mb)) & 1, -1.0, 1.0)
    e = (c >> mb) & ((1 << eb) - 1)
    m = c & ((1 << mb) - 1)
    frac = m / float(1 << mb)
    val = np.where(e == 0, frac * 2.0 ** (1 - bias), (1.0 + frac) * np.exp2(e - bias))
    val = sign * val
    if nan:
        val = np.where((e == (1 << eb) - 1) & (m == (1 << mb) - 1), np.nan, val)
    return val


def _positive_table(fmt: str):
    """(values ascending, codes) of every finite non-negative code."""
    eb, mb, _, _, _ = FORMATS[fmt]
    codes = np.arange(1 << (eb + mb))
    vals = decode(codes, fmt)
    ok = np.isfinite(vals)
    order = np.argsort(vals[ok], kind="stable")
    return vals[ok][order], codes[ok][order]


def max_normal(fmt: str) -> float:
    return float(_positive_table(fmt)[0][-1])


def encode(x, fmt: str) -> np.ndarray:
    """Nearest code to each value (FP64), ties to the code with an even
    mantissa, magnitudes beyond the largest normal saturated; -0 and values
    that round to zero keep their sign."""
    eb, mb, _, _, _ = FORMATS[fmt]
    vals, codes = _positive_table(fmt)
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), vals[-1])
    hi = np.clip(np.searchsorted(vals, a, side="left"), 0, len(vals) - 1)
    lo = np.clip(hi - 1, 0, len(vals) - 1)
    dlo, dhi = a - vals[lo], vals[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ((codes[hi] & 1) == 0) & (hi != lo))
    mag = np.where(pick_hi, codes[hi], codes[lo])
    mag = np.where(a == vals[hi], codes[hi], mag)
    sign = np.signbit(x).astype(np.int64) << (eb + mb)
    return (mag | sign).astype(np.uint8)


def block_exponents(x, fmt: str) -> np.ndarray:
    """Shared exponent s of each 32-element block of the rows of x [R, K]."""
    x = np.asarray(x, dtype=np.float64)
    R, K = x.shape
    amax = np.abs(x.reshape(R, K // BLOCK, BLOCK)).max(axis=2)
    _, ex = np.frexp(np.where(amax > 0, amax, 1.0))
    s = (ex - 1) - FORMATS[fmt][3]
    return np.where(amax > 0, np.clip(s, -127, 127), 0).astype(np.int64)


def quantize(x, fmt: str):
    """MX quantisation of the rows of x [R, K] (K % 32 == 0) in 1 x 32 blocks.
    Returns (codes uint8 [R, K], one code per byte; scale bytes uint8
    [R, K / 32] = s + 127)."""
    x = np.asarray(x, dtype=np.float64)
    R, K = x.shape
    s = block_exponents(x, fmt)
    X = np.repeat(np.exp2(s.astype(np.float64)), BLOCK, axis=1)
    return encode(x / X, fmt), (s + 127).astype(np.uint8)


def dequantize(codes, scale_bytes, fmt: str) -> np.ndarray:
    s = np.asarray(scale_bytes, dtype=np.int64) - 127
    return decode(codes, fmt) * np.repeat(np.exp2(s.astype(np.float64)), BLOCK, axis=-1)


def pack(codes, fmt: str) -> np.ndarray:
    """Memory layout of a code matrix [R, K] (see the module header)."""
    c = np.asarray(codes, dtype=np.uint8)
    R, K = c.shape
    if BITS[fmt] == 8:
        return c.copy()
    if BITS[fmt] == 4:
        return (c[:, 0::2] | (c[:, 1::2] << 4)).astype(np.uint8)
    g = c.reshape(R, K // 4, 4).astype(np.uint32)
    word = g[..., 0] | (g[..., 1] << 6) | (g[..., 2] << 12) | (g[..., 3] << 18)
    dense = np.stack([word & 0xFF, (word >> 8) & 0xFF, (word >> 16) & 0xFF], axis=-1)
    dense = dense.reshape(R, K // BLOCK, 24)
    out = np.zeros((R, K // BLOCK, 32), np.uint8)
    out[..., :24] = dense
    return out.reshape(R, K)


def unpack(packed, K: int, fmt: str) -> np.ndarray:
    p = np.asarray(packed, dtype=np.uint8)
    R = p.shape[0]
    if BITS[fmt] == 8:
        return p[:, :K].copy()
    if BITS[fmt] == 4:
        out = np.empty((R, K), np.uint8)
        out[:, 0::2] = p & 0xF
        out[:, 1::2] = p >> 4
        return out
    b = p.reshape(R, K // BLOCK, 32)[..., :24].reshape(R, K // 4, 3).astype(np.uint32)
    word = b[..., 0] | (b[..., 1] << 8) | (b[..., 2] << 16)
    out = np.stack([(word >> (6 * i)) & 0x3F for i in range(4)], axis=-1)
    return out.reshape(R, K).astype(np.uint8)


def row_bytes(K: int, fmt: str) -> int:
    return K // 2 if BITS[fmt] == 4 else K


def slots_forward(X, row_map, offsets, W13q, W13s, W2q, W2s, fmt: str):
    """MX expert path over the slots (reading; the paper defines none).

    X [T,d] holds the stored token values (BF16 values as float64); they
    are MX-quantised once per token (1 x 32 blocks along d) and gathered
    into slot order.  W13q / W13s: per-expert codes [E, 2f, d] (one code per
    byte) and scale bytes [E, 2f, d/32]; W2q / W2s likewise [E, d, f] and
    [E, d, f/32].  Per expert: [A|B] = Xd W13d^T with dequantised operands
    (exact in FP64: the products are the block sums of the scaled codes),
    h = silu(A) * B rounded to BF16 and MX-quantised in 1 x 32 blocks along
    f, Y = hd W2d^T.

    Returns dict of Xq, Xs (per-token codes / scale bytes), h (BF16 values
    [N,f]), hq, hs, Y [N,d] (FP64)."""
    import scipy.special

    from .fp8 import round_bf16

    X = np.asarray(X, np.float32).astype(np.float64)
    Xq, Xs = quantize(X, fmt)
    Xd = dequantize(Xq, Xs, fmt)[row_map]
    E = offsets.shape[0] - 1
    f = W13q.shape[1] // 2
    N, d = Xd.shape
    h = np.zeros((N, f))
    for e in range(E):
        a, b = int(offsets[e]), int(offsets[e + 1])
        if a == b:
            continue
        W = dequantize(W13q[e], W13s[e], fmt)
        A = Xd[a:b] @ W[:f].T
        B = Xd[a:b] @ W[f:].T
        h[a:b] = round_bf16(A * scipy.special.expit(A) * B)
    hq, hs = quantize(h, fmt)
    hd = dequantize(hq, hs, fmt)
    Y = np.zeros((N, d))
    for e in range(E):
        a, b = int(offsets[e]), int(offsets[e + 1])
        if a == b:
            continue
        Y[a:b] = hd[a:b] @ dequantize(W2q[e], W2s[e], fmt).T
    return dict(Xq=Xq, Xs=Xs, h=h, hq=hq, hs=hs, Y=Y)


def quantize_experts(W, fmt: str):
    """Per-expert MX quantisation of W [E, R, C] along C: (codes [E,R,C],
    scale bytes [E, R, C/32])."""
    W = np.asarray(W, np.float64)
    qs = [quantize(W[e], fmt) for e in range(W.shape[0])]
    return np.stack([q for q, _ in qs]), np.stack([s for _, s in qs])
