"""Pins of the oracle's OCP Microscaling (MX) formats (oracle/mx.py)
against values fixed by the specification and by independent routines."""
import numpy as np
import pytest
import torch

from oracle import mx

F32 = np.float32


def test_e2m1_value_table():
    # the eight magnitudes of FP4 E2M1 listed by the specification
    want = [0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0]
    np.testing.assert_array_equal(mx.decode(np.arange(8), "e2m1"), want)
    np.testing.assert_array_equal(mx.decode(np.arange(8, 16), "e2m1"), [-v for v in want])


@pytest.mark.parametrize("fmt,mx_normal,min_sub,min_normal", [
    ("e2m3", 7.5, 0.125, 1.0), ("e3m2", 28.0, 0.0625, 0.25), ("e4m3", 448.0, 2.0 ** -9, 2.0 ** -6),
    ("e2m1", 6.0, 0.5, 1.0)])
def test_format_extremes(fmt, mx_normal, min_sub, min_normal):
    assert mx.max_normal(fmt) == mx_normal
    v = mx.decode(np.arange(1 << mx.BITS[fmt]), fmt)
    pos = np.sort(v[np.isfinite(v) & (v > 0)])
    assert pos[0] == min_sub
    eb, mb = mx.FORMATS[fmt][:2]
    # first normal: exponent field 1, mantissa 0
    assert mx.decode(np.array([1 << mb]), fmt)[0] == min_normal
    # no infinities; e4m3 has NaN only at S.1111.111
    assert not np.any(np.isinf(v))
    assert np.sum(np.isnan(v)) == (2 if fmt == "e4m3" else 0)


def test_e4m3_matches_torch_float8():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().double().numpy()
    got = mx.decode(codes, "e4m3")
    np.testing.assert_array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    np.testing.assert_array_equal(got[ok], ref[ok])
    # encoding: torch's round-to-nearest-even cast on in-range values
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 20000), rng.standard_normal(20000) * 2.0 ** -7,
                        mx.decode(codes[:127], "e4m3") * 1.0000001])
    x = x.astype(F32)
    t = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(mx.encode(x.astype(np.float64), "e4m3"), t)


def test_round_to_nearest_even_and_saturation():
    # e2m1: midpoints go to the even mantissa; beyond 6 saturates
    x = [0.25, 0.75, 1.25, 1.75, 2.5, 3.5, 5.0, 7.0, 100.0, -0.25, -5.0]
    want = [0.0, 1.0, 1.0, 2.0, 2.0, 4.0, 4.0, 6.0, 6.0, -0.0, -4.0]
    got = mx.decode(mx.encode(x, "e2m1"), "e2m1")
    np.testing.assert_array_equal(got, want)
    assert np.signbit(got[9])  # -0.25 rounds to -0
    # e2m3: spacing 0.125 below 2, 0.25 in [2, 4), 0.5 in [4, 7.5]
    x = [0.0625, 0.1875, 2.125, 2.375, 7.25, 7.75, 9.0]
    want = [0.0, 0.25, 2.0, 2.5, 7.0, 7.5, 7.5]
    np.testing.assert_array_equal(mx.decode(mx.encode(x, "e2m3"), "e2m3"), want)
    # e4m3 saturates instead of producing NaN
    np.testing.assert_array_equal(mx.decode(mx.encode([470.0, 1e6, -1e6], "e4m3"), "e4m3"),
                                  [448.0, 448.0, -448.0])


def test_block_scale_rule():
    """s = floor(log2(amax)) - emax per 32-element block (amax 0: s = 0)."""
    x = np.zeros((1, 128))
    x[0, 0] = 6.0      # e2m1 emax 2: floor(log2 6) = 2 -> s = 0
    x[0, 32] = 6.5     # s = 0, 6.5 saturates to 6
    x[0, 64] = 0.3     # floor(log2 0.3) = -2 -> s = -4, 0.3 * 16 = 4.8 -> 4 (nearest)
    q, s = mx.quantize(x, "e2m1")
    np.testing.assert_array_equal(s[0].astype(int) - 127, [0, 0, -4, 0])
    np.testing.assert_array_equal(mx.dequantize(q, s, "e2m1")[0, [0, 32, 64, 96]],
                                  [6.0, 6.0, 0.25, 0.0])
    # e4m3: amax 1.0 -> s = -8, the block maximum lands on 256
    y = np.full((1, 32), 0.5)
    y[0, 7] = -1.0
    q, s = mx.quantize(y, "e4m3")
    assert int(s[0, 0]) - 127 == -8
    assert mx.decode(q[0, 7:8], "e4m3")[0] == -256.0
    # the block's largest element never needs more than the largest normal
    rng = np.random.default_rng(2)
    z = rng.standard_normal((50, 256)) * np.exp(rng.uniform(-20, 20, (50, 1)))
    for fmt in mx.FORMATS:
        qz, sz = mx.quantize(z, fmt)
        sc = np.repeat(np.exp2(sz.astype(np.int64) - 127.0), 32, axis=1)
        ratio = np.abs(z) / sc
        assert ratio.max() < 2.0 ** (mx.FORMATS[fmt][3] + 1)
        # every element within half a grid step of its code (no saturation
        # happens except above the largest normal)
        err = np.abs(mx.dequantize(qz, sz, fmt) - z) / sc
        top = mx.max_normal(fmt)
        assert np.all((err <= top * 2.0 ** -(mx.FORMATS[fmt][1] + 1) + 1e-12) | (ratio > top))


def test_pack_layouts():
    # e2m1: two codes per byte, lower index in the low nibble
    c = np.array([[1, 2, 3, 4, 15, 0, 7, 8]], np.uint8)
    np.testing.assert_array_equal(mx.pack(c, "e2m1"), [[0x21, 0x43, 0x0F, 0x87]])
    # e2m3: code i at bits 6i..6i+5 of the block's little-endian bit string,
    # 24 bytes, then 8 zero bytes
    c = np.zeros((1, 32), np.uint8)
    c[0, :4] = [0x01, 0x02, 0x03, 0x3F]
    c[0, 31] = 0x2A
    word = 0x01 | (0x02 << 6) | (0x03 << 12) | (0x3F << 18)
    want = np.zeros(32, np.uint8)
    want[:3] = [word & 0xFF, (word >> 8) & 0xFF, word >> 16]
    want[23] = 0x2A << 2  # code 31 at bits 186..191: the top six bits of byte 23
    np.testing.assert_array_equal(mx.pack(c, "e2m3")[0], want)
    rng = np.random.default_rng(3)
    for fmt in mx.FORMATS:
        codes = rng.integers(0, 1 << mx.BITS[fmt], (7, 64)).astype(np.uint8)
        p = mx.pack(codes, fmt)
        assert p.shape == (7, mx.row_bytes(64, fmt))
        np.testing.assert_array_equal(mx.unpack(p, 64, fmt), codes)


def test_block_product_is_exact_integer_arithmetic():
    """Dequantised products equal the block sums X_a X_b sum_i qa_i qb_i
    computed in integers (e2m1 values are halves of integers)."""
    rng = np.random.default_rng(4)
    a = rng.standard_normal((5, 96))
    b = rng.standard_normal((3, 96))
    qa, sa = mx.quantize(a, "e2m1")
    qb, sb = mx.quantize(b, "e2m1")
    got = mx.dequantize(qa, sa, "e2m1") @ mx.dequantize(qb, sb, "e2m1").T
    ia = np.rint(mx.decode(qa, "e2m1") * 2).astype(np.int64)
    ib = np.rint(mx.decode(qb, "e2m1") * 2).astype(np.int64)
    want = np.zeros((5, 3))
    for blk in range(3):
        sl = slice(32 * blk, 32 * blk + 32)
        part = ia[:, sl] @ ib[:, sl].T  # exact
        scale = np.exp2((sa[:, blk].astype(np.int64)[:, None] - 127)
                        + (sb[:, blk].astype(np.int64)[None, :] - 127) - 2.0)
        want += part * scale
    np.testing.assert_array_equal(got, want)
