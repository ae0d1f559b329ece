"""Host-only checks of the C ABI: the library loads, exports every function
include/moe.h declares, and rejects bad arguments before launching anything."""
import ctypes
import os
import re

import pytest

from paper_2606_17065_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(moe_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = _declared()
    assert "moe_route" in names and "moe_combine" in names
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    bound = set(L.SIGNATURES) | {"moe_strerror"}
    assert _declared() <= bound


def test_strerror_texts():
    assert L.strerror(0) == "ok"
    assert "infeasible" in L.strerror(L.MOE_EINFEASIBLE)
    assert L.strerror(12345) == "unknown status"


def _cfg(**kw):
    base = dict(T=512, d=128, E=8, k=2, d_ff=256, capacity=160, max_iters=50,
                act=L.MOE_F32, w=L.MOE_F32, price_mode=L.MOE_PRICE_ACP)
    base.update(kw)
    return L.make_cfg(**base)


def test_workspace_bytes_and_shape_checks():
    n = L.moe_workspace_bytes(_cfg())
    assert n > 512 * 8 * 4 * 2  # transposed logits and margin keys at least
    with pytest.raises(L.MoEError) as e:
        L.moe_workspace_bytes(_cfg(k=9))
    assert e.value.status == L.MOE_EINFEASIBLE
    with pytest.raises(L.MoEError) as e:
        L.moe_workspace_bytes(_cfg(capacity=127))  # 8*127 < 512*2
    assert e.value.status == L.MOE_EINFEASIBLE
    with pytest.raises(L.MoEError) as e:
        L.moe_workspace_bytes(_cfg(d=100))
    assert e.value.status == L.MOE_EUNSUPPORTED
    with pytest.raises(L.MoEError) as e:
        L.moe_workspace_bytes(_cfg(act=7))
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:
        L.moe_workspace_bytes(_cfg(E=2000, capacity=100))
    assert e.value.status == L.MOE_EUNSUPPORTED


def test_entry_points_reject_bad_arguments_on_the_host():
    cfg = _cfg()
    fake = 1 << 20  # never dereferenced: every call below fails its host checks
    with pytest.raises(L.MoEError) as e:
        L.moe_route(cfg, None, fake, fake, fake, fake, fake, fake, fake, fake, fake, 1 << 30, None)
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:
        L.moe_route(cfg, fake + 4, fake, fake, fake, fake, fake, fake, fake, fake, fake, 1 << 30, None)
    assert e.value.status == L.MOE_EINVAL  # X misaligned
    with pytest.raises(L.MoEError) as e:
        L.moe_route(cfg, fake, fake, fake, fake, fake, fake, fake, fake, fake, fake, 16, None)
    assert e.value.status == L.MOE_EWORKSPACE
    bad = _cfg(price_mode=L.MOE_PRICE_SUBGRAD + 1)
    with pytest.raises(L.MoEError) as e:
        L.moe_route(bad, fake, fake, fake, fake, fake, fake, fake, fake, fake, fake, 1 << 30, None)
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:
        L.moe_dispatch(cfg, fake, fake, fake, fake, fake, fake, None, fake, 0, None)
    assert e.value.status == L.MOE_EWORKSPACE
    with pytest.raises(L.MoEError) as e:
        L.moe_expert_ffn(_cfg(act=L.MOE_F32, w=L.MOE_BF16), fake, None, fake, fake, None, fake,
                         None, fake, fake, 1 << 30, None)
    assert e.value.status == L.MOE_EUNSUPPORTED
    with pytest.raises(L.MoEError) as e:  # FP8 experts need the weight scales
        L.moe_expert_ffn(_cfg(act=L.MOE_BF16, w=L.MOE_FP8E4M3), fake, fake, fake, fake, None, fake,
                         None, fake, fake, 1 << 30, None)
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:  # FP8 dispatch needs the scale output
        L.moe_dispatch(_cfg(w=L.MOE_FP8E4M3), fake, fake, fake, fake, fake, fake, None, fake,
                       1 << 30, None)
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:  # the fused gather is BF16-only
        L.moe_expert_ffn_gather(_cfg(act=L.MOE_F32, w=L.MOE_F32), fake, fake, fake, fake, fake,
                                fake, fake, 1 << 30, None)
    assert e.value.status == L.MOE_EUNSUPPORTED
    with pytest.raises(L.MoEError) as e:  # row_map missing
        L.moe_expert_ffn_gather(_cfg(d=256, act=L.MOE_BF16, w=L.MOE_BF16), fake, None, fake, fake, fake,
                                fake, fake, 1 << 30, None)
    assert e.value.status == L.MOE_EINVAL
    bf = _cfg(d=256, act=L.MOE_BF16, w=L.MOE_BF16)
    with pytest.raises(L.MoEError) as e:  # the saving forward needs the AB output
        L.moe_expert_ffn_gather_save(bf, fake, fake, fake, fake, fake, fake, None, fake, 1 << 30,
                                     None)
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:  # AB misaligned
        L.moe_expert_ffn_gather_save(bf, fake, fake, fake, fake, fake, fake, fake + 8, fake,
                                     1 << 30, None)
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:  # the saved-input backward needs AB
        L.moe_expert_ffn_bwd_saved(bf, fake, fake, fake, fake, fake, fake, None, fake, fake, fake,
                                   L.MOE_F32, fake, 1 << 30, None)
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:  # BF16 only, as the recomputing backward
        L.moe_expert_ffn_bwd_saved(_cfg(), fake, fake, fake, fake, fake, fake, fake, fake, fake,
                                   fake, L.MOE_F32, fake, 1 << 30, None)
    assert e.value.status == L.MOE_EUNSUPPORTED
    with pytest.raises(L.MoEError) as e:
        L.moe_quantize_fp8(4, 100, 1, L.MOE_BF16, fake, fake, fake, None)  # cols % 128
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:
        L.moe_quantize_fp8(4, 128, 2, L.MOE_BF16, fake, fake, fake, None)  # block rows
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:
        L.moe_combine(cfg, None, fake, fake, fake, None)
    assert e.value.status == L.MOE_EINVAL
    with pytest.raises(L.MoEError) as e:
        L.moe_price_update(cfg, fake, fake, fake, fake, 16, None)
    assert e.value.status == L.MOE_EWORKSPACE
    with pytest.raises(L.MoEError) as e:
        L.moe_price_update(cfg, None, fake, fake, fake, 1 << 30, None)
    assert e.value.status == L.MOE_EINVAL


def test_missing_library_fails_loudly():
    """Without libmoe.so the binding raises on first use (no CPU fallback)."""
    import subprocess
    import sys
    code = ("import paper_2606_17065_amd._lib as L\n"
            "L.LIB_PATH = '/nonexistent/libmoe.so'\n"
            "L._lib = None\n"
            "try:\n"
            "    L.moe_workspace_bytes(L.make_cfg(8, 8, 2, 1, 8, 8, 1, L.MOE_F32, L.MOE_F32,"
            " L.MOE_PRICE_ACP))\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    raise SystemExit('no error')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    assert "raised:" in r.stdout and "missing" in r.stdout


def test_noalloc_dispatch_rejects_oversized_counts_on_the_host():
    """The fixed scratch of moe_dispatch_noalloc holds 4 MiB of counts:
    ceil(T / 256) * E int32 above that is refused before any launch."""
    fake = 1 << 20
    T, E, k = 256 * 1025, 1024, 2
    big = L.make_cfg(T, 128, E, k, 128, (T * k + E - 1) // E + 1, 50, L.MOE_BF16, L.MOE_BF16,
                     L.MOE_PRICE_ACP)
    with pytest.raises(L.MoEError) as e:
        L.moe_dispatch_noalloc(big, fake, fake, fake, fake, fake, None, None, None)
    assert e.value.status == L.MOE_EUNSUPPORTED


@pytest.mark.parametrize("stages", [-1, 9])
def test_price_stages_out_of_range_rejected(stages):
    cfg = _cfg()
    cfg.price_stages = stages
    with pytest.raises(L.MoEError) as e:
        L.moe_workspace_bytes(cfg)
    assert e.value.status == L.MOE_EINVAL
