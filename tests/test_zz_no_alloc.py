"""moe_dispatch_noalloc (fixed device scratch, no workspace argument) against
moe_dispatch with a caller workspace, through the C ABI: bit-identical maps,
permuted rows and FP8 codes / scales on two calls in a row, the second with
fewer tokens (so it runs on counts the first call left in the array)."""
import numpy as np
import pytest
import torch

from paper_2606_17065_amd import _lib as L

pytestmark = pytest.mark.gpu


def _routing(T, E, k, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    # k distinct experts per token, skewed towards low expert indices
    pop = 1.0 / np.arange(1, E + 1) ** 1.2
    pop /= pop.sum()
    idx = np.stack([rng.choice(E, size=k, replace=False, p=pop) for _ in range(T)])
    return idx.astype(np.int32)


def _run(cfg, X, idx, noalloc):
    dev = X.device
    T, E, k, d = cfg.T, cfg.E, cfg.k, cfg.d
    fp8 = cfg.w == L.MOE_FP8E4M3
    o = dict(offsets=torch.full((E + 1,), -7, dtype=torch.int32, device=dev),
             row_map=torch.full((T * k,), -7, dtype=torch.int32, device=dev),
             inv_map=torch.full((T, k), -7, dtype=torch.int32, device=dev),
             X_perm=torch.zeros(T * k, d, dtype=torch.uint8 if fp8 else X.dtype, device=dev),
             X_perm_scale=(torch.zeros(T * k, d // 128, dtype=torch.float32, device=dev)
                           if fp8 else None))
    stream = torch.cuda.current_stream().cuda_stream
    sc = None if o["X_perm_scale"] is None else o["X_perm_scale"].data_ptr()
    args = (cfg, X.data_ptr(), idx.data_ptr(), o["offsets"].data_ptr(), o["row_map"].data_ptr(),
            o["inv_map"].data_ptr(), o["X_perm"].data_ptr(), sc)
    if noalloc:
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        L.moe_dispatch_noalloc(*args, stream)
        torch.cuda.synchronize()
        o["free_delta"] = torch.cuda.mem_get_info()[0] - free0
    else:
        n = max(L.moe_workspace_bytes(cfg), 256)
        ws = torch.empty(n, dtype=torch.uint8, device=dev)
        L.moe_dispatch(*args, ws.data_ptr(), n, stream)
        torch.cuda.synchronize()
    return o


@pytest.mark.parametrize("w", [L.MOE_BF16, L.MOE_FP8E4M3])
def test_noalloc_dispatch_matches_workspace_dispatch(w):
    for call, (T, E, k, d) in enumerate([(5000, 64, 8, 256), (777, 64, 8, 256)]):
        cfg = L.make_cfg(T, d, E, k, 256, (5 * T * k + 4 * E - 1) // (4 * E), 50, L.MOE_BF16, w,
                         L.MOE_PRICE_ACP)
        gen = torch.Generator().manual_seed(11 + call)
        X = torch.randn(T, d, generator=gen).to(torch.bfloat16).cuda()
        idx = torch.from_numpy(_routing(T, E, k, 21 + call)).cuda()
        ref = _run(cfg, X, idx, False)
        got = _run(cfg, X, idx, True)
        if call > 0:  # after the first call's one-time address lookup
            assert got["free_delta"] == 0, f"device memory changed by {got['free_delta']}"
        for name in ("offsets", "row_map", "inv_map", "X_perm", "X_perm_scale"):
            if ref[name] is None:
                continue
            a, b = got[name].cpu(), ref[name].cpu()
            if a.dtype == torch.bfloat16:  # compare the stored bit patterns
                a, b = a.view(torch.int16), b.view(torch.int16)
            a, b = a.numpy(), b.numpy()
            if a.dtype == np.float32:
                a, b = a.view(np.uint32), b.view(np.uint32)
            np.testing.assert_array_equal(a, b, err_msg=f"call {call}: {name}")
        # the maps are a valid stable sort of the slots by expert
        off = got["offsets"].cpu().numpy()
        assert off[0] == 0 and off[-1] == T * k and np.all(np.diff(off) >= 0)
