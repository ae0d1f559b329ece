"""GPU parity of the learned-price path (logit statistics, price network,
its loss, backward and Adam, routing from given logits, the certificate)
against the CPU oracle, through the C ABI.

Tolerances (FP32 kernels against FP64 definitions):
  features      |gpu - ref| <= 2e-6 * max(1, |ref|): FP64 sums rounded to
                FP32 once; the GPU's margins are FP32-rounded differences,
                the oracle's exact, which moves a quantile by <= 1 ulp
  network       p_hat and the loss: rel <= 1e-5 (FP32 dot products of
                length <= 256); gradients: rel. Frobenius <= 2e-5 per block
  Adam          rtol 1e-6 after three steps
  certificate   primal and dual: rel <= 1e-12 (FP64 sums of the same FP32
                values in another order)
Routing from given logits (any price mode, learned prices included) must be
bit-identical to the FP32 replica given the same logits and p_hat.
"""
import numpy as np
import pytest
import torch

from oracle import mlp as M
from oracle import routing as R
from paper_2606_17065_amd import _lib as L
from paper_2606_17065_amd import price as P
from paper_2606_17065_amd import synth

from _helpers import assert_route_matches, rel_fro, replica_route

pytestmark = pytest.mark.gpu

F32 = np.float32


def _cfg(T, E, k, C=None, mode=L.MOE_PRICE_ACP, gamma=0.9, max_iters=50):
    C = synth.capacity(T, k, E) if C is None else C
    return L.make_cfg(T, 8, E, k, 1, C, max_iters, L.MOE_F32, L.MOE_F32, mode, gamma)


def _logits(T, E, seed, s_z=1.2, scale=0.64):
    s = synth.make_logits(T, E, s_z, seed, scale)
    return s, torch.from_numpy(s).cuda()


# (T, E, k, capacity or None, seed): ragged tiles, E not a multiple of 64,
# k = 1 and k = E - 1, T <= C (quantile = column minimum), a wide batch
STATS_CASES = [(1000, 64, 8, None, 51), (333, 40, 3, None, 52), (50, 5, 4, None, 53),
               (777, 100, 1, None, 54), (4100, 256, 8, None, 55), (200, 17, 16, 200, 56),
               (65, 3, 2, 70, 57)]


@pytest.mark.parametrize("tied", [False, True])
@pytest.mark.parametrize("T,E,k,C,seed", STATS_CASES)
def test_logit_stats_match_oracle(T, E, k, C, seed, tied):
    """tied: logits on a 0.25 grid, so the plain top-k behind f4 meets equal
    keys (broken towards the lower expert)."""
    s, sd = _logits(T, E, seed)
    if tied:
        # rounding also leaves -0.0 next to +0.0: the key order ranks it lower
        s = (np.round(s * 4.0) / 4.0).astype(np.float32)
        sd = torch.from_numpy(s).cuda()
    cfg = _cfg(T, E, k, C)
    feats, sigma = P.logit_stats(cfg, sd)
    torch.cuda.synchronize()
    ref = M.features(s, k, cfg.capacity)
    got = feats.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 2e-6, (err.max(), np.unravel_index(err.argmax(), err.shape))
    # the plain top-k loads behind f4 are integers and must agree exactly
    np.testing.assert_array_equal(np.rint(got[:, 4] * cfg.capacity),
                                  np.rint(ref[:, 4] * cfg.capacity))
    assert abs(float(sigma.item()) - s.astype(np.float64).std()) <= 1e-6 * s.std()


# batches longer than 16384 tokens: the statistics' per-expert selection
# keeps 64 keys per lane up to 65536 tokens and streams the column beyond;
# the fwd+bwd (32768 x 128) and FP8 (65536 x 64) workload shapes, the
# learned-price workload's widest batches (E = 256) and a batch past 65536
LONG_STATS_CASES = [(32768, 128, 8, 1.3, 61), (65536, 64, 8, 1.2, 62), (40001, 256, 8, 1.5, 63),
                    (65536, 256, 8, 1.0, 64), (70001, 64, 8, 1.2, 65)]


@pytest.mark.parametrize("T,E,k,s_z,seed", LONG_STATS_CASES)
def test_logit_stats_match_oracle_long_batches(T, E, k, s_z, seed):
    s, sd = _logits(T, E, seed, s_z)
    cfg = _cfg(T, E, k)
    feats, sigma = P.logit_stats(cfg, sd)
    torch.cuda.synchronize()
    ref = M.features(s, k, cfg.capacity)
    got = feats.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 2e-6, (err.max(), np.unravel_index(err.argmax(), err.shape))
    np.testing.assert_array_equal(np.rint(got[:, 4] * cfg.capacity),
                                  np.rint(ref[:, 4] * cfg.capacity))


def test_logit_stats_rejects_bad_shapes():
    s, sd = _logits(10, 4, 1)
    with pytest.raises(L.MoEError) as e:
        P.logit_stats(_cfg(10, 4, 4, 10), sd)  # k == E: no (k+1)-th score
    assert e.value.status == L.MOE_EUNSUPPORTED
    cfg = _cfg(0, 4, 2, 0)
    with pytest.raises(L.MoEError) as e:
        L.moe_logit_stats(cfg, 0, sd.data_ptr(), 0, sd.data_ptr(), 1 << 20, 0)
    assert e.value.status == L.MOE_EINVAL


def _feature_rows(R_, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((R_, 8)).astype(F32)


def test_mlp_forward_matches_oracle():
    theta = M.init_params(3)
    F = _feature_rows(300, 4)
    params = torch.from_numpy(theta).cuda()
    sigma = torch.tensor([1.7], dtype=torch.float32, device="cuda")
    phat, acts = P.mlp_forward(params, torch.from_numpy(F).cuda(), sigma)
    torch.cuda.synchronize()
    z, _ = M.forward(theta.astype(np.float64), F.astype(np.float64))
    ref = np.float64(F32(1.7)) * M.softplus(z)
    got = phat.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    nz = acts[4 * 256 * 300:].cpu().numpy()
    assert np.abs(nz - z).max() <= 1e-5 * max(1.0, np.abs(z).max())


@pytest.mark.parametrize("rows", [1, 300, 1100])
def test_mlp_loss_and_gradient_match_oracle(rows):
    theta = M.init_params(5 + rows)
    F = _feature_rows(rows, 6 + rows)
    y = np.abs(np.random.Generator(np.random.PCG64(rows)).standard_normal(rows)).astype(F32)
    params = torch.from_numpy(theta).cuda()
    Fd = torch.from_numpy(F).cuda()
    phat, acts = P.mlp_forward(params, Fd)
    loss, dprice = P.mse(phat, torch.from_numpy(y).cuda())
    grads = P.mlp_backward(params, Fd, acts, dprice)
    torch.cuda.synchronize()
    ref_loss, ref_g = M.loss_and_grad(theta.astype(np.float64), F.astype(np.float64), y)
    assert abs(float(loss.item()) - ref_loss) <= 1e-5 * abs(ref_loss)
    g = grads.cpu().numpy()
    o = 0
    for name, shp in M.SIZES:
        n = int(np.prod(shp))
        assert rel_fro(g[o:o + n], ref_g[o:o + n]) <= 2e-5, name
        o += n


def test_mse_groups_divide_by_their_sigma():
    E, B = 7, 5
    rng = np.random.Generator(np.random.PCG64(9))
    ph = rng.standard_normal(E * B).astype(F32)
    tg = rng.uniform(0, 3, E * B).astype(F32)
    sg = rng.uniform(0.5, 2, B).astype(F32)
    loss, dp = P.mse(torch.from_numpy(ph).cuda(), torch.from_numpy(tg).cuda(),
                     torch.from_numpy(sg).cuda(), group=E)
    torch.cuda.synchronize()
    y = tg.astype(np.float64) / np.repeat(sg.astype(np.float64), E)
    r = ph - y
    assert abs(float(loss.item()) - np.mean(r * r)) <= 1e-6 * np.mean(r * r)
    np.testing.assert_allclose(dp.cpu().numpy(), 2 * r / (E * B), rtol=1e-5, atol=1e-8)


def test_adam_matches_oracle():
    n = M.N_PARAMS
    rng = np.random.Generator(np.random.PCG64(11))
    theta = M.init_params(12)
    p = torch.from_numpy(theta.copy()).cuda()
    opt = P.Adam(p, lr=1e-2)
    th, m, v = theta.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 4):
        g = (rng.standard_normal(n) * 10.0 ** rng.uniform(-4, 0, n)).astype(F32)
        opt.step(torch.from_numpy(g).cuda())
        th, m, v = M.adam_step(th, g.astype(np.float64), m, v, step, 1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(p.cpu().numpy(), th, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("mode", [L.MOE_PRICE_ACP, L.MOE_PRICE_NONE])
def test_route_logits_bit_exact(mode):
    s, sd = _logits(3001, 48, 61)
    cfg = _cfg(3001, 48, 6, mode=mode)
    r = P.route_logits(cfg, sd)
    torch.cuda.synchronize()
    ref = replica_route(cfg, s)
    if mode == L.MOE_PRICE_ACP:
        assert ref["iters"] > 0
    assert_route_matches(cfg, r, ref)


# shapes at the limits of the ranking kernel: more than 64 experts per
# wavefront range (logits streamed in chunks, E = 300 and the maximum
# E = 1024), the top-17 lists (k = 12 and the maximum k = 16), and k = 1.
# The raised prices make price-adjusted scores of different experts equal
# (several experts' prices sit on the same token's margin), and these
# shapes were the first to show a tie broken against the lower expert.
@pytest.mark.parametrize("T,E,k,seed", [(1500, 300, 12, 81), (700, 1024, 16, 82),
                                        (900, 8, 1, 83)])
def test_route_logits_bit_exact_at_shape_limits(T, E, k, seed):
    s, sd = _logits(T, E, seed)
    cfg = _cfg(T, E, k)
    r = P.route_logits(cfg, sd)
    torch.cuda.synchronize()
    ref = replica_route(cfg, s)
    assert ref["iters"] > 0
    assert_route_matches(cfg, r, ref)


# logits on a grid of 0.25: exact ties between experts everywhere, in the
# register-cached ranking (E = 64: 8 experts per wavefront range; E = 200:
# 25) and the chunked one (E = 600: 75 experts per range, more than the
# 64 a wavefront keeps in registers)
@pytest.mark.parametrize("T,E,k,seed", [(1000, 64, 8, 84), (600, 200, 6, 85),
                                        (500, 600, 6, 86)])
def test_route_logits_bit_exact_with_tied_logits(T, E, k, seed):
    s = (np.round(synth.make_logits(T, E, 1.2, seed) * 4.0) / 4.0).astype(np.float32)
    sd = torch.from_numpy(s).cuda()
    cfg = _cfg(T, E, k)
    r = P.route_logits(cfg, sd)
    torch.cuda.synchronize()
    ref = replica_route(cfg, s)
    assert ref["iters"] > 0
    assert_route_matches(cfg, r, ref)


# the capacity repair on logits with exact ties (grid of 0.25): evictions
# and acceptances where equal keys straddle the capacity take the ordered
# path (token order among equal keys), the others decide each token by its
# own key; plain top-k (cap 0), one update, and the subgradient rule
@pytest.mark.parametrize("T,E,k,seed,mode,cap", [
    (1000, 64, 8, 87, L.MOE_PRICE_ACP, 0), (3000, 16, 2, 88, L.MOE_PRICE_ACP, 1),
    (1200, 32, 4, 89, L.MOE_PRICE_SUBGRAD, 3), (700, 24, 3, 90, L.MOE_PRICE_NONE, 0)])
def test_capacity_repair_bit_exact_with_tied_logits(T, E, k, seed, mode, cap):
    s = (np.round(synth.make_logits(T, E, 1.3, seed) * 4.0) / 4.0).astype(np.float32)
    sd = torch.from_numpy(s).cuda()
    cfg = _cfg(T, E, k, mode=mode, max_iters=cap)
    r = P.route_logits(cfg, sd)
    torch.cuda.synchronize()
    ref = replica_route(cfg, s)
    assert ref["status"] == R.OK and ref["enforced"]
    assert_route_matches(cfg, r, ref)
    assert int(r["info"][L.INFO_ROUNDS]) == ref["rounds"]


# every instantiation of the ranking kernel: top-k lists padded to 3, 5, 9
# or 17 entries (k = 2, 4, 8, 10), eight expert ranges for k <= 8 and four
# above, and each register cache of 4, 8, 16, 32 or 64 logits per lane (the
# range size rounded up); T = 450 leaves a ragged last token group
_RANK_E8 = (24, 60, 100, 200, 400)
_RANK_E4 = (16, 30, 60, 120, 240)
RANK_VARIANTS = [(450, E, k, 100 + 10 * i + j)
                 for i, (k, Es) in enumerate(((2, _RANK_E8), (4, _RANK_E8), (8, _RANK_E8),
                                              (10, _RANK_E4)))
                 for j, E in enumerate(Es)]


@pytest.mark.parametrize("T,E,k,seed", RANK_VARIANTS)
def test_route_logits_bit_exact_for_every_ranking_variant(T, E, k, seed):
    s, sd = _logits(T, E, seed)
    cfg = _cfg(T, E, k)
    r = P.route_logits(cfg, sd)
    torch.cuda.synchronize()
    ref = replica_route(cfg, s)
    assert ref["iters"] > 0
    assert_route_matches(cfg, r, ref)


# batches longer than 16384 tokens, where each selection block streams its
# margin column from memory in every radix pass instead of holding it in
# registers: just past the switch, an uneven length, the FP8 workload
# shape (65536 x 64, Zipf 1.2), the fwd+bwd workload shape (32768 x 128,
# Zipf 1.3) and a batch past 65536 tokens
# (logit scale 0.02 * sqrt(d_model): 1.28 at d = 4096, 0.905 at d = 2048)
LONG_ROUTE_CASES = [(16385, 64, 8, 1.2, 0.64, 71), (40000, 64, 8, 1.2, 0.64, 72),
                    (65536, 64, 8, 1.2, 1.28, 73), (32768, 128, 8, 1.3, 0.905, 74),
                    (70001, 32, 4, 1.2, 0.64, 75)]


@pytest.mark.parametrize("T,E,k,s_z,scale,seed", LONG_ROUTE_CASES)
def test_route_logits_bit_exact_long_batches(T, E, k, s_z, scale, seed):
    s, sd = _logits(T, E, seed, s_z, scale)
    cfg = _cfg(T, E, k)
    r = P.route_logits(cfg, sd)
    torch.cuda.synchronize()
    ref = replica_route(cfg, s)
    assert ref["iters"] > 0
    assert_route_matches(cfg, r, ref)


@pytest.mark.parametrize("mode", [L.MOE_PRICE_ACP, L.MOE_PRICE_WARM])
def test_price_update_alone_matches_route(mode):
    """moe_price_update gives the prices and info of moe_route_logits (and
    of the FP32 replica of the update) bit for bit."""
    s, sd = _logits(2049, 40, 63)
    cfg = _cfg(2049, 40, 5, mode=mode)
    p0 = torch.full((40,), 0.05, dtype=torch.float32, device="cuda")
    price, info = P.price_update(cfg, sd, p0.clone())
    r = P.route_logits(cfg, sd, p0.clone())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(price.cpu().numpy().view(np.uint32),
                                  r["price"].cpu().numpy().view(np.uint32))
    np.testing.assert_array_equal(info.cpu().numpy(), r["info"].cpu().numpy())
    ref = replica_route(cfg, s, p0.cpu().numpy())
    assert ref["iters"] > 0
    np.testing.assert_array_equal(price.cpu().numpy().view(np.uint32),
                                  np.asarray(ref["p"], np.float32).view(np.uint32))
    assert int(info[L.INFO_ITERS]) == ref["iters"]


def test_route_logits_empty_batch():
    cfg = _cfg(0, 8, 2, 0)
    r = P.route_logits(cfg, torch.empty(0, 8, device="cuda"))
    torch.cuda.synchronize()
    assert int(r["info"][L.INFO_STATUS]) == 0 and int(r["load"].sum()) == 0


def test_certificate_matches_oracle():
    s, sd = _logits(2500, 32, 71)
    cfg = _cfg(2500, 32, 4)
    r = P.route_logits(cfg, sd)
    cert = P.certify(cfg, sd, r["price"], r["idx"]).cpu().numpy()
    p = r["price"].cpu().numpy()
    sel = r["idx"].cpu().numpy()
    prim = R.primal_objective(s, sel)
    dual = R.dual_objective(s, p, cfg.k, cfg.capacity)
    assert abs(cert[0] - prim) <= 1e-12 * abs(prim)
    assert abs(cert[1] - dual) <= 1e-12 * abs(dual)
    assert abs(cert[2] - (dual - prim) / abs(dual)) <= 1e-12
    if not int(r["info"][L.INFO_REPAIRED]):
        load = r["load"].cpu().numpy()
        ident = float(np.sum(p.astype(np.float64) * (cfg.capacity - load)))
        assert abs((cert[1] - cert[0]) - ident) <= 1e-9 * abs(dual)
    # the epsilon rule's gap: ~5e-4 at 16k tokens, up to ~2e-3 on small batches
    assert 0.0 <= cert[2] <= 5e-3


def _small_dataset(n, E, k, seed0):
    out = []
    for i in range(n):
        T = 600 + (i * 397) % 2500
        s = synth.make_logits(T, E, 1.0 + 0.5 * ((i * 7) % 11) / 10.0, seed0 + i)
        out.append((torch.from_numpy(s).cuda(), synth.capacity(T, k, E)))
    return out


def _assert_judged(cfg, r, s, phat, mode, tol, gamma=0.9):
    """The judged routing against the oracle's: the keep-or-fallback
    decision, the routing returned (bit-exact against the FP32 replica of
    the pass that produced it) and the verdict."""
    ref = R.judged_route(s, cfg.k, cfg.capacity, phat, mode, gamma, tol, cfg.max_iters,
                         cfg.price_stages)
    v = P.verdict_dict(r)
    assert v["kept"] == ref["kept"], (v, ref["gap_learned"])
    if ref["kept"]:
        pm = L.MOE_PRICE_WARM if mode == "warm" else L.MOE_PRICE_GIVEN
        c = L.make_cfg(cfg.T, cfg.d, cfg.E, cfg.k, cfg.d_ff, cfg.capacity,
                       cfg.max_iters if mode == "warm" else 0, cfg.act, cfg.w, pm, gamma,
                       cfg.price_stages)
        assert_route_matches(c, r, replica_route(c, s, phat))
    else:
        c = L.make_cfg(cfg.T, cfg.d, cfg.E, cfg.k, cfg.d_ff, cfg.capacity, cfg.max_iters, cfg.act,
                       cfg.w, L.MOE_PRICE_ACP, 0.9, cfg.price_stages)
        assert_route_matches(c, r, replica_route(c, s))
    assert v["V"] == ref["V"]
    assert v["learned_iters"] == ref["learned_iters"]
    assert abs(v["gap_learned"] - ref["gap_learned"]) <= 1e-12
    assert abs(v["gap"] - ref["gap"]) <= 1e-12
    return v, ref


# learned prices: the exact clearing prices and a 10 % under-estimate of
# them; tolerances that keep (1.0), judge (5e-3) and reject (0.0)
@pytest.mark.parametrize("fallback", ["device", "host"])
@pytest.mark.parametrize("tol", [1.0, 5e-3, 0.0])
@pytest.mark.parametrize("scale", [1.0, 0.9])
@pytest.mark.parametrize("mode", ["warm", "replace"])
def test_judged_route_matches_oracle(mode, scale, tol, fallback):
    """fallback "host": moe_route_learned, then the update from p = 0 only
    when the verdict rejects the learned routing."""
    T, E, k = 3001, 48, 6
    s, sd = _logits(T, E, 93)
    cfg = _cfg(T, E, k)
    pstar = R.route(s, k, cfg.capacity, 50)["p"]
    phat = (pstar * F32(scale)).astype(F32)
    r = P.judged_route(cfg, sd, torch.from_numpy(phat).cuda(), mode, gap_tol=tol,
                       fallback=fallback)
    torch.cuda.synchronize()
    v, ref = _assert_judged(cfg, r, s, phat, mode, tol)
    if tol == 1.0:
        assert v["kept"]
    if tol == 0.0:
        assert not v["kept"]


def test_judged_route_empty_batch_and_bad_mode():
    cfg = _cfg(0, 8, 2, 0)
    r = P.judged_route(cfg, torch.empty(0, 8, device="cuda"), torch.zeros(8, device="cuda"))
    torch.cuda.synchronize()
    assert int(r["info"][L.INFO_STATUS]) == 0 and P.verdict_dict(r)["kept"]
    s, sd = _logits(100, 8, 94)
    c = _cfg(100, 8, 2, mode=L.MOE_PRICE_ACP)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.MoEError) as e:
        L.moe_route_judged(c, sd.data_ptr(), sd.data_ptr(), 5e-3, sd.data_ptr(), sd.data_ptr(),
                           sd.data_ptr(), sd.data_ptr(), sd.data_ptr(), sd.data_ptr(),
                           ws.data_ptr(), ws.numel(), 0)
    assert e.value.status == L.MOE_EINVAL


def test_learned_prices_train_and_route_bit_exact():
    """Train on small batches, then route a fresh batch from the network's
    prices: warm start and replacement, each judged on the device and
    checked against the oracle's judged routing."""
    E, k = 64, 8
    ds = P.build_dataset(_small_dataset(24, E, k, 900), E, k)
    params, hist = P.train(ds, steps=300, batches_per_step=8, lr=1e-3, seed=3, log_every=50)
    torch.cuda.synchronize()
    assert hist[-1][1] < 0.5 * hist[0][1], hist
    T = 2048
    s = synth.make_logits(T, E, 1.25, 12345)
    sd = torch.from_numpy(s).cuda()
    cfg = _cfg(T, E, k)
    for mode in ("warm", "replace"):
        r = P.learned_route(cfg, sd, params, mode=mode)
        torch.cuda.synchronize()
        _assert_judged(cfg, r, s, r["p_hat"].cpu().numpy(), mode, P.GAP_TOL)


def test_learned_price_path_at_full_size():
    """Learned-price workload shapes (E=256, d=2048, top-8, T=16384 tokens
    through the router): features against the oracle, warm-started routing
    bit-exact against the replica started from gamma * p_hat, and the
    certificate against the oracle's objectives."""
    from _helpers import device_inputs
    from paper_2606_17065_amd import layer
    shape = synth.SHAPES[5]
    inp = synth.make_inputs(shape, 5, rep=2, experts=False)
    d, h = device_inputs(shape, inp)
    T, E, k = shape.T, shape.E, shape.k
    cfg = L.make_cfg(T, shape.d, E, k, shape.f, shape.capacity, 50, L.MOE_BF16, L.MOE_BF16,
                     L.MOE_PRICE_ACP)
    logits = layer.route(cfg, d["X"], d["Wr"], d["br"])["logits"]
    torch.cuda.synchronize()
    s = logits.cpu().numpy()
    feats, _ = P.logit_stats(cfg, logits)
    ref = M.features(s, k, cfg.capacity)
    got = feats.cpu().numpy().astype(np.float64)
    assert (np.abs(got - ref) / np.maximum(1.0, np.abs(ref))).max() <= 2e-6
    params = torch.from_numpy(M.init_params(21)).cuda()
    rw = P.learned_route(cfg, logits, params, mode="warm")
    torch.cuda.synchronize()
    _assert_judged(cfg, rw, s, rw["p_hat"].cpu().numpy(), "warm", P.GAP_TOL)
    cert = P.certify(cfg, logits, rw["price"], rw["idx"]).cpu().numpy()
    sel = rw["idx"].cpu().numpy()
    prim = R.primal_objective(s, sel)
    dual = R.dual_objective(s, rw["price"].cpu().numpy(), k, cfg.capacity)
    assert abs(cert[0] - prim) <= 1e-12 * abs(prim)
    assert abs(cert[1] - dual) <= 1e-12 * abs(dual)


def test_learned_warm_start_saves_updates_on_held_out_batches():
    """What the trained network gains: on fresh batches (seeds and lengths
    not seen in training) the warm start from 0.9 p_hat needs fewer price
    updates than the cold update from zero prices, and the judge keeps the
    warm routing (certificate gap within GAP_TOL) on every batch."""
    E, k = 64, 8
    train_sets = []
    for i in range(400):
        T = 1000 + (i * 613) % 5000
        s = synth.make_logits(T, E, 1.0 + 0.5 * ((i * 7) % 11) / 10.0, 70000 + i)
        train_sets.append((torch.from_numpy(s).cuda(), synth.capacity(T, k, E)))
    ds = P.build_dataset(train_sets, E, k)
    params, hist = P.train(ds, steps=1500, batches_per_step=16, lr=1e-3, seed=5, log_every=500)
    torch.cuda.synchronize()
    cold, warm = [], []
    for j, (T, s_z) in enumerate([(1777, 1.05), (2999, 1.45), (4321, 1.2), (5555, 1.3),
                                  (6101, 1.12), (3333, 1.38)]):
        s = synth.make_logits(T, E, s_z, 90000 + j)
        sd = torch.from_numpy(s).cuda()
        cfg = _cfg(T, E, k)
        rc = P.route_logits(cfg, sd)
        rw = P.learned_route(cfg, sd, params, mode="warm")
        torch.cuda.synchronize()
        v = P.verdict_dict(rw)
        assert v["kept"] and v["gap"] <= P.GAP_TOL, v
        _assert_judged(cfg, rw, s, rw["p_hat"].cpu().numpy(), "warm", P.GAP_TOL)
        cold.append(int(rc["info"][L.INFO_ITERS]))
        warm.append(v["learned_iters"])
    assert np.mean(warm) < np.mean(cold), (warm, cold)
    assert sum(w < c for w, c in zip(warm, cold)) >= 4, (warm, cold)


def test_learned_layer_forward_matches_oracle():
    """The layer forward from learned prices: the router alone gives the
    logits of moe_route bit for bit; the judged routing matches the
    oracle's; the output is within the BF16 bar of the FP64 layer on that
    routing."""
    from _helpers import assert_close, device_inputs
    from oracle import ffn
    from paper_2606_17065_amd import layer
    shape = synth.MoEShape("learned-layer", T=900, d=256, E=16, k=2, f=128, zipf=1.3,
                           act="bf16", w="bf16")
    inp = synth.make_inputs(shape, 61)
    d, h = device_inputs(shape, inp)
    cfg = L.make_cfg(shape.T, shape.d, shape.E, shape.k, shape.f, shape.capacity, 50,
                     L.MOE_BF16, L.MOE_BF16, L.MOE_PRICE_ACP)
    logits = layer.router_logits(cfg, d["X"], d["Wr"], d["br"])
    full = layer.route(cfg, d["X"], d["Wr"], d["br"])
    params = torch.from_numpy(M.init_params(22)).cuda()
    r = P.learned_layer_forward(cfg, d["X"], d["Wr"], d["br"], d["W13"], d["W2"], params)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(logits.cpu().numpy().view(np.uint32),
                                  full["logits"].cpu().numpy().view(np.uint32))
    s = logits.cpu().numpy()
    _assert_judged(cfg, r, s, r["p_hat"].cpu().numpy(), "warm", P.GAP_TOL)
    sel = r["idx"].cpu().numpy()
    s64 = R.logits_fp64(h["X"], h["Wr"], h["br"])
    w64 = R.gate_weights(s64, sel)
    ref = ffn.layer_forward(h["X"], sel, w64, h["W13"], h["W2"])["out"]
    assert_close(r["out"].float().cpu().numpy(), ref, 1.5e-2, "out")
