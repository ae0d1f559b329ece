"""FP32-replica router of the oracle -- TEST INFRASTRUCTURE ONLY.

Parity unpinned by the paper: the paper defines no routing rule.  The
reading implemented here, stated in full:

Problem.  Scores s[T,E] are FP32 router logits.  Choose x[t,e] in {0,1}
maximising sum s*x subject to sum_e x[t,e] = k for every token and
sum_t x[t,e] <= C for every expert.  The constraint matrix is that of a
bipartite b-matching (totally unimodular), so the LP relaxation has an
integral optimum.  Dualising the capacity rows with prices p >= 0 gives

    D(p) = C * sum_e p_e + sum_t topk_sum(s_t - p),

whose inner maximisation is plain top-k of a = s - p: zero prices reduce
to plain top-k.  If x is top-k under p, load <= C, and p_e > 0 implies
load_e = C, then sum s*x = D(p) and x is optimal.

Ascending clearing price (Jacobi form), all arithmetic FP32, one rounding
per operation, no contraction:

  sigma_s = std of all of s by the fixed-order FP64 reduction of
  ``score_sigma``; eps = fl32(fl32(1e-3) * sigma_s).
  p = p0 (zero unless warm-started); iters = 0.  Loop:
   1. a = fl32(s - p).  Rank each token's experts by the sortable key of a,
      descending, ties to the lower expert index.  S_t = first k,
      kappa1_t = a at rank k, kappa2_t = a at rank k+1.
   2. load_e = #{t : e in S_t}.  If every load_e <= C: converged, stop.
      If iters == max_iters: stop unconverged.
   3. For each expert with load_e > C: margins
      m[t] = fl32(s[t,e] - (e in S_t ? kappa2_t : kappa1_t)); let q be the
      (C+1)-th largest margin in key order;
      p_e = max(p_e, fl32(nextafter(q, +inf) + eps)).  Other prices stay.
   4. iters += 1, repeat.

Variant rule, epsilon-scaled restarts ("scaled", reading stated here): the
update above is stage 0.  While the previous stage ended converged with
some expert priced above zero and below capacity (a nonzero certificate
gap), and fewer than ``stages`` restarts have run: p = max(0, fl32(p - fl32(4 *
eps))), eps = fl32(eps / 8), and the update runs again from those prices
(at most ``max_iters`` updates per stage; a lowered price that is not
positive becomes +0).  Lowering every price by a few
increments puts it back below the clearing level that the previous stage
overshot by up to one increment; the next stage climbs back with a smaller
increment, so the certificate gap shrinks with each stage.  The iteration
count reported is the sum over the stages.

Variant rule, projected dual subgradient ("subgrad", reading stated here):
prices start at zero and every expert's price moves along the negative
subgradient of D, whose e-th component at p is C - load_e (load under the
top-k ranking of step 1), projected back onto p >= 0.  Step 1 and the stop
test of step 2 are those above; step 3 becomes, for every expert,

      eta = fl32(eta0 / fl32(sqrt(fl32(iters + 1)))),  eta0 = fl32(256 * eps)
      g_e = fl32(fl32(load_e - C) / fl32(C))
      x   = fl32(p_e + fl32(eta * g_e)),  p_e = (x > 0 ? x : +0).

The step is relative to the capacity and shrinks as 1/sqrt of the update
count (the classic diminishing step of subgradient methods); eta0 is a
quarter of the score standard deviation.  Prices of underloaded experts fall
back towards zero, so unlike the ascending rule the prices are not
monotone; the iteration can end at max_iters with some expert over
capacity, and the repair then places the overflow.

The routing returned is S_t of the last ranking, in rank order.  Gate
weights are the softmax of the raw logits over the k chosen experts.  If the
final routing still overloads an expert, ``enforce_capacity`` repairs it.

Sortable key: for FP32 bit pattern u, key = ~u if the sign bit is set, else
u | 0x80000000 (so -0 < +0 and the key order is the float order).
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32

# Status codes shared in meaning (not in code) with the C library.
OK = 0
EINVAL = -1
EINFEASIBLE = -2
ENAN = -6
ECAPACITY = -7

SIGMA_BLOCK = 256  # block width of the fixed-order reduction
EPS_REL = F32(1e-3)


def f32_key(a: np.ndarray) -> np.ndarray:
    """Order-preserving uint32 key of float32 values."""
    u = np.ascontiguousarray(a, dtype=F32).view(np.uint32)
    return np.where(u >> np.uint32(31), ~u, u | np.uint32(0x80000000)).astype(np.uint32)


def rank_experts(a32: np.ndarray, m: int) -> np.ndarray:
    """First ``m`` experts of each row of a32, best first: key descending,
    ties to the lower expert index.  Returns int32 [T, m]."""
    T, E = a32.shape
    key = f32_key(a32).astype(np.uint64)
    tie = np.uint64(0xFFFFFFFF) - np.arange(E, dtype=np.uint64)
    k64 = (key << np.uint64(32)) | tie[None, :]
    order = np.argsort(k64, axis=1, kind="stable")[:, ::-1]
    return np.ascontiguousarray(order[:, :m]).astype(np.int32)


def _fixed_tree_sum(v: np.ndarray) -> float:
    """Sum of float64 values in a fixed order: blocks of 256 consecutive
    entries (zero-padded) reduced by halving (i += i + stride for stride =
    128, 64, ..., 1); then the block totals are folded into 256 running sums
    (running sum i takes totals i, i+256, i+512, ... in order) and those are
    reduced by the same halving tree."""
    B = SIGMA_BLOCK
    n = v.shape[0]
    nb = max(1, -(-n // B))
    x = np.zeros(nb * B, dtype=np.float64)
    x[:n] = v
    x = x.reshape(nb, B)
    stride = B // 2
    while stride >= 1:
        x[:, :stride] = x[:, :stride] + x[:, stride:2 * stride]
        stride //= 2
    parts = x[:, 0].copy()
    acc = np.zeros(B, dtype=np.float64)
    for j in range(0, nb, B):
        chunk = parts[j:j + B]
        acc[:chunk.shape[0]] = acc[:chunk.shape[0]] + chunk
    stride = B // 2
    while stride >= 1:
        acc[:stride] = acc[:stride] + acc[stride:2 * stride]
        stride //= 2
    return float(acc[0])


def score_sums(s32: np.ndarray) -> tuple[float, float]:
    """(sum s, sum s^2) over all of s in the fixed order: each token row is
    accumulated in FP64 from expert 0 upward, then rows are combined by
    ``_fixed_tree_sum``."""
    T, E = s32.shape
    r1 = np.zeros(T, dtype=np.float64)
    r2 = np.zeros(T, dtype=np.float64)
    for e in range(E):
        v = s32[:, e].astype(np.float64)
        r1 = r1 + v
        r2 = r2 + v * v
    return _fixed_tree_sum(r1), _fixed_tree_sum(r2)


def score_sigma(s32: np.ndarray) -> F32:
    """Population standard deviation of all scores, rounded to FP32:
    mean = S1/n, var = max(S2/n - mean*mean, 0), sigma = fl32(sqrt(var))."""
    S1, S2 = score_sums(s32)
    n = float(s32.size)
    mean = S1 / n
    var = S2 / n - mean * mean
    var = max(var, 0.0)
    return F32(math.sqrt(var))


def price_eps(s32: np.ndarray) -> F32:
    return F32(EPS_REL * score_sigma(s32))


def loads(sel: np.ndarray, E: int) -> np.ndarray:
    return np.bincount(sel.ravel(), minlength=E).astype(np.int64)


def topk_under_prices(s32: np.ndarray, p32: np.ndarray, k: int):
    """One ranking pass: returns (sel [T,k] in rank order, kappa1 [T],
    kappa2 [T] (-inf when k == E), a [T,E])."""
    T, E = s32.shape
    a = (s32 - p32[None, :].astype(F32)).astype(F32)
    m = min(k + 1, E)
    order = rank_experts(a, m)
    rows = np.arange(T)
    sel = order[:, :k]
    kap1 = a[rows, order[:, k - 1]]
    if k < E:
        kap2 = a[rows, order[:, k]]
    else:
        kap2 = np.full(T, -np.inf, dtype=F32)
    return sel, kap1.astype(F32), kap2.astype(F32), a


def kth_largest_by_key(m32: np.ndarray, r: int) -> F32:
    """The r-th largest (1-based) of float32 values in sortable-key order."""
    key = f32_key(m32)
    order = np.argsort(key, kind="stable")
    return F32(m32[order[m32.shape[0] - r]])


def acp_prices(s32, k, C, max_iters=50, p0=None, eps=None):
    """Ascending clearing-price iteration (module header, steps 1-4).

    Returns dict(p, iters, converged, sel, load, eps)."""
    s32 = np.ascontiguousarray(s32, dtype=F32)
    T, E = s32.shape
    p = np.zeros(E, dtype=F32) if p0 is None else np.array(p0, dtype=F32).copy()
    if eps is None:
        eps = price_eps(s32)
    eps = F32(eps)
    iters = 0
    inf = F32(np.inf)
    while True:
        sel, kap1, kap2, a = topk_under_prices(s32, p, k)
        load = loads(sel, E)
        if np.all(load <= C):
            return dict(p=p, iters=iters, converged=True, sel=sel, load=load, eps=eps)
        if iters >= max_iters:
            return dict(p=p, iters=iters, converged=False, sel=sel, load=load, eps=eps)
        held = np.zeros((T, E), dtype=bool)
        held[np.arange(T)[:, None], sel] = True
        newp = p.copy()
        for e in np.nonzero(load > C)[0]:
            ref = np.where(held[:, e], kap2, kap1).astype(F32)
            m = (s32[:, e] - ref).astype(F32)
            q = kth_largest_by_key(m, C + 1)
            cand = F32(F32(np.nextafter(q, inf)) + eps)
            newp[e] = max(p[e], cand)
        p = newp
        iters += 1


SUBGRAD_ETA0 = F32(256.0)  # subgradient step: eta0 = 256 increments


def subgrad_prices(s32, k, C, max_iters=50, eps=None):
    """Projected dual subgradient iteration (module header, "subgrad").

    Returns dict(p, iters, converged, sel, load, eps)."""
    s32 = np.ascontiguousarray(s32, dtype=F32)
    T, E = s32.shape
    p = np.zeros(E, dtype=F32)
    if eps is None:
        eps = price_eps(s32)
    eps = F32(eps)
    eta0 = F32(SUBGRAD_ETA0 * eps)
    iters = 0
    while True:
        sel, _, _, _ = topk_under_prices(s32, p, k)
        load = loads(sel, E)
        if np.all(load <= C):
            return dict(p=p, iters=iters, converged=True, sel=sel, load=load, eps=eps)
        if iters >= max_iters:
            return dict(p=p, iters=iters, converged=False, sel=sel, load=load, eps=eps)
        eta = F32(eta0 / F32(np.sqrt(F32(iters + 1))))
        g = (load - C).astype(F32) / F32(C)
        x = (p + (eta * g).astype(F32)).astype(F32)
        p = np.where(x > 0, x, F32(0.0)).astype(F32)
        iters += 1


SCALED_BACK = F32(4.0)    # restart: prices lowered by this many increments
SCALED_SHRINK = F32(8.0)  # and the increment divided by this


def _slack_free(p, load, C) -> bool:
    """Complementary slackness of a feasible top-k routing: every expert with
    a positive price is full, so the certificate gap is zero (optimal)."""
    return bool(np.all((p == 0) | (load == C)))


def acp_scaled_prices(s32, k, C, max_iters=50, p0=None, eps=None, stages=3):
    """Epsilon-scaled restarts of the ascending clearing price (module
    header, "Variant rule").  Returns the dict of ``acp_prices`` for the
    last stage with ``iters`` summed over the stages and ``stages_run``."""
    s32 = np.ascontiguousarray(s32, dtype=F32)
    if eps is None:
        eps = price_eps(s32)
    eps = F32(eps)
    r = acp_prices(s32, k, C, max_iters, p0, eps)
    total = r["iters"]
    run = 0
    while r["converged"] and run < stages and not _slack_free(r["p"], r["load"], C):
        lowered = (r["p"] - F32(SCALED_BACK * eps)).astype(F32)
        p = np.where(lowered > F32(0.0), lowered, F32(0.0)).astype(F32)
        eps = F32(eps / SCALED_SHRINK)
        r = acp_prices(s32, k, C, max_iters, p, eps)
        total += r["iters"]
        run += 1
    r["iters"] = total
    r["stages_run"] = run
    return r


def enforce_capacity(s32, p32, sel, k, C):
    """Repair a routing that overloads some expert (reading stated here).

    a = fl32(s - p).  1) Every expert with load > C keeps the C holders with
    the best (key(a) desc, token asc) and evicts the rest; an evicted
    expert counts as tried by that token.  2) Rounds: each token short of k
    proposes to as many of its best untried, unheld experts (key(a) desc,
    expert asc) as it is short; each expert accepts proposals in (key(a)
    desc, token asc) order while it has room; every proposal marks the
    expert as tried.  A token that needs more experts than it has untried
    ones fails the repair with ECAPACITY.

    Returns (sel [T,k] in rank order, status, rounds)."""
    s32 = np.ascontiguousarray(s32, dtype=F32)
    T, E = s32.shape
    a = (s32 - np.asarray(p32, dtype=F32)[None, :]).astype(F32)
    key = f32_key(a).astype(np.int64)
    held = np.zeros((T, E), dtype=bool)
    held[np.arange(T)[:, None], sel] = True
    tried = held.copy()
    load = held.sum(axis=0)
    missing = np.zeros(T, dtype=np.int64)
    for e in np.nonzero(load > C)[0]:
        holders = np.nonzero(held[:, e])[0]
        order = np.lexsort((holders, -key[holders, e]))  # key desc, t asc
        evict = holders[order[C:]]
        held[evict, e] = False
        missing[evict] += 1
        load[e] = C
    rounds = 0
    while missing.any():
        rounds += 1
        proposals = [[] for _ in range(E)]
        for t in np.nonzero(missing)[0]:
            cands = np.nonzero(~tried[t])[0]
            if cands.shape[0] < missing[t]:
                return None, ECAPACITY, rounds
            order = np.lexsort((cands, -key[t, cands]))  # key desc, e asc
            for e in cands[order[:missing[t]]]:
                proposals[e].append(t)
                tried[t, e] = True
        for e in range(E):
            if not proposals[e]:
                continue
            props = np.array(proposals[e], dtype=np.int64)
            order = np.lexsort((props, -key[props, e]))  # key desc, t asc
            room = C - load[e]
            acc = props[order[:max(room, 0)]]
            held[acc, e] = True
            load[e] += acc.shape[0]
            missing[acc] -= 1
    # rebuild the per-token lists in rank order
    tie = np.uint64(0xFFFFFFFF) - np.arange(E, dtype=np.uint64)
    k64 = (f32_key(a).astype(np.uint64) << np.uint64(32)) | tie[None, :]
    k64 = np.where(held, k64, np.uint64(0))
    order = np.argsort(k64, axis=1, kind="stable")[:, ::-1][:, :k]
    return np.ascontiguousarray(order).astype(np.int32), OK, rounds


def gate_weights(s: np.ndarray, sel: np.ndarray) -> np.ndarray:
    """w[t,j] = exp(s[t,e_j] - M_t) / sum_i exp(s[t,e_i] - M_t), M_t the max
    of the selected raw logits (FP64)."""
    rows = np.arange(sel.shape[0])[:, None]
    z = np.asarray(s, dtype=np.float64)[rows, sel]
    z = z - z.max(axis=1, keepdims=True)
    ez = np.exp(z)
    return ez / ez.sum(axis=1, keepdims=True)


def route(s32, k, C, max_iters=50, p0=None, mode="acp", stages=0):
    """The whole routing step on FP32 logits.

    mode: "none" (p = 0, no update), "acp" (from p0 or 0), "given" (p = p0,
    no update), "subgrad" (the projected dual subgradient from 0).  stages
    > 0 (with "acp") runs the epsilon-scaled restarts after the update.  Returns dict with sel, w (FP64), load, p, iters,
    converged, enforced, status, eps, sigma."""
    s32 = np.ascontiguousarray(s32, dtype=F32)
    T, E = s32.shape
    res = dict(sel=None, w=None, load=None, p=None, iters=0, converged=False,
               enforced=False, status=OK, eps=None, sigma=None, rounds=0)
    if k < 1 or k > E or C < 0:
        res["status"] = EINFEASIBLE if k > E else EINVAL
        return res
    if E * C < T * k:
        res["status"] = EINFEASIBLE
        return res
    if not np.all(np.isfinite(s32)):
        res["status"] = ENAN
        return res
    res["sigma"] = score_sigma(s32)
    eps = F32(EPS_REL * res["sigma"])
    res["eps"] = eps
    p = np.zeros(E, dtype=F32) if p0 is None else np.array(p0, dtype=F32)
    if mode == "acp":
        if stages > 0 and max_iters > 0:
            r = acp_scaled_prices(s32, k, C, max_iters, p, eps, stages)
        else:
            r = acp_prices(s32, k, C, max_iters, p, eps)
        res["eps"] = r["eps"]  # the increment of the last stage
        p, sel, load = r["p"], r["sel"], r["load"]
        res["iters"], res["converged"] = r["iters"], r["converged"]
    elif mode == "subgrad":
        r = subgrad_prices(s32, k, C, max_iters, eps)
        p, sel, load = r["p"], r["sel"], r["load"]
        res["iters"], res["converged"] = r["iters"], r["converged"]
    else:
        sel, _, _, _ = topk_under_prices(s32, p, k)
        load = loads(sel, E)
        res["converged"] = bool(np.all(load <= C))
    if np.any(load > C):
        sel2, st, rounds = enforce_capacity(s32, p, sel, k, C)
        res["enforced"], res["rounds"] = True, rounds
        if st != OK:
            res["status"] = st
            res["p"] = p
            return res
        sel = sel2
        load = loads(sel, E)
    res["sel"], res["load"], res["p"] = sel, load, p
    res["w"] = gate_weights(s32, sel)
    return res


def judged_route(s32, k, C, p_hat, mode="warm", gamma=0.9, gap_tol=5e-3, max_iters=50,
                 stages=0):
    """Routing from learned prices, judged by the duality certificate, with
    the update from zero prices as fallback (reading stated here).

    Learned pass: "warm" runs the clearing-price update from p0 =
    fl32(gamma * p_hat) (at most max_iters updates); "replace" routes under
    p_hat alone (no update; the capacity repair places any overflow).  The
    learned routing is kept when its status is OK and its relative gap
    (D(p) - sum s x) / |D(p)| under its own prices is <= gap_tol (weak
    duality makes this a valid bound for any routing within capacity,
    repaired ones included).  Otherwise the batch is routed by the update
    from p = 0.  A non-finite logit is reported as such, with no fallback.
    stages > 0 adds that many epsilon-scaled restarts to both updates.

    Returns the dict of ``route`` for the routing kept, plus V (overflow of
    the learned ranking before any repair, divided by N = T k), gap_learned,
    kept, gap (of the routing returned) and learned_iters."""
    s32 = np.ascontiguousarray(s32, dtype=F32)
    T, E = s32.shape
    ph = np.asarray(p_hat, dtype=F32)
    if mode == "warm":
        r = route(s32, k, C, max_iters, (F32(gamma) * ph).astype(F32), "acp", stages)
    elif mode == "replace":
        r = route(s32, k, C, 0, ph, "given")
    else:
        raise ValueError(mode)
    N = max(T * k, 1)
    extra = dict(V=0.0, gap_learned=float("nan"), kept=False, gap=float("nan"),
                 learned_iters=r["iters"])
    if r["status"] == ENAN:
        return {**r, **extra}
    if r["p"] is not None:
        sel0 = topk_under_prices(s32, r["p"], k)[0]
        extra["V"] = float(np.maximum(loads(sel0, E) - C, 0).sum()) / N

    def rel_gap(res):
        prim = primal_objective(s32, res["sel"])
        dual = dual_objective(s32, res["p"], k, C)
        return (dual - prim) / (abs(dual) if dual != 0.0 else 1.0)

    if r["status"] == OK:
        extra["gap_learned"] = rel_gap(r)
        extra["kept"] = extra["gap_learned"] <= gap_tol
    if not extra["kept"]:
        r = route(s32, k, C, max_iters, None, "acp", stages)
    if r["status"] == OK:
        extra["gap"] = rel_gap(r)
    return {**r, **extra}


def primal_objective(s, sel) -> float:
    rows = np.arange(sel.shape[0])[:, None]
    return float(np.asarray(s, dtype=np.float64)[rows, sel].sum())


def dual_objective(s, p, k, C) -> float:
    """D(p) = C*sum p + sum_t (sum of the k largest of s_t - p), in FP64."""
    a = np.asarray(s, dtype=np.float64) - np.asarray(p, dtype=np.float64)[None, :]
    part = -np.partition(-a, k - 1, axis=1)[:, :k]
    return float(C * np.sum(np.asarray(p, dtype=np.float64)) + part.sum())


def logits_fp64(X, Wr, br) -> np.ndarray:
    """s = X W_r^T + b_r in FP64."""
    return np.asarray(X, np.float64) @ np.asarray(Wr, np.float64).T + np.asarray(br, np.float64)[None, :]
