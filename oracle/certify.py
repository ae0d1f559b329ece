"""Independent optimality and feasibility checks -- TEST INFRASTRUCTURE ONLY.

These do not reuse the price iteration: they solve the routing problem of
``oracle.routing`` (maximise sum s*x, exactly k experts per token, at most C
tokens per expert) by other means.

* ``brute_force_opt``: enumeration of every routing (tiny inputs only).
* ``lp_opt``: the LP relaxation through SciPy's HiGHS; integral because the
  constraint matrix is totally unimodular.
* ``max_flow_feasible``: whether any routing at all respects the capacities,
  given a set of allowed (token, expert) pairs, by a max-flow.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.optimize
import scipy.sparse
import scipy.sparse.csgraph


def brute_force_opt(s: np.ndarray, k: int, C: int):
    """Best objective and one optimal routing over all C(E,k)^T choices.
    Returns (opt or None if infeasible, sel)."""
    s = np.asarray(s, dtype=np.float64)
    T, E = s.shape
    combos = np.array(list(itertools.combinations(range(E), k)), dtype=np.int64)  # [M,k]
    M = combos.shape[0]
    if M ** T > 3_000_000:
        raise ValueError("instance too large for enumeration")
    # value of each combo for each token: [T, M]
    val = s[:, combos].sum(axis=2)
    onehot = np.zeros((M, E), dtype=np.int64)
    onehot[np.arange(M)[:, None], combos] = 1
    grid = np.array(list(itertools.product(range(M), repeat=T)), dtype=np.int64)  # [M^T, T]
    obj = val[np.arange(T)[None, :], grid].sum(axis=1)
    load = onehot[grid].sum(axis=1)  # [M^T, E]
    feas = np.all(load <= C, axis=1)
    if not feas.any():
        return None, None
    obj = np.where(feas, obj, -np.inf)
    best = int(np.argmax(obj))
    return float(obj[best]), combos[grid[best]]


def lp_opt(s: np.ndarray, k: int, C: int):
    """LP relaxation optimum (HiGHS).  Returns (opt, x [T,E])."""
    s = np.asarray(s, dtype=np.float64)
    T, E = s.shape
    n = T * E
    # variable index v = t*E + e
    rows_eq = np.repeat(np.arange(T), E)
    A_eq = scipy.sparse.csr_matrix((np.ones(n), (rows_eq, np.arange(n))), shape=(T, n))
    rows_ub = np.tile(np.arange(E), T)
    A_ub = scipy.sparse.csr_matrix((np.ones(n), (rows_ub, np.arange(n))), shape=(E, n))
    res = scipy.optimize.linprog(
        -s.ravel(), A_ub=A_ub, b_ub=np.full(E, float(C)), A_eq=A_eq,
        b_eq=np.full(T, float(k)), bounds=(0.0, 1.0), method="highs")
    if res.status != 0:
        return None, None
    return float(-res.fun), res.x.reshape(T, E)


def max_flow_feasible(allowed: np.ndarray, k: int, C: int) -> bool:
    """True iff some routing gives every token k distinct allowed experts
    with no expert above C tokens.  allowed: bool [T,E]."""
    T, E = allowed.shape
    src, snk = T + E, T + E + 1
    ts, es = np.nonzero(allowed)
    rows = np.concatenate([np.full(T, src), ts, T + np.arange(E)])
    cols = np.concatenate([np.arange(T), T + es, np.full(E, snk)])
    caps = np.concatenate([np.full(T, k), np.ones(ts.shape[0], dtype=np.int64), np.full(E, C)])
    g = scipy.sparse.csr_matrix((caps.astype(np.int32), (rows, cols)), shape=(T + E + 2, T + E + 2))
    flow = scipy.sparse.csgraph.maximum_flow(g, src, snk).flow_value
    return int(flow) == T * k
