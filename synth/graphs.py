"""Seeded generators for the synthetic MaxCut and matrix-completion workloads.

Every generator takes an integer seed and draws from numpy's PCG64 stream, so the
same call returns byte-identical arrays on any machine.  Nothing here evaluates
the SDP (no Laplacian, constraint map or objective); the outputs are edge lists,
weights, planted factors and random starting points that both the oracle and the
GPU library consume.

Workload shapes (the paper measures on Gset and SuiteSparse graphs, which are not
available here; these synthetic families stand in for them):

* ``erdos_renyi_edges``: ``m`` distinct unordered pairs drawn uniformly without
  replacement from the ``n(n-1)/2`` possible pairs.
* ``chung_lu_edges``: power-law expected degrees, weight of node ``i`` proportional
  to ``(i+1)^(-1/(beta-1))``; both endpoints drawn proportionally to the weight
  (multinomial counts per node, shuffled), self-loops and repeats rejected until
  ``m`` distinct edges exist; node ids then relabelled by a uniform random
  permutation.
* ``completion_instance``: planted ``M = U V^T`` with ``U, V`` i.i.d. N(0, 1/k) and a
  fixed number of distinct observed columns per row.
"""

from __future__ import annotations

import sys

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _first_occurrences(keys: np.ndarray) -> np.ndarray:
    """Positions of the first occurrence of every distinct value of ``keys``, in
    increasing order (what ``np.unique(..., return_index=True)`` gives once
    sorted, without its stable argsort of the whole array: repeats are rare, so
    only the positions holding a repeated value are sorted by position)."""
    s = np.sort(keys)
    rep = s[1:][s[1:] == s[:-1]]
    if rep.size == 0:
        return np.arange(keys.size)
    rep = np.unique(rep)
    slot = np.searchsorted(rep, keys)
    slot[slot == rep.size] = 0
    pos = np.flatnonzero(rep[slot] == keys)          # every position holding a repeated value
    kp = keys[pos]
    order = np.argsort(kp, kind="stable")            # by value, then by position
    ks = kp[order]
    later = np.zeros(ks.size, dtype=bool)
    later[1:] = ks[1:] == ks[:-1]
    keep = np.ones(keys.size, dtype=bool)
    keep[pos[order[later]]] = False
    return np.flatnonzero(keep)


def _distinct_pairs(draw, n: int, m: int, rng: np.random.Generator, overdraw=None):
    """Draw endpoint pairs with ``draw(rng, k)`` until ``m`` distinct unordered,
    loop-free pairs exist; keep them in order of first appearance (so the result
    is a uniform sample without replacement when ``draw`` is uniform).
    ``overdraw(need)`` is the number of pairs drawn in a round (default twice
    the number still missing)."""
    keys = np.empty(0, dtype=np.int64)
    rounds = 0
    while keys.size < m:
        if m >= 10_000_000:
            print(f"[synth] distinct pairs: {keys.size}/{m} after {rounds} rounds", file=sys.stderr, flush=True)
        rounds += 1
        need = m - keys.size
        k = overdraw(need) if overdraw else max(2 * need, 1024)
        u, v = draw(rng, k)
        keep = u != v
        a = np.minimum(u, v)[keep].astype(np.int64)
        b = np.maximum(u, v)[keep].astype(np.int64)
        cand = np.concatenate([keys, a * n + b])
        del u, v, a, b, keep
        keys = cand[_first_occurrences(cand)]
    keys = keys[:m]
    return (keys // n).astype(np.int32), (keys % n).astype(np.int32)


def erdos_renyi_edges(n: int, m: int, seed: int):
    """Uniform random graph with exactly ``m`` edges on ``n`` nodes (G(n, m))."""
    if m > n * (n - 1) // 2:
        raise ValueError("more edges than node pairs")
    rng = _rng(seed)

    def draw(g, k):
        return g.integers(0, n, k), g.integers(0, n, k)

    return _distinct_pairs(draw, n, m, rng)


def chung_lu_edges(n: int, m: int, beta: float, seed: int, relabel: bool = True):
    """Chung-Lu power-law graph with degree exponent ``beta`` and ``m`` edges.

    Endpoints are i.i.d. draws with probability proportional to
    ``(i+1)^(-1/(beta-1))``.  A round of ``k`` pairs takes its ``2k`` endpoints
    as multinomial counts per node laid out in node order and shuffled by a
    uniform permutation, which is the law of ``2k`` i.i.d. draws (and avoids a
    binary search per draw); consecutive endpoints form the pairs."""
    if m > n * (n - 1) // 2:
        raise ValueError("more edges than node pairs")
    rng = _rng(seed)
    theta = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (beta - 1.0))
    prob = theta / theta.sum()
    ids = np.arange(n, dtype=np.int32)

    def draw(g, k):
        ends = np.repeat(ids, g.multinomial(2 * k, prob))
        g.shuffle(ends)
        return ends[0::2], ends[1::2]

    u, v = _distinct_pairs(draw, n, m, rng, overdraw=lambda need: need + need // 16 + 1024)
    if relabel:
        perm = rng.permutation(n).astype(np.int32)
        u, v = perm[u], perm[v]
        a, b = np.minimum(u, v), np.maximum(u, v)
        u, v = a, b
    return u, v


def pm1_weights(m: int, seed: int) -> np.ndarray:
    """Edge weights drawn uniformly from {-1, +1}."""
    rng = _rng(seed)
    return np.where(rng.integers(0, 2, m) == 1, 1.0, -1.0)


def init_factor(n: int, r: int, seed: int) -> np.ndarray:
    """Starting factor: i.i.d. N(0, 1) entries, each row scaled to unit length."""
    rng = _rng(seed)
    R = rng.standard_normal((n, r))
    nr = np.sqrt((R * R).sum(axis=1))
    nr[nr == 0] = 1.0
    return R / nr[:, None]


def gaussian_factor(n: int, r: int, scale: float, seed: int) -> np.ndarray:
    """i.i.d. N(0, scale^2) entries (used as a starting point for completion)."""
    rng = _rng(seed)
    return rng.standard_normal((n, r)) * scale


def completion_instance(n1: int, n2: int, k: int, per_row: int, seed: int):
    """Planted low-rank completion instance.

    Returns ``(i, j, Mij, U, V)`` where ``M = U V^T``, ``U`` is n1 x k and ``V`` is
    n2 x k with i.i.d. N(0, 1/k) entries, and every row ``i`` of M has ``per_row``
    distinct observed columns drawn uniformly.  Samples are sorted by (i, j).
    """
    if per_row > n2:
        raise ValueError("per_row exceeds the number of columns")
    rng = _rng(seed)
    U = rng.standard_normal((n1, k)) / np.sqrt(k)
    V = rng.standard_normal((n2, k)) / np.sqrt(k)
    if per_row * per_row * 4 > n2:
        cols = np.stack([rng.choice(n2, per_row, replace=False) for _ in range(n1)])
    else:
        cols = rng.integers(0, n2, (n1, per_row))
        while True:
            cols.sort(axis=1)
            bad = np.nonzero((np.diff(cols, axis=1) == 0).any(axis=1))[0]
            if bad.size == 0:
                break
            cols[bad] = rng.integers(0, n2, (bad.size, per_row))
    cols.sort(axis=1)
    i = np.repeat(np.arange(n1, dtype=np.int32), per_row)
    j = cols.reshape(-1).astype(np.int32)
    Mij = np.einsum("ak,ak->a", U[i], V[j])
    return i, j, Mij, U, V


# Named MaxCut workloads: (kind, n, m, beta, weights, rank, seed)
MAXCUT_CONFIGS = {
    # Erdos-Renyi, 1e3 nodes, 5e3 edges, unit weights, rank 10
    "er_1k": ("er", 1_000, 5_000, None, "unit", 10, 15049),
    # Erdos-Renyi, 1e6 nodes, 5e6 edges, +-1 weights, rank 20
    "er_1m_pm1": ("er", 1_000_000, 5_000_000, None, "pm1", 20, 15050),
    # Chung-Lu beta 2.5, 1e6 nodes, mean degree 10, +-1 weights, rank 20
    "cl_1m_pm1": ("cl", 1_000_000, 5_000_000, 2.5, "pm1", 20, 15051),
    # Chung-Lu beta 2.5, 1e7 nodes, mean degree 8, unit weights, rank 24
    "cl_10m": ("cl", 10_000_000, 40_000_000, 2.5, "unit", 24, 15052),
    # Chung-Lu beta 2.5, 5e7 nodes, mean degree 4, unit weights, rank 26
    "cl_50m": ("cl", 50_000_000, 100_000_000, 2.5, "unit", 26, 15053),
}


def maxcut_instance(name: str):
    """Materialise a named MaxCut workload: dict(n, u, v, w, rank, seed)."""
    kind, n, m, beta, wkind, rank, seed = MAXCUT_CONFIGS[name]
    if kind == "er":
        u, v = erdos_renyi_edges(n, m, seed)
    else:
        u, v = chung_lu_edges(n, m, beta, seed)
    w = None if wkind == "unit" else pm1_weights(m, seed + 7919)
    return dict(name=name, n=n, u=u, v=v, w=w, rank=rank, seed=seed)
