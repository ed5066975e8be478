"""Seeded general (single-block) SDP instances given as triplets.

Only data is drawn or written out here; the constraint map and everything the
method computes live in the oracle and the library.  Conventions of the
triplets: an off-diagonal entry (r, c, v), r != c, stands for both (r, c) and
(c, r) of a symmetric matrix.

* ``theta_triplets``: the Lovasz theta SDP of a graph in minimisation form,
  min <-J, X> s.t. trace X = 1 and X_uv = 0 for every edge (the second as
  <E_uv + E_vu, X> = 0); its optimum is minus the theta number.
* ``random_general_triplets``: a trace constraint (trace X = n, which keeps the
  feasible set bounded) plus m - 1 constraints with ``per_con`` random
  positions each (a share of them on the diagonal) and N(0, 1) values, a
  sparse N(0, 1) objective, and a random feasible point W W^T (W of rank r0,
  scaled to trace n) from which the caller forms b.
* ``random_box_triplets``: diag(X) = 1 (the MaxCut constraints) plus ``extra``
  random constraints of ``per_con`` positions each, a sparse N(0, 1)
  objective, and a feasible factor W with unit rows from which the caller
  forms the right-hand sides.
"""

from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def theta_triplets(n: int, u, v):
    """(c_row, c_col, c_val, m, a_con, a_row, a_col, a_val, b) of the theta SDP."""
    u = np.asarray(u, dtype=np.int32)
    v = np.asarray(v, dtype=np.int32)
    iu = np.triu_indices(n)
    c_row, c_col = iu[0].astype(np.int32), iu[1].astype(np.int32)
    c_val = -np.ones(len(c_row))
    m = 1 + len(u)
    diag = np.arange(n, dtype=np.int32)
    a_con = np.concatenate([np.zeros(n, np.int32), 1 + np.arange(len(u), dtype=np.int32)])
    a_row = np.concatenate([diag, u])
    a_col = np.concatenate([diag, v])
    a_val = np.ones(len(a_con))
    b = np.zeros(m)
    b[0] = 1.0
    return c_row, c_col, c_val, m, a_con, a_row, a_col, a_val, b


def cycle_edges(n: int):
    u = np.arange(n, dtype=np.int32)
    return u, ((u + 1) % n).astype(np.int32)


def petersen_edges():
    """Outer 5-cycle 0..4, spokes i -- i+5, inner pentagram 5..9."""
    u, v = [], []
    for i in range(5):
        u += [i, i, 5 + i]
        v += [(i + 1) % 5, 5 + i, 5 + (i + 2) % 5]
    return np.array(u, np.int32), np.array(v, np.int32)


def random_general_triplets(n: int, m: int, per_con: int, c_nnz: int, r0: int, seed: int):
    """Returns (c_row, c_col, c_val, m, a_con, a_row, a_col, a_val, W): the data
    of the instance and the factor W (n x r0, trace of W W^T = n) of a feasible
    point; b is <A_k, W W^T>, formed by the caller."""
    g = _rng(seed)
    c_row = g.integers(0, n, c_nnz).astype(np.int32)
    c_col = g.integers(0, n, c_nnz).astype(np.int32)
    c_val = g.standard_normal(c_nnz)
    diag = np.arange(n, dtype=np.int32)
    k = np.repeat(np.arange(1, m, dtype=np.int32), per_con)
    rr = g.integers(0, n, k.size).astype(np.int32)
    cc = np.where(g.random(k.size) < 0.25, rr, g.integers(0, n, k.size)).astype(np.int32)
    a_con = np.concatenate([np.zeros(n, np.int32), k])
    a_row = np.concatenate([diag, rr])
    a_col = np.concatenate([diag, cc])
    a_val = np.concatenate([np.ones(n), g.standard_normal(k.size)])
    W = g.standard_normal((n, r0))
    W *= np.sqrt(n / np.sum(W * W))
    return c_row, c_col, c_val, m, a_con, a_row, a_col, a_val, W


def random_box_triplets(n: int, extra: int, per_con: int, c_nnz: int, r0: int, seed: int):
    """Returns (c_row, c_col, c_val, m, a_con, a_row, a_col, a_val, W), m = n + extra."""
    g = _rng(seed)
    c_row = g.integers(0, n, c_nnz).astype(np.int32)
    c_col = g.integers(0, n, c_nnz).astype(np.int32)
    c_val = g.standard_normal(c_nnz)
    diag = np.arange(n, dtype=np.int32)
    k = np.repeat(np.arange(n, n + extra, dtype=np.int32), per_con)
    rr = g.integers(0, n, k.size).astype(np.int32)
    cc = g.integers(0, n, k.size).astype(np.int32)
    a_con = np.concatenate([diag, k])
    a_row = np.concatenate([diag, rr])
    a_col = np.concatenate([diag, cc])
    a_val = np.concatenate([np.ones(n), g.standard_normal(k.size)])
    W = g.standard_normal((n, r0))
    W /= np.sqrt(np.sum(W * W, axis=1))[:, None]
    return c_row, c_col, c_val, n + extra, a_con, a_row, a_col, a_val, W
