"""Dual certificates and brute-force references.

Test infrastructure only (see the package docstring).

* ``lambda_min``: smallest eigenvalue of the dual slack S = C - A*(y) (dense
  symmetric eigensolver for small n, ARPACK Lanczos otherwise); gives the dual
  infeasibility err2 of the paper's experimental setting.
* ``maxcut_dual_bound``: for MaxCut A*(1) = I, so y + min(0, lambda_min) 1 is
  dual feasible for ANY y and its dual objective is a certified lower bound on the
  minimisation optimum.
* ``completion_dual_bound``: for completion C = I, and y / max(1, ||Y||_2) is dual
  feasible, where Y is the n1 x n2 matrix carrying y_k at the observed (i, j).
* ``brute_force_maxcut``: exact max cut by enumerating all 2^(n-1) partitions.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .problem import SDPProblem


def lambda_min(prob: SDPProblem, y: np.ndarray, dense_limit: int = 6000) -> float:
    S = (prob.C - prob.A_adj(y)).tocsr()
    if prob.n <= dense_limit:
        return float(sla.eigvalsh(S.toarray(), subset_by_index=[0, 0])[0])
    vals = spla.eigsh(S, k=1, which="SA", tol=1e-10, maxiter=20 * prob.n,
                      return_eigenvectors=False)
    return float(vals[0])


def err2(prob: SDPProblem, y: np.ndarray) -> float:
    lm = lambda_min(prob, y)
    return abs(min(0.0, lm)) / (1.0 + prob.c_l1)


def maxcut_dual_bound(prob: SDPProblem, y: np.ndarray) -> float:
    lm = lambda_min(prob, y)
    return float(y.sum()) + prob.n * min(0.0, lm)


def completion_dual_bound(prob: SDPProblem, n1: int, n2: int, i, j, y) -> float:
    Y = sp.csr_matrix((y, (np.asarray(i), np.asarray(j))), shape=(n1, n2))
    if min(n1, n2) <= 1500:
        s = float(np.linalg.norm(Y.toarray(), 2))
    else:
        s = float(spla.svds(Y, k=1, return_singular_vectors=False, tol=1e-10)[0])
    return float(prob.b @ y) / max(1.0, s)


def brute_force_maxcut(n: int, u, v, w=None) -> float:
    """Maximum cut weight over all partitions (node n-1 fixed on one side)."""
    if n > 24:
        raise ValueError("brute force limited to n <= 24")
    u = np.asarray(u)
    v = np.asarray(v)
    w = np.ones(len(u)) if w is None else np.asarray(w, dtype=np.float64)
    best = -np.inf
    chunk = 1 << 16
    total = 1 << (n - 1)
    for start in range(0, total, chunk):
        masks = np.arange(start, min(total, start + chunk), dtype=np.int64)
        side_u = (masks[:, None] >> u[None, :]) & 1
        side_v = (masks[:, None] >> v[None, :]) & 1
        cut = ((side_u != side_v) * w[None, :]).sum(axis=1)
        best = max(best, float(cut.max()))
    return best


def cut_value(u, v, w, side) -> float:
    """Weight of the edges whose endpoints have different sides (+1 / -1)."""
    w = np.ones(len(u)) if w is None else np.asarray(w)
    side = np.asarray(side)
    return float(w[side[u] != side[v]].sum())
