"""Pins of the oracle's large-size eigen- and singular-value branches.

The dual certificate uses a dense eigensolver up to n = 6000 and ARPACK above
(``lambda_min``), and a dense 2-norm up to min(n1, n2) = 1500 and ``svds``
above (``completion_dual_bound``).  The large branches are checked against
closed forms at sizes past the cut-offs and against the dense branches on the
same inputs.
"""

import numpy as np

from oracle import certify
from oracle.problem import completion_problem, maxcut_problem


def random_bipartite(n_half, deg, seed):
    """Random bipartite graph between nodes [0, h) and [h, 2h) with positive weights."""
    g = np.random.default_rng(seed)
    a = g.integers(0, n_half, n_half * deg)
    b = n_half + g.integers(0, n_half, n_half * deg)
    key = np.unique(a * (2 * n_half) + b)
    u, v = key // (2 * n_half), key % (2 * n_half)
    w = g.uniform(0.5, 2.0, u.size)
    return 2 * n_half, u, v, w


def test_arpack_branch_bipartite_closed_form():
    # Bipartite graph, w >= 0 (MaxCut section): the SDP optimum is -sum(w), reached by
    # y*_i = -1/2 sum_j w_ij, where C - Diag(y*) is a quarter of the signless Laplacian:
    # PSD with lambda_min = 0 (eigenvector +1 on one side, -1 on the other).
    n, u, v, w = random_bipartite(3001, 3, 7)          # n = 6002 > 6000: ARPACK branch
    prob = maxcut_problem(n, u, v, w)
    wdeg = np.bincount(u, weights=w, minlength=n) + np.bincount(v, weights=w, minlength=n)
    ystar = -0.5 * wdeg
    lam = certify.lambda_min(prob, ystar)
    assert abs(lam) <= 1e-8 * wdeg.max()
    assert np.isclose(certify.maxcut_dual_bound(prob, ystar), -w.sum(), rtol=1e-10)
    # a multiplier shifted down by 0.3 gives lambda_min = 0.3 exactly
    assert np.isclose(certify.lambda_min(prob, ystar - 0.3), 0.3, rtol=1e-8)


def test_arpack_branch_matches_dense_branch():
    n, u, v, w = random_bipartite(200, 4, 3)
    w = w * np.where(np.arange(w.size) % 3 == 0, -1.0, 1.0)
    prob = maxcut_problem(n, u, v, w)
    y = np.random.default_rng(5).standard_normal(n)
    dense = certify.lambda_min(prob, y)
    arpack = certify.lambda_min(prob, y, dense_limit=0)
    assert abs(dense - arpack) <= 1e-8 * (1.0 + abs(dense))


def test_svds_branch_rank_one_fully_observed():
    # M = c u v^T fully observed with y_k = u_i v_j: ||Y||_2 = ||u|| ||v|| (> 1 here), so
    # the certified bound b^T y / ||Y||_2 = 2 c ||u||^2 ||v||^2 / (||u|| ||v||) = 2 c ||u|| ||v||,
    # which is 2 ||M||_* (the optimum of the fully observed problem): the bound is tight.
    n1, n2, c = 1501, 1502, 0.7                         # min(n1, n2) > 1500: svds branch
    g = np.random.default_rng(11)
    uu, vv = g.standard_normal(n1), g.standard_normal(n2)
    i = np.repeat(np.arange(n1), n2)
    j = np.tile(np.arange(n2), n1)
    M = c * uu[i] * vv[j]
    prob = completion_problem(n1, n2, i, j, M)
    y = uu[i] * vv[j]
    bound = certify.completion_dual_bound(prob, n1, n2, i, j, y)
    assert np.isclose(bound, 2 * c * np.linalg.norm(uu) * np.linalg.norm(vv), rtol=1e-9)


def test_svds_branch_matches_dense_norm():
    n1, n2, per_row = 1600, 1700, 12
    g = np.random.default_rng(12)
    i = np.repeat(np.arange(n1), per_row)
    j = np.concatenate([g.choice(n2, per_row, replace=False) for _ in range(n1)])
    M = g.standard_normal(i.size)
    prob = completion_problem(n1, n2, i, j, M)
    y = 0.2 * g.standard_normal(i.size)
    Y = np.zeros((n1, n2))
    Y[i, j] = y
    s = np.linalg.norm(Y, 2)
    assert s > 1.0
    bound = certify.completion_dual_bound(prob, n1, n2, i, j, y)
    assert np.isclose(bound, float(prob.b @ y) / s, rtol=1e-9)
