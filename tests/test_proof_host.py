"""Host proof of a lower bound on lambda_min(C - A*(y)) (lrsdp_certify_dense).

The library factorises C - A*(y) - shift I by Cholesky on the host and, when
every pivot is positive, proves lambda_min >= shift - margin from the rounding
analysis of Cholesky.  The cases pin it against values fixed independently of
the library: the complete graph at its optimal multipliers (S = J/4, so
lambda_min = 0 and the MaxCut SDP optimum -n^2/4), the completion slack
I - A*(y), whose smallest eigenvalue is 1 - sigma_max of the n1 x n2 matrix of
the multipliers (an SVD), and the oracle's dense eigensolver on random MaxCut
and general instances.  A shift a little below lambda_min must be proven with a
bound below lambda_min; a shift a little above must fail.  No GPU is used.
"""

import numpy as np
import pytest

from oracle import certify as OC
from oracle.problem import completion_problem, general_problem, maxcut_problem
from synth import erdos_renyi_edges, pm1_weights
from synth.general import random_general_triplets

from paper_2407_15049_amd import lrsdp as L


def complete_graph(n):
    u, v = np.triu_indices(n, 1)
    return u.astype(np.int32), v.astype(np.int32)


def check_brackets(prob, y, lam, rel=1e-7):
    """shift below lambda_min: proven, bound <= lambda_min; shift above: fails."""
    d = rel * (1.0 + abs(lam))
    lo = L.certify_dense(prob, y, lam - d)
    assert lo.status == 0, lo.as_dict()
    assert lo.lambda_lb <= lam and lo.lambda_lb >= lam - 2 * d
    assert 0.0 < lo.margin < 0.1 * d
    hi = L.certify_dense(prob, y, lam + d)
    assert hi.status == 1 and np.isnan(hi.lambda_lb)
    return lo


@pytest.mark.parametrize("order", ["input", "degree"])
def test_complete_graph_at_its_optimal_multipliers(order):
    # C = -L/4 of K_n and y = -n/4: S = J/4, lambda_min = 0 (n - 1 times); the
    # optimum of min <C, X> over diag(X) = 1 is -n^2/4
    n = 40
    u, v = complete_graph(n)
    node_order = L.ORDER_DEGREE if order == "degree" else None
    prob = L.Problem.maxcut(n, u, v, node_order=node_order)
    y = np.full(n, -n / 4.0)
    p = L.certify_dense(prob, y, -1e-9)
    assert p.status == 0 and -1e-9 - 1e-12 <= p.lambda_lb <= -1e-9
    assert p.by == -n * n / 4.0
    assert -n * n / 4.0 - 1e-6 <= p.dual_bound <= -n * n / 4.0
    assert L.certify_dense(prob, y, 1e-6).status == 1


@pytest.mark.parametrize("weights", ["unit", "pm1", "real"])
@pytest.mark.parametrize("order", ["input", "degree"])
def test_random_maxcut_against_the_dense_eigensolver(weights, order):
    n = 300
    u, v = erdos_renyi_edges(n, 1500, 21)
    w = {"unit": None, "pm1": pm1_weights(len(u), 22),
         "real": np.random.default_rng(23).uniform(0.1, 2.0, len(u))}[weights]
    prob = L.Problem.maxcut(n, u, v, w, node_order=L.ORDER_DEGREE if order == "degree" else None)
    oprob = maxcut_problem(n, u, v, w)
    y = np.random.default_rng(24).normal(-2.0, 1.0, n)
    lam = OC.lambda_min(oprob, y)
    p = check_brackets(prob, y, lam)
    # the dual bound is the MaxCut formula at the proven bound
    want = y.sum() + n * min(0.0, p.lambda_lb)
    assert p.dual_bound <= want and p.dual_bound >= want - 1e-9 * abs(want)


def test_completion_slack_is_one_minus_the_spectral_norm():
    n1, n2, m = 30, 25, 200
    g = np.random.default_rng(31)
    cells = g.choice(n1 * n2, m, replace=False)
    i, j = (cells // n2).astype(np.int32), (cells % n2).astype(np.int32)
    Mij = g.standard_normal(m)
    prob = L.Problem.completion(n1, n2, i, j, Mij)
    y = 0.3 * g.standard_normal(m)
    Y = np.zeros((n1, n2))
    Y[i, j] = y
    lam = 1.0 - np.linalg.svd(Y, compute_uv=False)[0]
    assert lam == pytest.approx(OC.lambda_min(completion_problem(n1, n2, i, j, Mij), y), abs=1e-12)
    p = check_brackets(prob, y, lam)
    by = float(np.dot(2.0 * Mij, y))
    want = by / (1.0 - min(0.0, p.lambda_lb))
    assert p.dual_bound <= want and p.dual_bound >= want - 1e-9 * abs(want)


@pytest.mark.parametrize("storage", [None, L.C_DENSE])
def test_general_against_the_dense_eigensolver(storage):
    n = 120
    c_row, c_col, c_val, m, a_con, a_row, a_col, a_val, _ = random_general_triplets(n, 40, 6, 500, 4, 41)
    b = np.ones(m)
    prob = L.Problem.general(n, c_row, c_col, c_val, m, a_con, a_row, a_col, a_val, b, c_storage=storage)
    oprob = general_problem(n, c_row, c_col, c_val, m, a_con, a_row, a_col, a_val, b)
    y = np.random.default_rng(42).standard_normal(m)
    lam = OC.lambda_min(oprob, y)
    p = check_brackets(prob, y, lam)
    assert np.isnan(p.dual_bound)


def test_margin_grows_with_the_scale_of_s():
    # the rounding allowance is relative: scaling the multipliers and the shift
    # by 1e6 scales the diagonal, and with it the margin
    n = 60
    u, v = complete_graph(n)
    prob = L.Problem.maxcut(n, u, v)
    y = np.full(n, -n / 4.0)
    a = L.certify_dense(prob, y, -1.0)
    b = L.certify_dense(prob, 1e6 * y, -1e6)
    assert a.status == 0 and b.status == 0
    assert b.margin > 1e3 * a.margin


def test_errors():
    n = L.PROOF_MAX_N + 1
    u = np.arange(n - 1, dtype=np.int32)
    prob = L.Problem.maxcut(n, u, u + 1)
    with pytest.raises(L.LrsdpError) as e:
        L.certify_dense(prob, np.zeros(n), 0.0)
    assert e.value.code == L.EUNSUPPORTED
    small = L.Problem.maxcut(4, [0, 1, 2], [1, 2, 3])
    with pytest.raises(L.LrsdpError) as e:
        L.certify_dense(small, np.zeros(4), float("nan"))
    assert e.value.code == L.EINVAL
    y = np.zeros(4)
    y[2] = np.inf
    with pytest.raises(L.LrsdpError) as e:
        L.certify_dense(small, y, 0.0)
    assert e.value.code == L.EINVAL
    with pytest.raises(ValueError):
        L.certify_dense(small, np.zeros(3), 0.0)
