"""Oracle re-optimisation (Section 4.1) against what the mathematics fixes.

* Scaling identity: the Lagrangian of the problem with alpha C, at multipliers
  alpha y and penalty sigma, is alpha times the Lagrangian of C at multipliers
  y and penalty sigma / alpha; the gradients scale the same way.  This is what
  lets a round's result be stated for the original problem.
* A round stops on err1 alone; the final test recomputes err3 on the original
  problem from scratch (objective <C, RR^T> and b^T y of the returned R, y).
* The strict level also needs err2 <= tol: at a rank-2 stationary point that is
  not optimal (lambda_min(C - A*(y)) clearly negative) it can never hold, so the
  solve reports not converged after max_reopt rounds, while the mild level
  accepts the same point.
"""

import numpy as np
import pytest

from oracle import certify
from oracle import kernels as K
from oracle.alm import Options, _alm_run, alm_solve, scaled_objective
from oracle.problem import completion_problem, maxcut_problem
from synth import chung_lu_edges, completion_instance, erdos_renyi_edges, init_factor, pm1_weights

# The schedule these cases were built on (penalty x2 on a stall, 2000 L-BFGS
# iterations per subproblem, two pairs): which round first meets err3 depends
# on it, and the properties pinned here are those of the re-optimisation logic.
SCHED = dict(sigma_factor=2.0, max_inner=2000, lbfgs_mem=2)


def cl2k():
    u, v = chung_lu_edges(2000, 8000, 2.5, 77)
    return maxcut_problem(2000, u, v, pm1_weights(8000, 3)), init_factor(2000, 8, 5)


@pytest.mark.parametrize("kind", ["maxcut", "completion"])
def test_scaled_lagrangian_identity(kind):
    rng = np.random.default_rng(3)
    if kind == "maxcut":
        u, v = erdos_renyi_edges(80, 300, 4)
        op = maxcut_problem(80, u, v, rng.uniform(-1, 2, 300))
    else:
        i, j, M, _, _ = completion_instance(30, 25, 2, 6, seed=5)
        op = completion_problem(30, 25, i, j, M)
    R = rng.standard_normal((op.n, 5))
    y = rng.standard_normal(op.m)
    sigma, alpha = 3.7, 0.01
    sc = scaled_objective(op, alpha)
    assert sc.c_l1 == pytest.approx(alpha * op.c_l1, rel=1e-14)
    lhs = K.lagrangian(sc, R, alpha * y, sigma)
    rhs = alpha * K.lagrangian(op, R, y, sigma / alpha)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    g1 = K.gradient(sc, R, alpha * y, sigma)
    g2 = alpha * K.gradient(op, R, y, sigma / alpha)
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * np.max(np.abs(g2))
    # the constraint map does not see the scale
    assert np.array_equal(sc.A_of(R), op.A_of(R)) and np.array_equal(sc.b, op.b)


def test_mild_reopt_meets_err3_on_the_original_problem():
    op, R0 = cl2k()
    first = _alm_run(op, R0, None, Options(**SCHED), err1_only=True)
    m0 = K.alm_measures(op, first.R, first.y)
    assert first.converged and m0["err1"] <= 1e-5 and abs(m0["err3"]) > 1e-5   # round 0 alone is not enough
    res = alm_solve(op, R0, opts=Options(**SCHED, reopt=1))
    assert res.converged and res.reopt_rounds >= 1
    m = K.alm_measures(op, res.R, res.y)
    assert m["err1"] <= 1e-5 and abs(m["err3"]) <= 1e-5
    assert res.obj == pytest.approx(m["obj"], rel=1e-13) and res.err3 == pytest.approx(m["err3"], rel=1e-9, abs=1e-15)
    # the first round is the err1-only run itself
    rounds = [h for h in res.history if "met" in h]
    assert rounds[0]["err3_original"] == pytest.approx(m0["err3"], rel=1e-12)
    assert not rounds[0]["met"] and rounds[-1]["met"]
    assert [h["alpha"] for h in rounds] == pytest.approx([0.1 ** k for k in range(len(rounds))], rel=1e-15)


def test_reopt_without_extra_rounds_is_the_err1_only_run():
    u, v = erdos_renyi_edges(1000, 5000, 15049)
    op = maxcut_problem(1000, u, v)
    R0 = init_factor(1000, 10, 15050)
    first = _alm_run(op, R0, None, Options(**SCHED), err1_only=True)
    res = alm_solve(op, R0, opts=Options(**SCHED, reopt=1))
    assert res.reopt_rounds == 0 and res.converged
    assert np.array_equal(res.R, first.R) and np.array_equal(res.y, first.y)
    assert res.outer == first.outer and res.inner == first.inner


def test_strict_reopt_rejects_a_rank_deficient_stationary_point():
    u, v = erdos_renyi_edges(200, 800, 5)
    op = maxcut_problem(200, u, v)
    R0 = init_factor(200, 2, 8)
    mild = alm_solve(op, R0, opts=Options(**SCHED, reopt=1))
    strict = alm_solve(op, R0, opts=Options(**SCHED, reopt=2, max_reopt=3))
    assert mild.converged and mild.reopt_rounds == 0
    assert not strict.converged and strict.reopt_rounds == 3
    lam = certify.lambda_min(op, strict.y)
    assert lam < -0.1
    assert strict.err2 == pytest.approx(-lam / (1 + op.c_l1), rel=1e-9)
    assert strict.err2 > 1e-5
    # first-order stationary all the same: (C - A*(y)) R is tiny
    S = (op.C - op.A_adj(strict.y)).tocsr()
    assert np.linalg.norm(S @ strict.R) <= 1e-4 * np.linalg.norm(S.toarray()) * np.linalg.norm(strict.R)


def test_strict_reopt_accepts_when_lambda_min_is_small():
    op, R0 = cl2k()
    res = alm_solve(op, R0, opts=Options(**SCHED, reopt=2))
    assert res.converged
    assert res.err2 == pytest.approx(certify.err2(op, res.y), rel=1e-9)
    assert res.err2 <= 1e-5
