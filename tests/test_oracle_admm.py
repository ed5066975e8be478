"""Pins of the oracle's splitting (ADMM) phase: the CG solve of eq. 2.2 makes
the U-gradient of the splitting Lagrangian vanish (central differences), the
MaxCut operator is block diagonal so a per-row Sherman-Morrison solve gives the
same U, and a converged splitting point is feasible and matches the ALM
objective on a graph whose optimum is known in closed form."""

import numpy as np

from oracle import kernels as K
from oracle.alm import Options, admm_phase, admm_step, alm_solve, cg, split_operator, split_rhs
from oracle.problem import completion_problem, maxcut_problem
from synth import completion_instance, erdos_renyi_edges, init_factor, pm1_weights


def split_lagrangian(prob, U, V, y, sigma):
    q0 = prob.b - prob.A_of(U, V)
    return prob.objective(U, V) + y @ q0 + 0.5 * sigma * q0 @ q0 + 0.5 * sigma * np.sum((U - V) ** 2)


def test_u_step_zeroes_gradient():
    for prob in [maxcut_problem(15, *erdos_renyi_edges(15, 40, 2), pm1_weights(40, 3)),
                 completion_problem(6, 7, *completion_instance(6, 7, 2, 4, seed=1)[:3])]:
        rng = np.random.default_rng(4)
        U = rng.standard_normal((prob.n, 3))
        V = rng.standard_normal((prob.n, 3))
        y = rng.standard_normal(prob.m)
        sigma = 1.7
        Us, _ = cg(split_operator(prob, V, sigma), split_rhs(prob, V, y, sigma), U, 1e-13, 2000)
        h = 1e-6
        for (a, c) in [(0, 0), (3, 1), (prob.n - 1, 2)]:
            E = np.zeros_like(U)
            E[a, c] = h
            fd = (split_lagrangian(prob, Us + E, V, y, sigma) - split_lagrangian(prob, Us - E, V, y, sigma)) / (2 * h)
            assert abs(fd) <= 1e-6 * (1 + np.abs(Us).max())


def test_maxcut_row_solve_equals_cg():
    n, m = 20, 60
    u, v = erdos_renyi_edges(n, m, 5)
    prob = maxcut_problem(n, u, v, pm1_weights(m, 6))
    rng = np.random.default_rng(7)
    V = rng.standard_normal((n, 4))
    y = rng.standard_normal(n)
    sigma = 2.3
    B = split_rhs(prob, V, y, sigma)
    Ucg, _ = cg(split_operator(prob, V, sigma), B, np.zeros_like(V), 1e-14, 500)
    # (sigma (v v^T + I)) u = b per row, by Sherman-Morrison
    vb = np.sum(V * B, axis=1)
    vv = np.sum(V * V, axis=1)
    Usm = (B - (vb / (1 + vv))[:, None] * V) / sigma
    assert np.allclose(Ucg, Usm, rtol=1e-10, atol=1e-12)
    # and B itself is -C V + (y + 2 sigma) V for MaxCut
    assert np.allclose(B, -(prob.C @ V) + (y + 2 * sigma)[:, None] * V)


def test_splitting_converges_on_odd_cycle():
    n = 9
    u = np.arange(n)
    v = (u + 1) % n
    prob = maxcut_problem(n, u, v)
    warm = alm_solve(prob, init_factor(n, 3, 1), opts=Options(tol=1e-3))
    R, U, V, y, meas, it = admm_phase(prob, warm.R, warm.y, warm.sigma, tol=1e-8, max_iter=5000)
    assert meas["err1"] <= 1e-8 and abs(meas["err3"]) <= 1e-8
    assert np.isclose(meas["obj"], -(n / 2) * (1 + np.cos(np.pi / n)), rtol=1e-6)
    assert np.linalg.norm(U - V) <= 1e-5 * np.linalg.norm(U)


def test_phase2_fallback_reproduces_alm_only():
    # a splitting phase that cannot finish (max_admm = 10 from an early switch)
    # is abandoned: the solve then equals the ALM alone, iterate for iterate
    from oracle.alm import Options, alm_solve
    from oracle.problem import maxcut_problem
    from synth import erdos_renyi_edges, init_factor
    n = 120
    u, v = erdos_renyi_edges(n, 500, 7)
    prob = maxcut_problem(n, u, v)
    R0 = init_factor(n, 8, 9)
    a = alm_solve(prob, R0, opts=Options())
    b = alm_solve(prob, R0, opts=Options(phase2=True, switch_err1=1e-1, max_admm=10, admm_check=10))
    assert b.admm_fallbacks == 1 and b.admm_iters == 10
    assert np.array_equal(a.R, b.R) and np.array_equal(a.y, b.y)
    assert a.obj == b.obj and a.outer == b.outer and a.inner == b.inner
