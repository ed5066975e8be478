"""Pins of the oracle's L-BFGS direction (Algorithm 1).

* On a strictly convex quadratic with exact line search, L-BFGS with H0 = I and
  any memory T >= 1 produces the conjugate-gradient iterates (Nocedal & Wright,
  Thm. on L-BFGS/CG equivalence for quadratics).
* The two-loop matrix H satisfies the secant condition H y_k = s_k for the newest
  pair, and H is symmetric positive definite when every <y_t, s_t> > 0.
"""

import numpy as np
import pytest

from oracle.lbfgs import two_loop


def spd(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q @ np.diag(np.linspace(1.0, 30.0, n)) @ Q.T, rng.standard_normal(n)


def cg_iterates(A, b, x0, k):
    x = x0.copy()
    r = b - A @ x
    p = r.copy()
    out = [x.copy()]
    for _ in range(k):
        Ap = A @ p
        alpha = (r @ r) / (p @ Ap)
        x = x + alpha * p
        rn = r - alpha * Ap
        p = rn + (rn @ rn) / (r @ r) * p
        r = rn
        out.append(x.copy())
    return out


@pytest.mark.parametrize("T", [1, 2, 4])
def test_lbfgs_equals_cg_on_quadratic(T):
    A, b = spd(30, 11)
    x = np.zeros(30)
    grad = lambda z: A @ z - b
    ref = cg_iterates(A, b, x, 12)
    pairs = []
    g = grad(x)
    for k in range(12):
        d = two_loop(g, pairs)
        tau = -(g @ d) / (d @ A @ d)           # exact step on the quadratic
        xn = x + tau * d
        gn = grad(xn)
        pairs.append((tau * d, gn - g))
        if len(pairs) > T:
            pairs.pop(0)
        x, g = xn, gn
        assert np.allclose(x, ref[k + 1], rtol=1e-9, atol=1e-9)


def test_secant_condition_and_spd():
    rng = np.random.default_rng(3)
    n = 15
    A, _ = spd(n, 4)
    pairs = []
    for _ in range(4):
        s = rng.standard_normal(n)
        pairs.append((s, A @ s))
    s_new, y_new = pairs[-1]
    # two_loop returns -H g; the secant condition gives H y_new = s_new
    assert np.allclose(-two_loop(y_new, pairs), s_new, rtol=1e-10, atol=1e-10)
    H = np.stack([-two_loop(e, pairs) for e in np.eye(n)], axis=1)
    assert np.allclose(H, H.T, atol=1e-10)
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > 0


def test_empty_memory_is_steepest_descent():
    g = np.arange(6.0)
    assert np.array_equal(two_loop(g, []), -g)


def pcg_iterates(A, b, x0, Minv, k):
    """Preconditioned conjugate gradients (Minv applies M^{-1}), textbook form."""
    x = x0.copy()
    r = b - A @ x
    z = Minv(r)
    p = z.copy()
    out = [x.copy()]
    for _ in range(k):
        Ap = A @ p
        a = (r @ z) / (p @ Ap)
        x = x + a * p
        rn = r - a * Ap
        zn = Minv(rn)
        p = zn + ((rn @ zn) / (r @ z)) * p
        r, z = rn, zn
        out.append(x.copy())
    return out


@pytest.mark.parametrize("T", [1, 2, 4])
def test_lbfgs_with_fixed_h0_equals_pcg(T):
    # with a fixed SPD H0 = M^{-1} and exact steps, L-BFGS iterates are the
    # preconditioned CG iterates (the same argument as for H0 = I)
    A, b = spd(30, 12)
    rng = np.random.default_rng(13)
    Q = rng.standard_normal((30, 30))
    M = Q @ Q.T / 30 + np.diag(rng.uniform(0.5, 3.0, 30))
    Minv = lambda v: np.linalg.solve(M, v)
    x = np.zeros(30)
    ref = pcg_iterates(A, b, x, Minv, 12)
    pairs = []
    g = A @ x - b
    for k in range(12):
        d = two_loop(g, pairs, Minv)
        tau = -(g @ d) / (d @ A @ d)
        xn = x + tau * d
        gn = A @ xn - b
        pairs.append((tau * d, gn - g))
        if len(pairs) > T:
            pairs.pop(0)
        x, g = xn, gn
        assert np.allclose(x, ref[k + 1], rtol=1e-8, atol=1e-8)


def test_row_block_h0_inverts_the_row_blocks():
    # P_i (P_i^{-1} q_i) = q_i with P_i = h_i I + 4 sigma R_i R_i^T formed explicitly
    from oracle.alm import row_block_h0
    from oracle.problem import maxcut_problem
    from synth import chung_lu_edges, init_factor
    u, v = chung_lu_edges(300, 1200, 2.3, 5)
    prob = maxcut_problem(340, u, v)                   # 40 isolated nodes: the floor of h
    R = init_factor(340, 6, 6) * np.random.default_rng(7).uniform(0.5, 1.5, (340, 1))
    sigma = 3.7
    Q = np.random.default_rng(8).standard_normal((340, 6))
    Z = row_block_h0(prob, R, sigma)(Q)
    rowabs = np.asarray(abs(prob.C).sum(axis=1)).ravel()
    h = 2.0 * np.maximum(rowabs, 1e-3 * prob.c_l1 / prob.n)
    for i in range(340):
        P = h[i] * np.eye(6) + 4 * sigma * np.outer(R[i], R[i])
        assert np.allclose(P @ Z[i], Q[i], rtol=1e-12, atol=1e-12)


def test_preconditioned_solve_reaches_the_same_optimum():
    # er_1k at rank 16 has a certified optimum; both H0 choices reach it
    from oracle.alm import Options, alm_solve
    from oracle.problem import maxcut_problem
    from synth import erdos_renyi_edges, init_factor
    u, v = erdos_renyi_edges(1000, 5000, 15049)
    prob = maxcut_problem(1000, u, v)
    R0 = init_factor(1000, 16, 15051)
    a = alm_solve(prob, R0, opts=Options())
    b = alm_solve(prob, R0, opts=Options(precond=True))
    assert a.converged and b.converged
    assert abs(a.obj - b.obj) <= 2e-5 * abs(a.obj)
    assert b.inner < a.inner
