"""Pins of the oracle's problem data, linear maps, gradient and line search.

Each check compares the oracle against something other than itself: dense brute
force built from the definitions, algebraic identities (Laplacian quadratic form,
adjointness), central finite differences, or direct evaluation of the Lagrangian.
"""

import numpy as np
import pytest

from oracle import kernels as K
from oracle.problem import completion_problem, laplacian, maxcut_problem
from synth import erdos_renyi_edges, completion_instance, pm1_weights


def small_maxcut(n=12, m=30, seed=3, signed=False):
    u, v = erdos_renyi_edges(n, m, seed)
    w = pm1_weights(m, seed + 1) * np.linspace(0.5, 2.0, m) if signed else None
    return n, u, v, w, maxcut_problem(n, u, v, w)


def dense_constraints(prob):
    """Dense A_k built from the problem's defining entries (for brute force)."""
    mats = np.zeros((prob.m, prob.n, prob.n))
    Ab = prob.Abar.tocoo()
    for k, p, val in zip(Ab.row, Ab.col, Ab.data):
        mats[k, prob.col_a[p], prob.col_b[p]] += val
    return mats


# --------------------------------------------------------------------------- build
def test_laplacian_quadratic_form_identity():
    # x^T L x = sum_edges w (x_u - x_v)^2, L 1 = 0 (Laplacian definition, MaxCut section)
    n, u, v, w, _ = small_maxcut(signed=True)
    L = laplacian(n, u, v, w).toarray()
    x = np.random.default_rng(0).standard_normal(n)
    assert np.isclose(x @ L @ x, np.sum(w * (x[u] - x[v]) ** 2), rtol=1e-13)
    assert np.allclose(L @ np.ones(n), 0.0, atol=1e-13)
    assert np.allclose(L, L.T)


def test_maxcut_objective_is_minus_cut_weight():
    # For a +-1 side vector s, <C, s s^T> = -cut(s): the min-form objective
    n, u, v, w, prob = small_maxcut(signed=True)
    rng = np.random.default_rng(1)
    for _ in range(5):
        s = rng.choice([-1.0, 1.0], n)
        cut = float(np.sum(w[s[u] != s[v]]))
        assert np.isclose(prob.objective(s[:, None]), -cut, rtol=1e-13, atol=1e-13)


def test_maxcut_constraint_map_brute_force():
    n, u, v, w, prob = small_maxcut()
    R = np.random.default_rng(2).standard_normal((n, 4))
    X = R @ R.T
    mats = dense_constraints(prob)
    expect = np.einsum("kab,ab->k", mats, X)
    assert np.allclose(prob.A_of(R), expect, rtol=1e-13, atol=1e-13)
    assert np.allclose(expect, np.diag(X))          # A(X) = diag(X) for MaxCut
    assert np.allclose(prob.b, 1.0)


def test_completion_constraint_map_brute_force():
    n1, n2 = 7, 5
    i, j, Mij, U, V = completion_instance(n1, n2, 2, 3, seed=4)
    prob = completion_problem(n1, n2, i, j, Mij)
    R = np.random.default_rng(3).standard_normal((n1 + n2, 3))
    X = R @ R.T
    mats = dense_constraints(prob)
    expect = np.einsum("kab,ab->k", mats, X)
    assert np.allclose(prob.A_of(R), expect, rtol=1e-13, atol=1e-13)
    assert np.allclose(expect, 2.0 * X[i, n1 + j])
    # planted M is feasible: R = [U; V] reproduces b
    assert np.allclose(prob.A_of(np.vstack([U, V])), prob.b, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kind", ["maxcut", "completion"])
def test_adjoint_identity(kind):
    # <A*(y), Z> = <y, A(Z)> for symmetric Z = U V^T + V U^T
    if kind == "maxcut":
        prob = small_maxcut(signed=True)[-1]
    else:
        i, j, Mij, _, _ = completion_instance(6, 6, 2, 3, seed=5)
        prob = completion_problem(6, 6, i, j, Mij)
    rng = np.random.default_rng(4)
    U = rng.standard_normal((prob.n, 3))
    V = rng.standard_normal((prob.n, 3))
    y = rng.standard_normal(prob.m)
    Z = U @ V.T + V @ U.T
    lhs = np.sum(prob.A_adj(y).toarray() * Z)
    rhs = y @ (prob.A_of(U, V) + prob.A_of(V, U))
    assert np.isclose(lhs, rhs, rtol=1e-12)


@pytest.mark.parametrize("kind", ["maxcut", "completion"])
def test_spmm_brute_force(kind):
    if kind == "maxcut":
        n, u, v, w, prob = small_maxcut(signed=True)
        L = np.zeros((n, n))
        for a, b_, ww in zip(u, v, w):       # Laplacian straight from its definition
            L[a, b_] -= ww
            L[b_, a] -= ww
            L[a, a] += ww
            L[b_, b_] += ww
        Cd = -L / 4.0
    else:
        n1, n2 = 6, 8
        i, j, Mij, _, _ = completion_instance(n1, n2, 2, 4, seed=6)
        prob = completion_problem(n1, n2, i, j, Mij)
        Cd = np.eye(n1 + n2)
    mats = dense_constraints(prob)
    rng = np.random.default_rng(5)
    ytil = rng.standard_normal(prob.m)
    V = rng.standard_normal((prob.n, 5))
    S = Cd - np.einsum("k,kab->ab", ytil, mats)
    assert np.allclose(K.spmm(prob, ytil, V), S @ V, rtol=1e-13, atol=1e-13)
    assert np.allclose(K.spmm(prob, None, V), Cd @ V, rtol=1e-13, atol=1e-13)


# --------------------------------------------------------------------------- gradient
@pytest.mark.parametrize("kind", ["maxcut", "completion"])
def test_gradient_central_differences(kind):
    if kind == "maxcut":
        prob = small_maxcut(n=10, m=20, signed=True)[-1]
    else:
        i, j, Mij, _, _ = completion_instance(5, 6, 2, 3, seed=7)
        prob = completion_problem(5, 6, i, j, Mij)
    rng = np.random.default_rng(6)
    R = rng.standard_normal((prob.n, 3))
    y = rng.standard_normal(prob.m)
    sigma = 1.7
    G = K.gradient(prob, R, y, sigma)
    h = 1e-6
    Gfd = np.zeros_like(R)
    for a in range(R.shape[0]):
        for c in range(R.shape[1]):
            Rp = R.copy(); Rp[a, c] += h
            Rm = R.copy(); Rm[a, c] -= h
            Gfd[a, c] = (K.lagrangian(prob, Rp, y, sigma) - K.lagrangian(prob, Rm, y, sigma)) / (2 * h)
    assert np.max(np.abs(G - Gfd)) <= 1e-6 * max(1.0, np.max(np.abs(G)))
    # gradient = 2 (C - A*(ytil)) R with ytil the multiplier estimate
    ytil = K.multiplier_estimate(prob, R, y, sigma)
    assert np.allclose(G, 2.0 * K.spmm(prob, ytil, R), rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------- line search
@pytest.mark.parametrize("kind", ["maxcut", "completion"])
def test_quartic_identity(kind):
    # L(R + tau D) - L(R) = a1 tau^4 + a2 tau^3 + a3 tau^2 + a4 tau (appendix A.2)
    if kind == "maxcut":
        prob = small_maxcut(signed=True)[-1]
    else:
        i, j, Mij, _, _ = completion_instance(6, 7, 2, 4, seed=8)
        prob = completion_problem(6, 7, i, j, Mij)
    rng = np.random.default_rng(7)
    R = rng.standard_normal((prob.n, 3))
    D = rng.standard_normal((prob.n, 3))
    y = rng.standard_normal(prob.m)
    sigma = 2.3
    c = K.linesearch_coeffs(prob, R, D, y, sigma)
    L0 = K.lagrangian(prob, R, y, sigma)
    scale = abs(L0) + 1.0
    for tau in (-1.3, 0.4, 2.0, 1e-3):
        direct = K.lagrangian(prob, R + tau * D, y, sigma) - L0
        poly = K.quartic((c["a1"], c["a2"], c["a3"], c["a4"]), tau)
        assert abs(direct - poly) <= 1e-12 * scale * (1 + tau ** 4)
    # a4 is the directional derivative <grad, D>
    G = K.gradient(prob, R, y, sigma)
    assert np.isclose(c["a4"], np.sum(G * D), rtol=1e-12, atol=1e-12)


def test_maxcut_a1_closed_form():
    # MaxCut: q2_i = ||D_i||^2, so a1 = sigma/2 sum_i ||D_i||^4
    prob = small_maxcut()[-1]
    rng = np.random.default_rng(8)
    R = rng.standard_normal((prob.n, 4))
    D = rng.standard_normal((prob.n, 4))
    c = K.linesearch_coeffs(prob, R, D, np.zeros(prob.n), 3.0)
    assert np.isclose(c["a1"], 1.5 * np.sum(np.sum(D * D, axis=1) ** 2), rtol=1e-13)


def test_exact_step_matches_grid_minimum():
    rng = np.random.default_rng(9)
    for trial in range(200):
        a1 = abs(rng.standard_normal()) + 1e-3
        a2, a3 = rng.standard_normal(2) * 2
        a4 = -abs(rng.standard_normal()) - 1e-3     # descent: f'(0) < 0
        tau = K.exact_step(a1, a2, a3, a4)
        assert tau > 0
        # f' vanishes at tau and tau is the best point on a fine grid of [0, 4 tau]
        fp = ((4 * a1 * tau + 3 * a2) * tau + 2 * a3) * tau + a4
        assert abs(fp) <= 1e-9 * (1 + abs(a4) + abs(a3) * tau + abs(a2) * tau ** 2 + a1 * tau ** 3)
        grid = np.linspace(0, 4 * tau + 10, 200001)
        fg = K.quartic((a1, a2, a3, a4), grid)
        assert K.quartic((a1, a2, a3, a4), tau) <= fg.min() + 1e-9 * (1 + abs(fg.min()))


def test_exact_step_special_cases():
    # quadratic (a1 = a2 = 0): tau = -a4 / (2 a3)
    assert np.isclose(K.exact_step(0.0, 0.0, 2.0, -3.0), 0.75)
    # not a descent direction: no positive step lowers the quartic
    assert K.exact_step(1.0, 0.0, 1.0, 0.5) == 0.0
    assert K.exact_step(0.0, 0.0, 0.0, 0.0) == 0.0
    # two local minima: picks the deeper one (f(t)=t^4-4t^3+4t^2-0.1t has minima near 0 and 2)
    t = K.exact_step(1.0, -4.0, 4.0, -0.1)
    assert t > 1.5


# --------------------------------------------------------------------------- measures by hand
def test_alm_measures_by_hand_maxcut():
    # Path 0-1-2 with unit weights: C = -L/4 = [[-1/4, 1/4, 0], [1/4, -1/2, 1/4], [0, 1/4, -1/4]].
    # R = [[1, 0], [0, 1], [1, 1]] gives X = RR^T = [[1, 0, 1], [0, 1, 1], [1, 1, 2]], so
    # <C, X> = (-1/4 - 1/2 - 2/4) + 2 (1/4 * 0 + 1/4 * 1 + 0 * 1) = -3/4 and
    # A(X) - b = diag(X) - 1 = (0, 0, 1).  With y = (1/2, -1, 2), b^T y = 3/2.
    # Error measures of the experimental setting: err1 = ||res|| / (1 + ||b||_1) = 1/4,
    # the infinity-norm variant 1 / (1 + 1) = 1/2, err3 = (-3/4 - 3/2) / (1 + 3/4 + 3/2) = -9/13.
    prob = maxcut_problem(3, [0, 1], [1, 2])
    R = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    y = np.array([0.5, -1.0, 2.0])
    m = K.alm_measures(prob, R, y)
    assert m["obj"] == -0.75
    assert m["res_norm"] == 1.0
    assert m["dual"] == 1.5
    assert m["err1"] == 0.25
    assert m["err1_inf"] == 0.5
    assert np.isclose(m["err3"], -9.0 / 13.0, rtol=1e-15)


def test_alm_measures_by_hand_completion():
    # n1 = n2 = 2, samples (0,0) M = 1.5, (1,1) M = -0.5, (0,1) M = 2, so b = (3, -1, 4).
    # Rows of R: top block R0 = (1, 2), R1 = (0, 1); bottom block R2 = (1, -1), R3 = (2, 0).
    # <I, RR^T> = ||R||_F^2 = 5 + 1 + 2 + 4 = 12; A(RR^T)_k = 2 R_i . R_{n1+j} = (-2, 0, 4);
    # res = (-5, 1, 0), ||res|| = sqrt(26), ||b||_1 = 8, ||b||_inf = 4.
    # y = (1, -2, 1/2): b^T y = 3 + 2 + 2 = 7, err3 = (12 - 7) / (1 + 12 + 7) = 1/4.
    prob = completion_problem(2, 2, [0, 1, 0], [0, 1, 1], [1.5, -0.5, 2.0])
    R = np.array([[1.0, 2.0], [0.0, 1.0], [1.0, -1.0], [2.0, 0.0]])
    y = np.array([1.0, -2.0, 0.5])
    m = K.alm_measures(prob, R, y)
    assert m["obj"] == 12.0
    assert np.allclose(K.constraint_map(prob, R), [-2.0, 0.0, 4.0], rtol=0, atol=0)
    assert np.isclose(m["res_norm"], np.sqrt(26.0), rtol=1e-15)
    assert m["dual"] == 7.0
    assert np.isclose(m["err1"], np.sqrt(26.0) / 9.0, rtol=1e-15)
    assert np.isclose(m["err1_inf"], np.sqrt(26.0) / 5.0, rtol=1e-15)
    assert m["err3"] == 0.25
