"""Pins of the warm-start oracle: features against vectorised re-derivations on
a tiny graph, the MLP gradient against central finite differences, Adam
against its closed form on the first step, and the label identity
y*_i = (C X*)_ii on a solved instance (t_i in [-2, 2])."""

import numpy as np

from oracle import mlp
from oracle.alm import Options, alm_solve
from oracle.problem import maxcut_problem
from synth import chung_lu_edges, erdos_renyi_edges, init_factor, pm1_weights


def test_features_small_graph_by_hand():
    # path 0-1-2 plus edge 1-3 with weights (2, -1, 3); node 4 isolated
    u = [0, 1, 1]
    v = [1, 2, 3]
    w = [2.0, -1.0, 3.0]
    F = mlp.features(5, u, v, w)
    d = np.array([1, 3, 1, 1, 0.0])
    # node 1: neighbours 0, 2, 3 with weights 2, -1, 3
    assert np.isclose(F[1, 0], np.log(4))
    assert np.isclose(F[1, 1], (2 - 1 + 3) / 6)
    assert np.isclose(F[1, 2], np.log(7))
    assert np.isclose(F[1, 3], np.log(2))               # all neighbours have degree 1
    assert np.isclose(F[1, 4], 0.0)
    bal = np.array([1.0, 4 / 6, -1.0, 1.0, 0.0])
    assert np.isclose(F[1, 5], (2 * bal[0] - 1 * bal[2] + 3 * bal[3]) / 3)
    assert np.isclose(F[1, 6], 0.5)
    assert np.isclose(F[1, 10], 4 / 3)
    assert np.isclose(F[1, 14], np.mean([1 / 4, 1 / 4, 1 / 4]))
    assert np.isclose(F[0, 13], np.log(4) - np.log(2))
    assert np.all(F[4, [3, 4, 5, 6, 10, 13, 14]] == 0) and F[4, 15] == 1
    assert np.allclose(F[:, 11], np.log(5) / 20)
    # dbar = 2|E|/n = 6/5: column 7 is log(1 + d_i/dbar), 8 is 1/(1 + d_i), 9 is a_i/max(d_i, 1)
    # (a_i = sum_j |w_ij| = 2, 6, 1, 3, 0), 12 is log(1 + dbar)
    assert np.allclose(F[:, 7], np.log([1 + 1 / 1.2, 1 + 3 / 1.2, 1 + 1 / 1.2, 1 + 1 / 1.2, 1.0]), rtol=1e-15)
    assert np.allclose(F[:, 8], [0.5, 0.25, 0.5, 0.5, 1.0], rtol=0, atol=0)
    assert np.allclose(F[:, 9], [2.0, 2.0, 1.0, 3.0, 0.0], rtol=0, atol=0)
    assert np.allclose(F[:, 12], np.log(2.2), rtol=1e-15)


def test_mlp_gradient_central_differences():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((7, mlp.NF))
    T = rng.standard_normal((7, mlp.NO))
    theta = mlp.init_params(3) + 0.1 * rng.standard_normal(mlp.NPARAM)
    g = mlp.loss_grad(theta, X, T)
    h = 1e-6
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        fd = (mlp.loss(theta + e, X, T) - mlp.loss(theta - e, X, T)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k]))


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, 0.01)
    assert np.allclose(th[:3], -0.01 * np.sign(g[:3]), rtol=1e-4)
    assert th[3] == 0.0


def test_labels_match_optimality_identity():
    # at a solved point y_i = (C X)_ii = R_i . (C R)_i, so t_i lies in [-2, 2]
    n, m = 60, 200
    u, v = erdos_renyi_edges(n, m, 3)
    w = pm1_weights(m, 4)
    prob = maxcut_problem(n, u, v, w)
    res = alm_solve(prob, init_factor(n, 8, 5), opts=Options(tol=1e-8))
    CR = prob.C @ res.R
    assert np.allclose(res.y, np.sum(res.R * CR, axis=1), atol=1e-5)
    absdeg = np.bincount(np.concatenate([u, v]), weights=np.abs(np.concatenate([w, w])), minlength=n)
    t = mlp.targets_from_solution(res.y, absdeg)
    assert np.all(np.abs(t) <= 2.0 + 1e-6)
    assert np.allclose(mlp.multipliers_from_output(np.stack([t, 0 * t], 1), absdeg), res.y, atol=1e-12)


def test_features_power_law_sane():
    u, v = chung_lu_edges(500, 2000, 2.5, 1)
    F = mlp.features(500, u, v)
    assert F.shape == (500, 16) and np.all(np.isfinite(F))
    deg = np.bincount(np.concatenate([u, v]), minlength=500)
    assert np.all(F[deg > 0, 1] == 1.0)           # unit weights: balance 1
    assert np.all(F[deg == 0, 1] == 0.0)


def test_bfloat16_rounding_by_hand():
    # bfloat16 keeps 8 significand bits: around 1 the spacing is 2^-7
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, 1 + 2 ** -9, -2.5,
                  2.0 ** 100 * (1 + 2 ** -8), -(2.0 ** -100) * (1 + 3 * 2 ** -8)], dtype=np.float32)
    got = mlp.to_bfloat16(x)
    # 1 + 2^-8 is a tie: to even (1); 1 + 3 2^-8 is a tie between 1 + 2^-7 (odd last bit) and
    # 1 + 2^-6 (even); just above the tie rounds up; below it rounds down; ties at other scales alike
    want = [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, 1.0, -2.5, 2.0 ** 100, -(2.0 ** -100) * (1 + 2 ** -6)]
    assert np.array_equal(got, want)


def test_warm_start_limits():
    out = np.array([[3.0, 0.5], [-2.5, 4.0], [1.0, -9.0]])
    absdeg = np.array([4.0, 8.0, 2.0])
    # t limited to [-2, 2]: (2, -2, 1) -> y0 = -t a / 4 = (-2, 4, -0.5)
    assert np.array_equal(mlp.multipliers_from_output(out, absdeg), [-2.0, 4.0, -0.5])
    # mean second output = -1.5: inside [-2, 1] it stays, [-1, 1] lifts it to -1; half of it
    # on the log scale: sigma0 = 10 exp(-0.75) and 10 exp(-0.5)
    assert np.isclose(mlp.initial_penalty(out, 10.0, -2.0, 1.0), 10.0 * np.exp(-0.75))
    assert np.isclose(mlp.initial_penalty(out, 10.0, -1.0, 1.0), 10.0 * np.exp(-0.5))
    assert np.isclose(mlp.sigma_label(40.0, 10.0), np.log(4.0))
