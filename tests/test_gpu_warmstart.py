"""GPU parity of the learned warm start against the FP64 oracle (oracle/mlp.py):
features, MLP forward, gradient (float32 kernels, float64 oracle: 1e-4
norm-wise), Adam, the multiplier prediction, and the gain of a trained model
over the cold start on a held-out graph."""

import numpy as np
import pytest

from oracle import mlp
from synth import chung_lu_edges, erdos_renyi_edges, init_factor, pm1_weights

from paper_2407_15049_amd import lrsdp as L
from paper_2407_15049_amd import warmstart as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return L.Context(0)


def graph(case):
    if case == "pm1":
        u, v = erdos_renyi_edges(777, 3001, 3)
        return 777, u, v, pm1_weights(3001, 4)
    if case == "cl":
        u, v = chung_lu_edges(5000, 20000, 2.5, 7)
        return 5000, u, v, None
    if case == "general":
        u, v = erdos_renyi_edges(501, 2000, 5)
        return 501, u, v, np.random.default_rng(6).uniform(-2, 3, 2000)
    if case == "isolated":
        u, v = erdos_renyi_edges(100, 400, 8)
        return 300, u, v, None
    raise KeyError(case)


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).cuda()


@pytest.mark.parametrize("case", ["pm1", "cl", "general", "isolated"])
def test_features_parity(ctx, case):
    import torch
    n, u, v, w = graph(case)
    print("CASE", dict(test="features", case=case), flush=True)
    prob = L.Problem.maxcut(n, u, v, w).upload(ctx)
    feat = torch.empty((n, 16), dtype=torch.float32, device="cuda")
    stats = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    L.ws_features(ctx, prob, feat, stats)
    torch.cuda.synchronize()
    F = feat.cpu().double().numpy()
    Fo = mlp.features(n, u, v, w)
    assert np.allclose(F, Fo, rtol=2e-5, atol=2e-5), np.max(np.abs(F - Fo))


@pytest.mark.parametrize("n", [37, 1000, 20011])
def test_forward_and_gradient_parity(ctx, n):
    import torch
    print("CASE", dict(test="mlp", n=n), flush=True)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 16)).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((n, 2)).astype(np.float32).astype(np.float64)
    theta = (mlp.init_params(5) + 0.2 * rng.standard_normal(mlp.NPARAM)).astype(np.float32).astype(np.float64)
    Xd, Td, Pd = dev(X, torch.float32), dev(T, torch.float32), dev(theta, torch.float32)
    out = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    L.mlp_forward(ctx, Pd, Xd, out)
    grad = torch.empty(mlp.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = torch.empty(256 * (mlp.NPARAM + 1), dtype=torch.float32, device="cuda")
    L.mlp_grad(ctx, Pd, Xd, Td, grad, loss, work)
    torch.cuda.synchronize()
    ref_out, _ = mlp.forward(theta, X)
    assert np.allclose(out.cpu().double().numpy(), ref_out, rtol=1e-4, atol=1e-5)
    g = grad.cpu().double().numpy()
    go = mlp.loss_grad(theta, X, T)
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], mlp.unpack(g).values(), mlp.unpack(go).values()):
        assert np.linalg.norm(a - b) <= 2e-4 * max(np.linalg.norm(b), 1e-6), name
    assert abs(loss.item() - mlp.loss(theta, X, T)) <= 1e-5 * mlp.loss(theta, X, T)
    # deterministic
    grad2 = torch.empty_like(grad)
    L.mlp_grad(ctx, Pd, Xd, Td, grad2, loss, work)
    torch.cuda.synchronize()
    assert torch.equal(grad, grad2)


def test_adam_parity(ctx):
    import torch
    rng = np.random.default_rng(1)
    th = rng.standard_normal(mlp.NPARAM).astype(np.float32).astype(np.float64)
    g1 = rng.standard_normal(mlp.NPARAM).astype(np.float32).astype(np.float64)
    g2 = rng.standard_normal(mlp.NPARAM).astype(np.float32).astype(np.float64)
    Pd, md, vd = dev(th, torch.float32), torch.zeros(mlp.NPARAM, device="cuda"), torch.zeros(mlp.NPARAM, device="cuda")
    for step, g in [(1, g1), (2, g2)]:
        L.mlp_adam(ctx, Pd, md, vd, dev(g, torch.float32), step, 1e-2)
    torch.cuda.synchronize()
    t, m, v = th, np.zeros_like(th), np.zeros_like(th)
    for step, g in [(1, g1), (2, g2)]:
        t, m, v = mlp.adam(t, m, v, g, step, 1e-2)
    assert np.allclose(Pd.cpu().double().numpy(), t, rtol=1e-5, atol=1e-6)


def test_warmstart_prediction_formula(ctx):
    import torch
    n, u, v, w = graph("pm1")
    prob = L.Problem.maxcut(n, u, v, w).upload(ctx)
    theta = (mlp.init_params(9) + 0.1).astype(np.float32).astype(np.float64)
    y0, sigma0 = W.warm_start(ctx, prob, dev(theta, torch.float32))
    torch.cuda.synchronize()
    F = mlp.features(n, u, v, w).astype(np.float32).astype(np.float64)
    out, _ = mlp.forward(theta, F)
    absdeg = np.bincount(np.concatenate([u, v]), weights=np.abs(np.concatenate([w, w])), minlength=n)
    assert np.allclose(y0.cpu().numpy(), mlp.multipliers_from_output(out, absdeg), rtol=1e-4, atol=1e-5)
    from oracle.problem import maxcut_problem
    base = 4.0 * maxcut_problem(n, u, v, w).c_l1 / n
    assert np.isclose(sigma0, base * np.exp(out[:, 1].mean()), rtol=1e-4)


def test_trained_warm_start_gains(ctx):
    """Train on a few small graphs; on a held-out graph the warm start needs fewer
    L-BFGS iterations than the cold start (parity unpinned: an empirical check)."""
    import torch
    specs = [s for s in W.TRAIN_SPECS if s[1] <= 60000][:6]
    data = W.make_training_set(ctx, specs, rank=12, log=print)
    params, hist = W.train(ctx, data, steps=200, lr=3e-3, log=print)
    assert hist[-1][1] < 0.5 * hist[0][1]
    n = 80000
    u, v = chung_lu_edges(n, n * 5, 2.5, 424242)
    w = pm1_weights(n * 5, 424243)
    prob = L.Problem.maxcut(n, u, v, w).upload(ctx)
    y0, sigma0 = W.warm_start(ctx, prob, params)
    R0 = init_factor(n, 12, 5)
    res = {}
    for mode in ["cold", "warm"]:
        opts = L.default_options(prec=L.F32, rank=12, ld=12)
        y = torch.zeros(n, dtype=torch.float64, device="cuda")
        if mode == "warm":
            y.copy_(y0)
            opts.sigma0 = sigma0
        R = torch.from_numpy(R0.astype(np.float32)).cuda()
        rc, r = L.solve(ctx, prob, R, y, opts)
        res[mode] = r
        print(mode, r.as_dict())
        assert rc == L.OK
    assert res["warm"].inner < res["cold"].inner


def test_warmstart_non_finite_falls_back_to_cold(ctx):
    import torch
    n, u, v, w = graph("pm1")
    prob = L.Problem.maxcut(n, u, v, w).upload(ctx)
    theta = mlp.init_params(9).astype(np.float32)
    theta[mlp.NPARAM - 2] = np.nan          # b3[0]: every t_i becomes NaN, log-penalty stays finite
    y0, sigma0 = W.warm_start(ctx, prob, dev(theta))
    torch.cuda.synchronize()
    assert sigma0 == 0.0 and torch.count_nonzero(y0).item() == 0
    with pytest.raises(L.LrsdpError) as e:
        L.warmstart(ctx, prob, dev(theta), torch.empty(22 * n, dtype=torch.float32, device="cuda"),
                    torch.empty(n, dtype=torch.float64, device="cuda"))
    assert e.value.code == L.ENUMERIC
