"""GPU parity of the learned warm start against the FP64 oracle (oracle/mlp.py):
features, MLP forward, gradient (float32 kernels, float64 oracle: 1e-4
norm-wise) with float32 and bfloat16 parameters, Adam, the training entry
point (bfloat16 parameters, float32 master), the labels, the multiplier and
penalty prediction with their limits, and the gain of a trained model over the
cold start on a held-out graph."""

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


@pytest.mark.parametrize("n", [37, 20011])
def test_bf16_forward_and_gradient_parity(ctx, n):
    import torch
    print("CASE", dict(test="mlp-bf16", n=n), flush=True)
    rng = np.random.default_rng(n + 1)
    X = rng.standard_normal((n, 16)).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((n, 2)).astype(np.float32).astype(np.float64)
    theta32 = (mlp.init_params(5) + 0.2 * rng.standard_normal(mlp.NPARAM)).astype(np.float32)
    theta = mlp.to_bfloat16(theta32)                    # the values the bfloat16 storage holds
    Pbf = dev(theta32).to(torch.bfloat16)               # torch's float32 -> bfloat16 is round to nearest even
    assert np.array_equal(Pbf.float().cpu().double().numpy(), theta)
    Xd, Td = dev(X, torch.float32), dev(T, torch.float32)
    out = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    L.mlp_forward(ctx, Pbf, Xd, out)
    grad = torch.empty(mlp.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = torch.empty(256 * (mlp.NPARAM + 1), dtype=torch.float32, device="cuda")
    L.mlp_grad(ctx, Pbf, Xd, Td, grad, loss, work)
    torch.cuda.synchronize()
    ref_out, _ = mlp.forward(theta, X)
    assert np.allclose(out.cpu().double().numpy(), ref_out, rtol=1e-4, atol=1e-5)
    go = mlp.loss_grad(theta, X, T)
    assert np.linalg.norm(grad.cpu().double().numpy() - go) <= 1e-4 * np.linalg.norm(go)


def test_train_entry_parity(ctx):
    """lrsdp_mlp_train: gradient at the bfloat16 parameters, Adam on the float32
    master, master rounded to bfloat16, against the same loop in the oracle."""
    import torch
    n, steps, lr = 3000, 6, 1e-2
    rng = np.random.default_rng(21)
    X = rng.standard_normal((n, 16)).astype(np.float32).astype(np.float64)
    T = (0.5 * rng.standard_normal((n, 2))).astype(np.float32).astype(np.float64)
    master0 = (mlp.init_params(7) + 0.05 * rng.standard_normal(mlp.NPARAM)).astype(np.float32)
    master = dev(master0)
    params = torch.empty(mlp.NPARAM, dtype=torch.bfloat16, device="cuda")
    m = torch.zeros(mlp.NPARAM, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    work = torch.empty(L.mlp_train_work_floats(), dtype=torch.float32, device="cuda")
    hist = torch.zeros(steps, dtype=torch.float64, device="cuda")
    L.mlp_train(ctx, master, params, m, v, dev(X, torch.float32), dev(T, torch.float32), 1, steps, lr, work, hist)
    torch.cuda.synchronize()
    th, mo, vo = master0.astype(np.float64), np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM)
    losses = []
    for step in range(1, steps + 1):
        p = mlp.to_bfloat16(th)
        losses.append(mlp.loss(p, X, T))
        th, mo, vo = mlp.adam(th, mo, vo, mlp.loss_grad(p, X, T), step, lr)
        th = th.astype(np.float32).astype(np.float64)   # the master is float32
    assert np.allclose(hist.cpu().numpy(), losses, rtol=1e-5)
    # Adam steps are about lr in size: compare against that scale
    assert np.linalg.norm(master.cpu().double().numpy() - th) <= 1e-2 * lr * np.sqrt(mlp.NPARAM)
    assert torch.equal(params, master.to(torch.bfloat16))


def test_targets_from_library(ctx):
    """Labels: t_i = -4 y_i / a_i and log(sigma_final / default sigma0), the default
    being 4 ||vec(C)||_1 / m."""
    import torch
    from oracle.problem import maxcut_problem
    n, u, v, w = graph("pm1")
    prob = L.Problem.maxcut(n, u, v, w).upload(ctx)
    y = np.random.default_rng(3).standard_normal(n)
    stats = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    feat = torch.empty((n, 16), dtype=torch.float32, device="cuda")
    L.ws_features(ctx, prob, feat, stats)
    target = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    L.ws_targets(ctx, prob, stats, dev(y), 123.0, target)
    torch.cuda.synchronize()
    absdeg = np.bincount(np.concatenate([u, v]), weights=np.abs(np.concatenate([w, w])), minlength=n)
    t = target.cpu().double().numpy()
    assert np.allclose(t[:, 0], mlp.targets_from_solution(y, absdeg), rtol=1e-6, atol=1e-6)
    default = 4.0 * maxcut_problem(n, u, v, w).c_l1 / n
    assert np.allclose(t[:, 1], mlp.sigma_label(123.0, default), rtol=1e-6)
    with pytest.raises(L.LrsdpError):
        L.ws_targets(ctx, prob, stats, dev(y), -1.0, target)


def test_warmstart_prediction_formula(ctx):
    import torch
    from oracle.problem import maxcut_problem
    n, u, v, w = graph("pm1")
    prob = L.Problem.maxcut(n, u, v, w).upload(ctx)
    theta = (mlp.init_params(9) + 0.1).astype(np.float32).astype(np.float64)
    F = mlp.features(n, u, v, w).astype(np.float32).astype(np.float64)
    # b3[0] (second-to-last parameter) shifts every t_i: put the median at 2, so
    # the limit acts on about half of the nodes
    theta[mlp.NPARAM - 2] = 0.0
    out0, _ = mlp.forward(theta, F)
    theta[mlp.NPARAM - 2] = float(np.float32(2.0 - np.median(out0[:, 0])))
    out, _ = mlp.forward(theta, F)
    assert (out[:, 0] > 2).any() and (out[:, 0] < 2).any()
    absdeg = np.bincount(np.concatenate([u, v]), weights=np.abs(np.concatenate([w, w])), minlength=n)
    base = 4.0 * maxcut_problem(n, u, v, w).c_l1 / n
    s = out[:, 1].mean()
    for lo, hi in [(-10.0, 10.0), (s + 0.5, s + 1.0), (s - 2.0, s - 1.0)]:
        model = W.Model(dev(theta, torch.float32), (lo, hi), {})
        y0, sigma0 = W.warm_start(ctx, prob, model)
        torch.cuda.synchronize()
        assert np.allclose(y0.cpu().numpy(), mlp.multipliers_from_output(out, absdeg), rtol=1e-4, atol=1e-5)
        assert np.isclose(sigma0, mlp.initial_penalty(out, base, lo, hi), rtol=1e-4)
    with pytest.raises(L.LrsdpError):
        L.warmstart(ctx, prob, dev(theta, torch.float32), torch.empty(22 * n, dtype=torch.float32, device="cuda"),
                    torch.empty(n, dtype=torch.float64, device="cuda"), (1.0, 0.0))


def test_trained_warm_start_gains(ctx):
    """Train on a few small graphs; on a held-out graph the warm start needs fewer
    L-BFGS iterations than the cold start (parity unpinned: an empirical check)."""
    import torch
    specs = [(20000, 2.5, 8.0, 1), (30000, 2.2, 5.0, 2), (40000, 2.8, 10.0, 3), (25000, 2.5, 4.0, 4),
             (50000, 2.4, 8.0, 5), (35000, 2.6, 6.0, 6)]
    feat, target, rng, recs = W.make_training_set(ctx, specs, log=print)
    assert all(r["rc"] == L.OK for r in recs)
    params, hist = W.train(ctx, feat, target, steps=200, lr=3e-3, log=print)
    assert params.dtype == torch.bfloat16
    assert hist[-1] < 0.5 * hist[0]
    model = W.Model(params, rng, {})
    n = 80000
    u, v = chung_lu_edges(n, n * 4, 2.5, 424242)
    prob = L.Problem.maxcut(n, u, v).upload(ctx)
    y0, sigma0 = W.warm_start(ctx, prob, model)
    R0 = init_factor(n, 16, 5)
    res = {}
    for mode in ["cold", "warm"]:
        opts = L.default_options(prec=L.F32, rank=16, ld=16)
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
