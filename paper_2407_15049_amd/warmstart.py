"""Learned warm start: training-set generation, training and prediction.

Orchestration only: the solves, features, targets, MLP forward/gradient/Adam
and the prediction all run in the library's HIP kernels (include/lrsdp.h,
learned warm start section); this module allocates device tensors and loops.
"""

from __future__ import annotations

import math
import time

import numpy as np

from . import lrsdp as L

# Training graphs: (kind, n, mean degree, beta, weights, seed).  Chung-Lu power
# law and Erdos-Renyi, unit and +-1 weights, n from 2e4 to 2e5.
TRAIN_SPECS = (
    [("cl", n, d, b, "pm1", 150490000 + k) for k, (n, d, b) in enumerate(
        [(20000, 10, 2.2), (50000, 10, 2.5), (100000, 10, 2.8), (200000, 10, 2.5),
         (30000, 6, 2.5), (80000, 12, 2.3)])]
    + [("er", n, d, None, "pm1", 150490100 + k) for k, (n, d) in enumerate(
        [(20000, 10), (60000, 10), (150000, 10), (40000, 8)])]
    + [("cl", n, d, b, "unit", 150490200 + k) for k, (n, d, b) in enumerate(
        [(30000, 8, 2.5), (100000, 8, 2.5), (60000, 4, 2.2), (150000, 6, 2.8)])]
)


def _graph(spec):
    from synth import chung_lu_edges, erdos_renyi_edges, pm1_weights
    kind, n, d, beta, wk, seed = spec
    m = n * d // 2
    u, v = chung_lu_edges(n, m, beta, seed) if kind == "cl" else erdos_renyi_edges(n, m, seed)
    w = pm1_weights(m, seed + 7) if wk == "pm1" else None
    return n, u, v, w


def make_training_set(ctx, specs=TRAIN_SPECS, rank=16, prec=L.F32, log=None):
    """Solve each training graph cold; return [(features, targets)] on device."""
    import torch
    from synth import init_factor
    dev = ctx.torch_device
    data = []
    for spec in specs:
        n, u, v, w = _graph(spec)
        prob = L.Problem.maxcut(n, u, v, w).upload(ctx)
        ld = L.padded_ld(rank, prec)
        opts = L.default_options(prec=prec, rank=rank, ld=ld)
        R = torch.zeros((n, ld), dtype=L.elem_dtype(prec), device=dev)
        R[:, :rank] = torch.from_numpy(init_factor(n, rank, spec[-1] + 1)).to(dev, R.dtype)
        y = torch.zeros(n, dtype=torch.float64, device=dev)
        t0 = time.perf_counter()
        rc, res = L.solve(ctx, prob, R, y, opts)
        feat = torch.empty((n, 16), dtype=torch.float32, device=dev)
        stats = torch.empty((n, 4), dtype=torch.float32, device=dev)
        L.ws_features(ctx, prob, feat, stats)
        sigma_default = 4.0 * prob.info.c_l1 / prob.info.m
        target = torch.empty((n, 2), dtype=torch.float32, device=dev)
        L.ws_targets(ctx, prob, stats, y, math.log(res.sigma / sigma_default), target)
        torch.cuda.synchronize()
        if log:
            log(f"train graph {spec}: rc {rc} outer {res.outer} inner {res.inner} "
                f"{time.perf_counter() - t0:.2f}s")
        data.append((feat, target))
    return data


def init_params(seed=0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for rows, cols in [(64, 16), (64, 0), (64, 64), (64, 0), (2, 64), (2, 0)]:
        if cols:
            lim = 1.0 / math.sqrt(cols)
            parts.append(rng.uniform(-lim, lim, rows * cols))
        else:
            parts.append(np.zeros(rows))
    return np.concatenate(parts).astype(np.float32)


def train(ctx, data, steps=400, lr=3e-3, seed=0, log=None):
    """Full-batch Adam over all training nodes (features concatenated)."""
    import torch
    dev = ctx.torch_device
    feat = torch.cat([f for f, _ in data]).contiguous()
    target = torch.cat([t for _, t in data]).contiguous()
    P = L.mlp_param_count()
    params = torch.from_numpy(init_params(seed)).to(dev)
    m = torch.zeros(P, dtype=torch.float32, device=dev)
    v = torch.zeros(P, dtype=torch.float32, device=dev)
    grad = torch.empty(P, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    work = torch.empty(256 * (P + 1), dtype=torch.float32, device=dev)
    hist = []
    for step in range(1, steps + 1):
        L.mlp_grad(ctx, params, feat, target, grad, loss, work)
        L.mlp_adam(ctx, params, m, v, grad, step, lr)
        if step == 1 or step % 50 == 0 or step == steps:
            hist.append((step, float(loss.item())))
            if log:
                log(f"train step {step}: loss {hist[-1][1]:.5f}")
    return params, hist


def warm_start(ctx, prob, params):
    """Predicted (y0 device float64, sigma0) for a MaxCut problem.

    Fallback: when the prediction is not finite the cold start is returned,
    y0 = 0 and sigma0 = 0.0 (0 selects the default initial penalty)."""
    import torch
    n = prob.info.n
    work = torch.empty(22 * n, dtype=torch.float32, device=ctx.torch_device)
    y0 = torch.empty(n, dtype=torch.float64, device=ctx.torch_device)
    try:
        sigma0 = L.warmstart(ctx, prob, params, work, y0)
    except L.LrsdpError as e:
        if e.code != L.ENUMERIC:
            raise
        y0.zero_()
        sigma0 = 0.0
    return y0, sigma0
