"""Learned warm start: training-set generation, training, model file and prediction.

Orchestration only: the solves, features, targets (labels), MLP forward /
gradient / Adam and the prediction all run in the library's HIP kernels
(include/lrsdp.h, learned warm start section); this module draws the training
graphs, allocates device tensors, picks the training nodes and moves bytes.

Training workload: 200 Chung-Lu MaxCut graphs, graph j drawn with seed
150490000 + j, n log-uniform in [1e4, 1e6], degree exponent uniform in
[2.1, 3.0], mean degree log-uniform in [3, 12], unit weights, each solved cold
in float32 at rank ceil(log2 n) to 1e-5.  Every graph gives the same number of
training nodes (all of its nodes, or a seeded sample of them), so graphs weigh
equally in the mean-squared loss.  The parameters are stored in bfloat16 with
a float32 master copy during training (lrsdp_mlp_train).

The model file (``warmstart_model.npz`` next to this module) holds the
bfloat16 parameter bits, the range of the penalty labels (the prediction is
limited to it) and a description of the training run.
"""

from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import lrsdp as L

MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warmstart_model.npz")
TRAIN_SEED = 150490000
N_TRAIN = 200
NODES_PER_GRAPH = 20000


def train_specs(count=N_TRAIN, seed=TRAIN_SEED):
    """(n, beta, mean degree, graph seed) of the training graphs."""
    g = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for j in range(count):
        n = int(round(10.0 ** g.uniform(4.0, 6.0)))
        beta = float(g.uniform(2.1, 3.0))
        dbar = float(10.0 ** g.uniform(math.log10(3.0), math.log10(12.0)))
        specs.append((n, beta, dbar, seed + j))
    return specs


def _graph(spec):
    from synth import chung_lu_edges
    n, beta, dbar, seed = spec
    m = int(round(n * dbar / 2))
    u, v = chung_lu_edges(n, m, beta, seed)
    return n, u, v


def make_training_set(ctx, specs=None, prec=L.F32, nodes_per_graph=NODES_PER_GRAPH, time_limit=120.0, log=None,
                      budget_s=None):
    """Solve each training graph cold; return (features, targets, label range,
    per-graph records) with the training nodes of all graphs stacked on the
    device.  With budget_s, graphs after the first that would start once
    budget_s seconds have passed are left out (the records say how many ran)."""
    import torch
    from synth import init_factor
    specs = train_specs() if specs is None else specs
    dev = ctx.torch_device
    feats, targets, recs = [], [], []
    t_start = time.perf_counter()
    for k, spec in enumerate(specs):
        if budget_s is not None and k > 0 and time.perf_counter() - t_start > budget_s:
            if log:
                log(f"label-solve budget of {budget_s:.0f}s spent after {k} graphs")
            break
        t0 = time.perf_counter()
        n, u, v = _graph(spec)
        prob = L.Problem.maxcut(n, u, v).upload(ctx)
        rank = max(2, math.ceil(math.log2(n)))
        ld = L.padded_ld(rank, prec)
        opts = L.default_options(prec=prec, rank=rank, ld=ld, time_limit_s=time_limit)
        R = torch.zeros((n, ld), dtype=L.elem_dtype(prec), device=dev)
        R[:, :rank] = torch.from_numpy(init_factor(n, rank, spec[-1] + 1)).to(dev, R.dtype)
        y = torch.zeros(n, dtype=torch.float64, device=dev)
        t1 = time.perf_counter()
        rc, res = L.solve(ctx, prob, R, y, opts)
        t2 = time.perf_counter()
        rec = dict(n=n, beta=round(spec[1], 4), dbar=round(spec[2], 4), seed=spec[3], rank=rank, rc=rc,
                   outer=res.outer, inner=res.inner, sigma=res.sigma, solve_s=round(t2 - t1, 3))
        recs.append(rec)
        if rc == L.OK:
            feat = torch.empty((n, 16), dtype=torch.float32, device=dev)
            stats = torch.empty((n, 4), dtype=torch.float32, device=dev)
            L.ws_features(ctx, prob, feat, stats)
            target = torch.empty((n, 2), dtype=torch.float32, device=dev)
            L.ws_targets(ctx, prob, stats, y, res.sigma, target)
            if n > nodes_per_graph:
                pick = np.sort(np.random.Generator(np.random.PCG64(spec[3] + 2)).choice(
                    n, nodes_per_graph, replace=False))
                idx = torch.from_numpy(pick).to(dev)
                feat, target = feat[idx].contiguous(), target[idx].contiguous()
            feats.append(feat)
            targets.append(target)
        if log:
            log(f"train graph {k}: n {n} beta {spec[1]:.2f} dbar {spec[2]:.2f} rc {rc} outer {res.outer} "
                f"inner {res.inner} sigma {res.sigma:.3e} solve {t2 - t1:.2f}s total {time.perf_counter() - t0:.2f}s")
        del prob, R, y
    feat = torch.cat(feats).contiguous()
    target = torch.cat(targets).contiguous()
    s = target[:, 1].to(torch.float64)
    label_range = (float(s.min().item()), float(s.max().item()))
    return feat, target, label_range, recs


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


def train(ctx, feat, target, steps=600, lr=3e-3, seed=0, chunk=50, log=None):
    """Full-batch Adam with bfloat16 parameters and a float32 master copy, all
    steps in lrsdp_mlp_train; returns (bfloat16 parameters, loss history)."""
    import torch
    dev = ctx.torch_device
    P = L.mlp_param_count()
    master = torch.from_numpy(init_params(seed)).to(dev)
    params = torch.empty(P, dtype=torch.bfloat16, device=dev)
    m = torch.zeros(P, dtype=torch.float32, device=dev)
    v = torch.zeros(P, dtype=torch.float32, device=dev)
    work = torch.empty(L.mlp_train_work_floats(), dtype=torch.float32, device=dev)
    hist = torch.zeros(steps, dtype=torch.float64, device=dev)
    for first in range(1, steps + 1, chunk):
        k = min(chunk, steps + 1 - first)
        L.mlp_train(ctx, master, params, m, v, feat, target, first, k, lr, work, hist[first - 1:])
        if log:
            log(f"train steps {first}-{first + k - 1}: loss {hist[first - 1].item():.5f} -> "
                f"{hist[first + k - 2].item():.5f}")
    return params, hist.cpu().numpy()


class Model:
    """A trained warm-start model on the device."""

    def __init__(self, params, log_range, meta):
        self.params = params            # device bfloat16, nparam
        self.log_range = log_range      # (lo, hi) of the penalty labels
        self.meta = meta


def save_model(path, params, log_range, meta):
    bits = params.view(torch_int16()).cpu().numpy().view(np.uint16)
    np.savez(path, params_bf16=bits, log_range=np.array(log_range, dtype=np.float64),
             meta=np.array(json.dumps(meta)))


def torch_int16():
    import torch
    return torch.int16


def load_model(dev, path=MODEL_PATH):
    """The committed model, or None when there is none."""
    import torch
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    bits = np.ascontiguousarray(z["params_bf16"]).view(np.int16)
    if bits.size != L.mlp_param_count():
        raise ValueError(f"{path}: {bits.size} parameters, the library expects {L.mlp_param_count()}")
    params = torch.from_numpy(bits.copy()).to(dev).view(torch.bfloat16)
    lo, hi = (float(x) for x in z["log_range"])
    return Model(params, (lo, hi), json.loads(str(z["meta"])))


def warm_start(ctx, prob, model):
    """Predicted (y0 device float64, sigma0) for a MaxCut problem.

    Fallback: when the prediction is not finite the cold start is returned,
    y0 = 0 and sigma0 = 0.0 (0 selects the default initial penalty)."""
    import torch
    n = prob.info.n
    work = torch.empty(22 * n, dtype=torch.float32, device=ctx.torch_device)
    y0 = torch.empty(n, dtype=torch.float64, device=ctx.torch_device)
    params = model.params if isinstance(model, Model) else model
    rng = model.log_range if isinstance(model, Model) else (-10.0, 10.0)
    try:
        sigma0 = L.warmstart(ctx, prob, params, work, y0, rng)
    except L.LrsdpError as e:
        if e.code != L.ENUMERIC:
            raise
        y0.zero_()
        sigma0 = 0.0
    return y0, sigma0


def main():
    """Train the model on the training workload and write the model file."""
    import argparse
    import sys

    import torch
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--graphs", type=int, default=N_TRAIN)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--nodes-per-graph", type=int, default=NODES_PER_GRAPH)
    ap.add_argument("--out", default=MODEL_PATH)
    ap.add_argument("--budget", type=float, default=None, help="seconds of label solves at most")
    a = ap.parse_args()

    def log(msg):
        print(f"[warmstart] {msg}", file=sys.stderr, flush=True)

    ctx = L.Context(0)
    t0 = time.perf_counter()
    feat, target, rng, recs = make_training_set(ctx, train_specs(a.graphs), nodes_per_graph=a.nodes_per_graph,
                                                log=log, budget_s=a.budget)
    t1 = time.perf_counter()
    params, hist = train(ctx, feat, target, steps=a.steps, lr=a.lr, log=log)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    meta = dict(name=f"cl{len(recs)}-bf16", graphs=len(recs), graphs_planned=a.graphs,
                converged=sum(r["rc"] == 0 for r in recs),
                train_nodes=int(feat.shape[0]), steps=a.steps, lr=a.lr, label_solves_s=round(t1 - t0, 1),
                train_s=round(t2 - t1, 2), loss_first=float(hist[0]), loss_last=float(hist[-1]),
                log_sigma_range=rng, solves=recs)
    save_model(a.out, params, rng, meta)
    log(f"wrote {a.out}: {meta['converged']}/{len(recs)} graphs, {meta['train_nodes']} nodes, loss "
        f"{hist[0]:.4f} -> {hist[-1]:.4f}, label range {rng}")


if __name__ == "__main__":
    main()
