"""Kernel parity at the full size of the timed workload: the 1e7-node Chung-Lu
MaxCut graph (beta 2.5, mean degree 8, 4e7 edges, unit weights), rank 24, in
float64 and float32, with the kernels' own grids (the timed solve runs the
same kernels on the same sizes; the per-kernel entry points take the graph in
its own labels).

* SpMM (C - Diag(ytil)) V: 4000 sampled rows, the 2000 of highest degree (hub
  rows split into segments) and 2000 uniform ones, each recomputed by the
  oracle from its CSR row; bound 1e-10 (float64) / 1e-4 (float32, on rounded
  inputs) of the sum of absolute values of the row's terms.
* Line-search coefficients a1..a4, p1, p2 and the per-row q1, q2 over the whole
  graph against the oracle's, same bounds as the smaller cases.
"""

import numpy as np
import pytest

from oracle import kernels as K
from oracle.problem import maxcut_problem
from synth import maxcut_instance

from paper_2407_15049_amd import lrsdp as L
from gpu_util import dev_factor, dev_vec, host, rounded

pytestmark = pytest.mark.gpu

TOL = {L.F64: 1e-10, L.F32: 1e-4}
_CACHE = {}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.Context(0)


def full_size(ctx):
    if not _CACHE:
        inst = maxcut_instance("cl_10m")
        n, u, v, w = inst["n"], inst["u"], inst["v"], inst["w"]
        _CACHE["n"], _CACHE["r"] = n, inst["rank"]
        _CACHE["prob"] = L.Problem.maxcut(n, u, v, w).upload(ctx)
        _CACHE["op"] = maxcut_problem(n, u, v, w)
        deg = np.bincount(u, minlength=n) + np.bincount(v, minlength=n)
        rng = np.random.default_rng(61)
        _CACHE["rows"] = np.unique(np.concatenate([np.argsort(-deg, kind="stable")[:2000],
                                                   rng.integers(0, n, 2000)]))
    return _CACHE["prob"], _CACHE["op"], _CACHE["n"], _CACHE["r"], _CACHE["rows"]


@pytest.mark.parametrize("prec", [L.F64, L.F32])
def test_spmm_sampled_rows_full_size(ctx, prec):
    import torch
    prob, op, n, r, rows = full_size(ctx)
    print("CASE", dict(test="spmm_full_size", n=n, r=r, prec=prec), flush=True)
    assert prob.info.max_row_nnz > 100_000
    rng = np.random.default_rng(62)
    V = rounded(rng.standard_normal((n, r)), prec)
    ytil = rng.standard_normal(n)
    Vd = dev_factor(V, prec)
    Yd = torch.full_like(Vd, np.nan)
    L.k_spmm(ctx, prob, prec, Vd, dev_vec(ytil), Yd)
    torch.cuda.synchronize()
    Y = host(Yd[torch.from_numpy(rows).cuda()], r)
    C = op.C[rows]
    want = C @ V - ytil[rows, None] * V[rows]
    bound = abs(C) @ np.abs(V) + np.abs(ytil[rows])[:, None] * np.abs(V[rows])
    err = np.abs(Y - want)
    print("max err / bound", np.max(err / (bound + 1e-300)), flush=True)
    assert np.all(err <= TOL[prec] * bound + 1e-300)
    del Vd, Yd


@pytest.mark.parametrize("prec", [L.F64, L.F32])
def test_linesearch_coeffs_full_size(ctx, prec):
    import torch
    prob, op, n, r, _ = full_size(ctx)
    print("CASE", dict(test="ls_full_size", n=n, r=r, prec=prec), flush=True)
    rng = np.random.default_rng(63)
    R = rounded(rng.standard_normal((n, r)) / np.sqrt(r), prec)
    D = rounded(rng.standard_normal((n, r)) * 0.1, prec)
    y = rng.standard_normal(n)
    sigma = 2.7
    Rd, Dd = dev_factor(R, prec), dev_factor(D, prec)
    esz = 8 if prec == L.F64 else 4
    work = torch.empty(2 * n * Rd.shape[1] * esz + 8 * n, dtype=torch.uint8, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    q1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    q2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    L.k_ls_coeffs(ctx, prob, prec, Rd, Dd, dev_vec(y), sigma, work, out, q1, q2)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    del Rd, Dd, work
    c = K.linesearch_coeffs(op, R, D, y, sigma)
    ytil = y + sigma * c["q0"]
    absC = abs(op.C)
    aR, aD = np.abs(R), np.abs(D)
    bq1 = 2 * np.sum(aR * aD, axis=1)
    bq2 = np.sum(aD * aD, axis=1)
    bp1 = 2 * np.sum((absC @ aR) * aD)
    bp2 = np.sum((absC @ aD) * aD)
    assert np.all(np.abs(q1.cpu().numpy() - c["q1"]) <= 1e-12 * bq1 + 1e-300)
    assert np.all(np.abs(q2.cpu().numpy() - c["q2"]) <= 1e-12 * bq2 + 1e-300)
    bounds = {
        "a1": 0.5 * sigma * np.sum(bq2 * bq2), "a2": sigma * np.sum(bq1 * bq2),
        "a3": bp2 + np.sum(np.abs(ytil) * bq2) + 0.5 * sigma * np.sum(bq1 * bq1),
        "a4": bp1 + np.sum(np.abs(ytil) * bq1), "p1": bp1, "p2": bp2,
    }
    for idx, name in enumerate(["a1", "a2", "a3", "a4", "p1", "p2"]):
        print(name, g[idx], c[name], abs(g[idx] - c[name]) / bounds[name], flush=True)
        assert abs(g[idx] - c[name]) <= TOL[prec] * bounds[name], (name, g[idx], c[name])
