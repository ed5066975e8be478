"""GPU dual certificate (block Lanczos on C - A*(y)) against the oracle.

The oracle's lambda_min is the dense symmetric eigensolver (n <= 6000).  The
GPU returns the smallest Ritz value theta (never below lambda_min, up to
rounding) and the residual of its Ritz pair; parity: |theta - lambda_min| <=
max(residual, 1e-9 ||S||).  Closed forms: the complete graph K_n and the odd
cycle C_n at their optimal multipliers (lambda_min = 0, dual bound = optimum).
"""

import math

import numpy as np
import pytest

from oracle import certify
from oracle.problem import completion_problem, maxcut_problem
from synth import chung_lu_edges, completion_instance, erdos_renyi_edges, init_factor, pm1_weights

from paper_2407_15049_amd import lrsdp as L
from gpu_util import dev_vec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.Context(0)


def print_case(**kw):
    print("CASE", kw, flush=True)


def spectral_scale(op, y):
    S = (op.C - op.A_adj(y)).tocsr()
    return float(abs(S).sum(axis=1).max())         # Gershgorin bound on ||S||


def maxcut_case(case):
    if case == "er":
        u, v = erdos_renyi_edges(2000, 10000, 31)
        return 2000, u, v, None
    if case == "pm1":
        u, v = erdos_renyi_edges(1500, 9000, 32)
        return 1500, u, v, pm1_weights(9000, 33)
    if case == "cl_heavy":                         # hubs above 128 neighbours: segment path
        u, v = chung_lu_edges(6000, 30000, 2.2, 34)
        return 6000, u, v, None
    if case == "general":
        u, v = erdos_renyi_edges(900, 4000, 35)
        return 900, u, v, np.random.default_rng(36).uniform(-2, 3, 4000)
    if case == "hub":                              # one row of 3000: eigenvalues far apart, ill-conditioned blocks
        u, v = erdos_renyi_edges(6000, 24000, 37)
        pairs = {(min(a, b), max(a, b)) for a, b in zip(u.tolist(), v.tolist())}
        for k in range(1, 3001):
            pairs.add((0, k))
        uv = np.array(sorted(pairs), dtype=np.int32)
        return 6000, uv[:, 0], uv[:, 1], pm1_weights(len(uv), 38)
    raise KeyError(case)


@pytest.mark.parametrize("case", ["er", "pm1", "cl_heavy", "general", "hub"])
def test_maxcut_lambda_min_parity(ctx, case):
    n, u, v, w = maxcut_case(case)
    print_case(test="certify", case=case, n=n)
    prob = L.Problem.maxcut(n, u, v, w).upload(ctx)
    op = maxcut_problem(n, u, v, w)
    rng = np.random.default_rng(40)
    # multipliers near the diagonal of C, so that lambda_min is small and the
    # spectrum's low end is crowded, as at a solution
    y = np.asarray(op.C.diagonal()).ravel() + 0.3 * rng.standard_normal(n)
    scale = spectral_scale(op, y)
    cert = L.certify(ctx, prob, dev_vec(y), max_iter=400, tol=1e-9 * scale)
    lam = certify.lambda_min(op, y)
    print(cert.as_dict(), "oracle", lam, "scale", scale)
    assert cert.block == 8 and cert.iters >= 1
    assert cert.lambda_min >= lam - 1e-9 * scale
    assert abs(cert.lambda_min - lam) <= max(cert.resid, 1e-9 * scale)
    assert abs(cert.by - y.sum()) <= 1e-12 * np.abs(y).sum()
    assert abs(cert.lambda_lb - (cert.lambda_min - cert.resid)) <= 1e-15 * scale
    bound = certify.maxcut_dual_bound(op, y)
    assert abs(cert.dual_bound - bound) <= n * max(cert.resid, 1e-9 * scale) + 1e-9 * abs(bound)
    assert cert.err2 == pytest.approx(max(0.0, -cert.lambda_min) / (1 + op.c_l1), rel=1e-12, abs=1e-300)
    # the largest Ritz value: a lower estimate of lambda_max, which the outer end
    # of the Krylov space resolves quickly
    import scipy.linalg as sla
    S = (op.C - op.A_adj(y)).toarray()
    lam_max = float(sla.eigvalsh(S, subset_by_index=[n - 1, n - 1])[0])
    assert lam_max - 1e-6 * scale <= cert.lambda_max <= lam_max + 1e-9 * scale


def test_complete_graph_closed_form(ctx):
    # K_n at y = -(n/4) 1: C - Diag(y) = J/4, lambda_min = 0, dual bound -n^2/4
    n = 40
    iu = np.triu_indices(n, 1)
    u, v = iu[0].astype(np.int32), iu[1].astype(np.int32)
    prob = L.Problem.maxcut(n, u, v).upload(ctx)
    y = np.full(n, -n / 4.0)
    cert = L.certify(ctx, prob, dev_vec(y), max_iter=50, tol=1e-12)
    print(cert.as_dict())
    assert cert.status in (0, 2)
    assert abs(cert.lambda_min) <= 1e-12 * n
    assert cert.dual_bound == pytest.approx(-n * n / 4.0, rel=1e-12)


def test_odd_cycle_closed_form(ctx):
    # C_n (n odd) at y_i = -(1 + cos(pi/n))/2: lambda_min = 0 and the bound is the
    # optimum -(n/2)(1 + cos(pi/n))
    n = 41
    u = np.arange(n, dtype=np.int32)
    v = ((u + 1) % n).astype(np.int32)
    prob = L.Problem.maxcut(n, u, v).upload(ctx)
    y = np.full(n, -(1 + math.cos(math.pi / n)) / 2)
    cert = L.certify(ctx, prob, dev_vec(y), max_iter=60, tol=1e-12)
    print(cert.as_dict())
    assert abs(cert.lambda_min) <= 1e-10
    assert cert.dual_bound == pytest.approx(-(n / 2) * (1 + math.cos(math.pi / n)), rel=1e-10)


def test_completion_spectral_norm(ctx):
    n1, n2 = 300, 250
    i, j, M, _, _ = completion_instance(n1, n2, 4, 20, seed=41)
    prob = L.Problem.completion(n1, n2, i, j, M).upload(ctx)
    op = completion_problem(n1, n2, i, j, M)
    y = 0.05 * np.random.default_rng(42).standard_normal(op.m)
    cert = L.certify(ctx, prob, dev_vec(y), max_iter=300, tol=1e-10)
    import scipy.sparse as sp
    s = np.linalg.norm(sp.csr_matrix((y, (i, j)), shape=(n1, n2)).toarray(), 2)
    print(cert.as_dict(), "||Y||_2", s)
    assert abs((1.0 - cert.lambda_min) - s) <= max(cert.resid, 1e-10 * (1 + s))
    assert abs(cert.by - float(op.b @ y)) <= 1e-12 * np.abs(op.b * y).sum()
    bound = certify.completion_dual_bound(op, n1, n2, i, j, y)
    assert abs(cert.dual_bound - bound) <= 1e-8 * (1 + abs(bound)) + abs(bound) * cert.resid


def test_certify_validation(ctx):
    n, u, v, w = maxcut_case("er")
    prob = L.Problem.maxcut(n, u, v, w).upload(ctx)
    import torch
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.LrsdpError) as e:
        L.certify(ctx, prob, y, max_iter=10, work=small)
    assert e.value.code == L.ENOMEM
    with pytest.raises(L.LrsdpError) as e:
        L.certify(ctx, prob, y, max_iter=0)
    assert e.value.code == L.EINVAL
    tiny = L.Problem.maxcut(10, np.array([0, 1], np.int32), np.array([1, 2], np.int32)).upload(ctx)
    with pytest.raises(L.LrsdpError) as e:
        L.certify(ctx, tiny, torch.zeros(10, dtype=torch.float64, device="cuda"), max_iter=10)
    assert e.value.code == L.EUNSUPPORTED


@pytest.mark.parametrize("rank", [10, 16])
def test_solve_then_certify_er_1k(ctx, rank):
    """After a solve, the GPU certificate equals the oracle's on the returned y.
    At rank 10 this instance stops at a stationary point that is not optimal:
    the certificate shows a clearly negative lambda_min; at rank 16 the
    certified gap closes."""
    import torch
    u, v = erdos_renyi_edges(1000, 5000, 15049)
    n = 1000
    prob = L.Problem.maxcut(n, u, v).upload(ctx)
    op = maxcut_problem(n, u, v)
    R0 = init_factor(n, rank, 15050 if rank == 10 else 15051)
    opts = L.default_options(prec=L.F64, rank=rank, ld=L.padded_ld(rank, L.F64))
    Rd = torch.zeros((n, opts.ld), dtype=torch.float64, device="cuda")
    Rd[:, :rank] = torch.from_numpy(R0).cuda()
    yd = torch.zeros(n, dtype=torch.float64, device="cuda")
    rc, res = L.solve(ctx, prob, Rd, yd, opts)
    assert rc == L.OK
    y = yd.cpu().numpy()
    scale = spectral_scale(op, y)
    cert = L.certify(ctx, prob, yd, max_iter=300, tol=1e-9 * scale)
    lam = certify.lambda_min(op, y)
    gap = (res.obj - cert.dual_bound) / (1 + abs(res.obj) + abs(cert.dual_bound))
    print("rank", rank, res.as_dict(), cert.as_dict(), "oracle", lam, "gap", gap)
    assert abs(cert.lambda_min - lam) <= max(cert.resid, 1e-9 * scale)
    assert cert.dual_bound <= res.obj + 1e-9 * abs(res.obj)
    if rank == 10:
        assert cert.lambda_min < -1e-3
    else:
        assert gap <= 2e-5


@pytest.mark.parametrize("rank", [10, 16])
def test_lanczos_estimate_then_host_proof(ctx, rank):
    """After a solve, the Lanczos estimate's lambda_lb (less 1e-7 of the
    spectral scale) is proven by the host Cholesky of C - Diag(y) - shift I, and
    the proven dual bound lies below the objective: the estimate and the proof
    agree where both apply."""
    import torch
    u, v = erdos_renyi_edges(1000, 5000, 15049)
    n = 1000
    print_case(test="certify_then_proof", rank=rank)
    prob = L.Problem.maxcut(n, u, v).upload(ctx)
    op = maxcut_problem(n, u, v)
    opts = L.default_options(prec=L.F64, rank=rank, ld=L.padded_ld(rank, L.F64))
    Rd = torch.zeros((n, opts.ld), dtype=torch.float64, device="cuda")
    Rd[:, :rank] = torch.from_numpy(init_factor(n, rank, 15050 if rank == 10 else 15051)).cuda()
    yd = torch.zeros(n, dtype=torch.float64, device="cuda")
    rc, res = L.solve(ctx, prob, Rd, yd, opts)
    assert rc == L.OK
    y = yd.cpu().numpy()
    scale = spectral_scale(op, y)
    cert = L.certify(ctx, prob, yd, max_iter=300, tol=1e-9 * scale)
    proof = L.certify_dense(prob, y, cert.lambda_lb - 1e-7 * scale)
    print(cert.as_dict(), proof.as_dict())
    assert proof.status == 0
    lam = certify.lambda_min(op, y)
    assert proof.lambda_lb <= lam <= cert.lambda_min + 1e-9 * scale
    assert proof.dual_bound <= res.obj
    # a shift above the smallest Ritz value cannot be proven
    assert L.certify_dense(prob, y, cert.lambda_min + 1e-6 * scale).status == 1
