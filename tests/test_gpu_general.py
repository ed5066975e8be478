"""GPU parity of the general-problem path (Section 3.4 compression) against the
FP64 oracle, whose general problem is the plain full-matrix definition.  Each
per-kernel case runs with C stored on Omega and with C stored densely (Section
3.5, last paragraph: the dense product on float64 matrix cores).

Per kernel, the float64 outputs agree with the oracle within 1e-12 (maps) or
1e-10 (reductions) of the sum of absolute values of their terms.  Float32
storage is checked on float32-rounded inputs at 1e-4.  End to end:
* the Lovasz theta SDPs reach their closed forms (-sqrt 5, -4, ...);
* random feasible instances match the oracle's solve to 1e-5 in objective (the
  two sides' L-BFGS paths part through rounding; err3 <= 1e-5 bounds the gap);
* a MaxCut SDP written as general triplets solves to the MaxCut path's
  objective.
"""

import math

import numpy as np
import pytest

from oracle import certify
from oracle import kernels as K
from oracle.alm import Options as OOptions
from oracle.alm import alm_solve
from oracle.problem import general_problem, maxcut_problem
from synth import (cycle_edges, erdos_renyi_edges, init_factor, petersen_edges, pm1_weights,
                   random_box_triplets, random_general_triplets, theta_triplets)

from paper_2407_15049_amd import lrsdp as L
from gpu_util import dev_factor, dev_vec, host, rounded

pytestmark = pytest.mark.gpu

TOL = {L.F64: 1e-10, L.F32: 1e-4}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.Context(0)


def print_case(**kw):
    print("CASE", kw, flush=True)


def random_case(n, m, per_con, c_nnz, seed):
    cr, cc, cv, m, ak, ar, ac, av, W = random_general_triplets(n, m, per_con, c_nnz, 3, seed)
    b = general_problem(n, cr, cc, cv, m, ak, ar, ac, av, np.zeros(m)).A_of(W)
    return n, (cr, cc, cv, m, ak, ar, ac, av, b)


def case_data(case):
    if case == "theta_petersen":
        u, v = petersen_edges()
        return 10, theta_triplets(10, u, v), 6
    if case == "theta_dense":           # C = -J: every row of the operator is full
        u, v = erdos_renyi_edges(300, 1500, 41)
        return 300, theta_triplets(300, u, v), 8
    if case == "random_small":
        n, t = random_case(60, 40, 4, 120, 5)
        return n, t, 10
    if case == "random_ragged":         # many blocks and a ragged tail; the trace row is a long row
        n, t = random_case(2003, 1501, 5, 6000, 6)
        return n, t, 12
    if case == "long_rows":             # every constraint row longer than 512: a workgroup per row,
        n, t = random_case(700, 1200, 600, 2000, 8)      # more rows than workgroups
        return n, t, 8
    raise KeyError(case)


CASES = ["theta_petersen", "theta_dense", "random_small", "random_ragged", "long_rows"]


STORAGE = [L.C_SPARSE, L.C_DENSE]


def setup(ctx, case, storage=None):
    n, t, r = case_data(case)
    prob = L.Problem.general(n, *t, c_storage=storage).upload(ctx)
    if storage is not None:
        assert prob.info.c_dense == (storage == L.C_DENSE)
    op = general_problem(n, *t)
    return prob, op, r


def test_automatic_storage_choice(ctx):
    # dense when n <= 8192 and at least 10% of the upper triangle of C is nonzero
    assert setup(ctx, "theta_dense")[0].info.c_dense == 1       # C = -J
    assert setup(ctx, "theta_petersen")[0].info.c_dense == 1
    assert setup(ctx, "random_ragged")[0].info.c_dense == 0     # 6000 of 2e6 positions
    assert setup(ctx, "random_small")[0].info.c_dense == 0      # 120 of 1830


@pytest.mark.parametrize("storage", STORAGE)
@pytest.mark.parametrize("prec", [L.F64, L.F32])
@pytest.mark.parametrize("case", CASES)
def test_spmm_parity(ctx, case, prec, storage):
    import torch
    prob, op, r = setup(ctx, case, storage)
    print_case(test="gen_spmm", case=case, prec=prec, storage=storage)
    rng = np.random.default_rng(1)
    V = rounded(rng.standard_normal((op.n, r)), prec)
    ytil = rng.standard_normal(op.m)
    Vd = dev_factor(V, prec)
    Yd = torch.full_like(Vd, np.nan)
    L.k_spmm(ctx, prob, prec, Vd, dev_vec(ytil), Yd)
    torch.cuda.synchronize()
    Y = host(Yd)
    assert np.all(Y[:, r:] == 0)
    ref = K.spmm(op, ytil, V)
    bound = (abs(op.C) + abs(op.A_adj(np.abs(ytil)))) @ np.abs(V)
    assert np.all(np.abs(Y[:, :r] - ref) <= TOL[prec] * bound + 1e-300)


@pytest.mark.parametrize("storage", STORAGE)
@pytest.mark.parametrize("prec", [L.F64, L.F32])
@pytest.mark.parametrize("case", CASES)
def test_constraint_map_parity(ctx, case, prec, storage):
    import torch
    prob, op, r = setup(ctx, case, storage)
    print_case(test="gen_constraint", case=case, prec=prec, storage=storage)
    rng = np.random.default_rng(2)
    U = rounded(rng.standard_normal((op.n, r)), prec)
    V = rounded(rng.standard_normal((op.n, r)), prec)
    out = torch.empty(op.m, dtype=torch.float64, device="cuda")
    L.k_constraint(ctx, prob, prec, dev_factor(U, prec), dev_factor(V, prec), out)
    torch.cuda.synchronize()
    ref = K.constraint_map(op, U, V)
    bound = abs(op.Abar) @ np.einsum("pc,pc->p", np.abs(U[op.col_a]), np.abs(V[op.col_b]))
    assert np.all(np.abs(out.cpu().numpy() - ref) <= 1e-12 * bound + 1e-300)


@pytest.mark.parametrize("storage", STORAGE)
@pytest.mark.parametrize("prec", [L.F64, L.F32])
@pytest.mark.parametrize("case", CASES)
def test_linesearch_coeffs_parity(ctx, case, prec, storage):
    import torch
    prob, op, r = setup(ctx, case, storage)
    print_case(test="gen_ls", case=case, prec=prec, storage=storage)
    rng = np.random.default_rng(3)
    R = rounded(rng.standard_normal((op.n, r)) / np.sqrt(r), prec)
    D = rounded(rng.standard_normal((op.n, r)) * 0.1, prec)
    y = rng.standard_normal(op.m)
    sigma = 1.9
    Rd, Dd = dev_factor(R, prec), dev_factor(D, prec)
    esz = 8 if prec == L.F64 else 4
    work = torch.empty(2 * op.n * Rd.shape[1] * esz + 16 * op.m, dtype=torch.uint8, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    q1 = torch.zeros(op.m, dtype=torch.float64, device="cuda")
    q2 = torch.zeros(op.m, dtype=torch.float64, device="cuda")
    L.k_ls_coeffs(ctx, prob, prec, Rd, Dd, dev_vec(y), sigma, work, out, q1, q2)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    c = K.linesearch_coeffs(op, R, D, y, sigma)
    ytil = y + sigma * c["q0"]
    aR, aD = np.abs(R), np.abs(D)
    aA = abs(op.Abar)
    pair = lambda X, Y: aA @ np.einsum("pc,pc->p", X[op.col_a], Y[op.col_b])
    bq1 = pair(aR, aD) + pair(aD, aR)
    bq2 = pair(aD, aD)
    assert np.all(np.abs(q1.cpu().numpy() - c["q1"]) <= 1e-12 * bq1 + 1e-300)
    assert np.all(np.abs(q2.cpu().numpy() - c["q2"]) <= 1e-12 * bq2 + 1e-300)
    aC = abs(op.C)
    bp1 = 2 * np.sum((aC @ aD) * aR)
    bp2 = np.sum((aC @ aD) * aD)
    tol = TOL[prec]
    bounds = {
        "a1": 0.5 * sigma * np.sum(bq2 * bq2), "a2": sigma * np.sum(bq1 * bq2),
        "a3": bp2 + np.sum(np.abs(ytil) * bq2) + 0.5 * sigma * np.sum(bq1 * bq1),
        "a4": bp1 + np.sum(np.abs(ytil) * bq1), "p1": bp1, "p2": bp2,
    }
    for idx, name in enumerate(["a1", "a2", "a3", "a4", "p1", "p2"]):
        assert abs(g[idx] - c[name]) <= tol * bounds[name] + 1e-300, (name, g[idx], c[name])


@pytest.mark.parametrize("storage", STORAGE)
@pytest.mark.parametrize("prec", [L.F64, L.F32])
@pytest.mark.parametrize("case", CASES)
def test_alm_step_parity(ctx, case, prec, storage):
    import torch
    prob, op, r = setup(ctx, case, storage)
    print_case(test="gen_alm", case=case, prec=prec, storage=storage)
    rng = np.random.default_rng(4)
    R = rounded(rng.standard_normal((op.n, r)) / np.sqrt(r), prec)
    y = rng.standard_normal(op.m)
    sigma = 0.7
    Rd = dev_factor(R, prec)
    yd = dev_vec(y)
    work = torch.empty(8 * max(op.m, op.n * Rd.shape[1]), dtype=torch.uint8, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    L.k_alm(ctx, prob, prec, Rd, yd, sigma, work, out)
    torch.cuda.synchronize()
    ynew = K.multiplier_estimate(op, R, y, sigma)
    m = K.alm_measures(op, R, ynew)
    bA = abs(op.Abar) @ np.einsum("pc,pc->p", np.abs(R[op.col_a]), np.abs(R[op.col_b]))
    assert np.all(np.abs(yd.cpu().numpy() - ynew) <= 1e-12 * (np.abs(y) + sigma * (np.abs(op.b) + bA)))
    g = out.cpu().numpy()
    bobj = np.sum((abs(op.C) @ np.abs(R)) * np.abs(R))
    assert abs(g[0] - m["obj"]) <= 1e-12 * bobj
    assert abs(g[1] - m["dual"]) <= 1e-11 * np.sum(np.abs(op.b * ynew)) + 1e-300
    assert abs(g[2] - m["res_norm"]) <= 1e-9 * (1 + m["res_norm"])


def gpu_solve(ctx, prob, R0, prec, m, **kw):
    import torch
    r = R0.shape[1]
    opts = L.default_options(prec=prec, rank=r, ld=L.padded_ld(r, prec), **kw)
    Rd = dev_factor(R0, prec)
    yd = torch.zeros(m, dtype=torch.float64, device="cuda")
    rc, res = L.solve(ctx, prob, Rd, yd, opts)
    torch.cuda.synchronize()
    return rc, res, host(Rd, r), yd.cpu().numpy()


@pytest.mark.parametrize("storage", STORAGE)
@pytest.mark.parametrize("graph", ["C5", "C7", "petersen"])
def test_theta_closed_forms(ctx, graph, storage):
    if graph == "petersen":
        n, (u, v), want = 10, petersen_edges(), 4.0
    else:
        n = int(graph[1:])
        c = math.cos(math.pi / n)
        (u, v), want = cycle_edges(n), n * c / (1 + c)
    print_case(test="theta", graph=graph, storage=storage)
    t = theta_triplets(n, u, v)
    prob = L.Problem.general(n, *t, c_storage=storage).upload(ctx)
    op = general_problem(n, *t)
    R0 = init_factor(n, 6, 3)
    rc, res, R, y = gpu_solve(ctx, prob, R0, L.F64, op.m, tol=1e-8)
    ores = alm_solve(op, R0, opts=OOptions(tol=1e-8))
    print(res.as_dict(), "oracle", ores.obj, "closed form", -want)
    assert rc == L.OK and ores.converged
    assert -res.obj == pytest.approx(want, rel=1e-6)
    assert abs(res.obj - ores.obj) <= 1e-7 * want
    m = K.alm_measures(op, R, y)
    assert abs(m["obj"] - res.obj) <= 1e-10 * want


@pytest.mark.parametrize("storage", STORAGE)
@pytest.mark.parametrize("prec", [L.F64, L.F32])
def test_random_general_solve_matches_oracle(ctx, prec, storage):
    prob, op, r = setup(ctx, "random_small", storage)
    print_case(test="gen_solve", case="random_small", prec=prec, storage=storage)
    R0 = init_factor(op.n, r, 4)
    rc, res, R, y = gpu_solve(ctx, prob, R0, prec, op.m)
    ores = alm_solve(op, R0, opts=OOptions())
    print(res.as_dict(), "oracle", ores.obj, ores.outer, ores.inner)
    assert rc == L.OK and ores.converged
    m = K.alm_measures(op, R, y)
    assert m["err1"] <= 1e-5 and abs(m["err3"]) <= 1e-5
    # the two sides' L-BFGS paths part after a few hundred iterations (rounding),
    # so the objectives agree to what the stopping tolerance on err3 allows
    if prec == L.F64:
        assert abs(res.obj - ores.obj) <= 1e-5 * abs(ores.obj)
    else:
        assert abs(m["obj"] - ores.obj) <= 1e-4 * abs(ores.obj)


def test_box_constrained_large_solve_matches_oracle(ctx):
    # diag(X) = 1 plus 30 random side constraints, n = 2003 (the random family
    # with 1501 constraints needs a rank near sqrt(2m) = 55, beyond the stride
    # limit, and stalls on both sides)
    import torch
    n = 2003
    cr, cc, cv, m, ak, ar, ac, av, W = random_box_triplets(n, 30, 5, 3 * n, 3, 7)
    b = general_problem(n, cr, cc, cv, m, ak, ar, ac, av, np.zeros(m)).A_of(W)
    t = (cr, cc, cv, m, ak, ar, ac, av, b)
    prob = L.Problem.general(n, *t).upload(ctx)
    op = general_problem(n, *t)
    print_case(test="gen_solve", case="box n=2003")
    R0 = init_factor(n, 16, 5)
    rc, res, R, y = gpu_solve(ctx, prob, R0, L.F64, op.m)
    ores = alm_solve(op, R0, opts=OOptions())
    print(res.as_dict(), "oracle", ores.obj, ores.outer, ores.inner)
    assert rc == L.OK and ores.converged
    assert abs(res.obj - ores.obj) <= 1e-5 * abs(ores.obj)
    m = K.alm_measures(op, R, y)
    assert m["err1"] <= 1e-5 and abs(m["err3"]) <= 1e-5
    lam = certify.lambda_min(op, y)
    cert = L.certify(ctx, prob, torch.from_numpy(y).cuda(), max_iter=400, tol=1e-8 * (1 + op.c_l1))
    print("lambda_min oracle", lam, "gpu", cert.as_dict())
    assert abs(cert.lambda_min - lam) <= max(cert.resid, 1e-8 * (1 + op.c_l1))
    assert np.isnan(cert.dual_bound)
    assert lam >= -1e-5 * (1 + op.c_l1)            # a certified optimum (err2 <= tol)


def test_maxcut_as_general_matches_maxcut_path(ctx):
    n = 800
    u, v = erdos_renyi_edges(n, 4000, 17)
    w = pm1_weights(4000, 18)
    deg = np.zeros(n)
    np.add.at(deg, u, w)
    np.add.at(deg, v, w)
    k = np.arange(n, dtype=np.int32)
    t = (np.concatenate([u, k]), np.concatenate([v, k]), np.concatenate([0.25 * w, -0.25 * deg]),
         n, k, k, k, np.ones(n), np.ones(n))
    print_case(test="maxcut_as_general")
    gp = L.Problem.general(n, *t).upload(ctx)
    mp = L.Problem.maxcut(n, u, v, w).upload(ctx)
    R0 = init_factor(n, 12, 19)
    rcg, resg, Rg, yg = gpu_solve(ctx, gp, R0, L.F64, n)
    rcm, resm, Rm, ym = gpu_solve(ctx, mp, R0, L.F64, n)
    ores = alm_solve(maxcut_problem(n, u, v, w), R0, opts=OOptions())
    print("general", resg.as_dict(), "maxcut", resm.as_dict(), "oracle", ores.obj)
    assert rcg == L.OK and rcm == L.OK
    assert abs(resg.obj - resm.obj) <= 1e-5 * abs(resm.obj)
    assert abs(resg.obj - ores.obj) <= 1e-5 * abs(ores.obj)


@pytest.mark.parametrize("storage", STORAGE)
def test_general_certificate_parity(ctx, storage):
    prob, op, r = setup(ctx, "theta_dense", storage)
    print_case(test="gen_certify", case="theta_dense", storage=storage)
    y = np.random.default_rng(9).standard_normal(op.m)
    scale = float(abs(op.C - op.A_adj(y)).sum(axis=1).max())
    cert = L.certify(ctx, prob, dev_vec(y), max_iter=300, tol=1e-9 * scale)
    lam = certify.lambda_min(op, y)
    print(cert.as_dict(), "oracle", lam)
    assert abs(cert.lambda_min - lam) <= max(cert.resid, 1e-9 * scale)
    assert abs(cert.by - float(op.b @ y)) <= 1e-12 * np.abs(op.b * y).sum() + 1e-300


def test_general_strict_reopt(ctx):
    # the strict level's err2 comes from the GPU certificate on the general
    # operator; the oracle's dense eigensolver on the returned y agrees
    prob, op, r = setup(ctx, "random_small")
    print_case(test="gen_reopt", case="random_small")
    R0 = init_factor(op.n, r, 4)
    rc, res, R, y = gpu_solve(ctx, prob, R0, L.F64, op.m, reopt=2)
    print(res.as_dict())
    assert rc == L.OK
    m = K.alm_measures(op, R, y)
    assert m["err1"] <= 1e-5 and abs(m["err3"]) <= 1e-5
    e2 = certify.err2(op, y)
    assert res.err2 <= 1e-5 and abs(res.err2 - e2) <= 1e-6


@pytest.mark.parametrize("case", ["two_theta", "slack"])
def test_blocks_closed_forms(ctx, case):
    from oracle.problem import general_blocks_problem
    from test_oracle_general import theta_with_slack_block, two_theta_blocks
    args = two_theta_blocks() if case == "two_theta" else theta_with_slack_block()
    want = math.sqrt(5) + 4.0 if case == "two_theta" else math.sqrt(5)
    print_case(test="blocks", case=case)
    prob = L.Problem.general_blocks(*args).upload(ctx)
    op = general_blocks_problem(*args)
    R0 = init_factor(op.n, 6 if case == "two_theta" else 4, 3)
    rc, res, R, y = gpu_solve(ctx, prob, R0, L.F64, op.m, tol=1e-8)
    ores = alm_solve(op, R0, opts=OOptions(tol=1e-8))
    print(res.as_dict(), "oracle", ores.obj, "closed form", -want)
    assert rc == L.OK and ores.converged
    assert -res.obj == pytest.approx(want, rel=1e-6)
    assert abs(res.obj - ores.obj) <= 1e-7 * want
    m = K.alm_measures(op, R, y)
    assert abs(m["obj"] - res.obj) <= 1e-10 * want


def test_block_ranks_iterates_and_solve_match_oracle(ctx):
    # blocks of orders 4 and 6 with ranks 1 and 3 (trace-one blocks: the optimum
    # is the sum of the blocks' smallest eigenvalues, reached at rank one); the
    # caller's factor has values in the masked entries, which the solve zeroes
    from oracle.problem import general_blocks_problem
    from test_oracle_general import trace_blocks
    args, mats = trace_blocks([4, 6], 7)
    print_case(test="block_ranks", ranks=[1, 3])
    op = general_blocks_problem(*args, block_rank=[1, 3])
    prob = L.Problem.general_blocks(*args, block_rank=[1, 3]).upload(ctx)
    R0 = init_factor(10, 3, 8)
    kw = dict(max_outer=1, max_inner=6, eta0=1e-14)
    rc, res, R, y = gpu_solve(ctx, prob, R0, L.F64, op.m, **kw)
    ores = alm_solve(op, R0, opts=OOptions(**kw))
    assert res.inner == ores.inner == 6
    assert np.all(R[:4, 1:] == 0.0)
    assert np.max(np.abs(R - ores.R)) <= 1e-9 * (1.0 + np.abs(ores.R).max())
    rc, res, R, y = gpu_solve(ctx, prob, R0, L.F64, op.m, tol=1e-9)
    want = sum(np.linalg.eigvalsh(M)[0] for M in mats)
    print(res.as_dict(), "closed form", want)
    assert rc == L.OK
    assert res.obj == pytest.approx(want, rel=1e-6, abs=1e-7)
    assert np.all(R[:4, 1:] == 0.0)


@pytest.mark.parametrize("rank", [1, 2])
def test_block_rank_one_cannot_hold_two_orthogonal_unit_rows(ctx, rank):
    # X_00 = X_11 = 1, X_01 = 0 needs rank 2 (closed form: a rank-one factor has
    # X_01 = +-1 once both diagonal constraints hold)
    args = ([2], np.array([0, 0], np.int32), np.array([0, 1], np.int32), np.array([0, 1], np.int32),
            np.array([1.0, 0.5]), 3, np.array([0, 1, 2], np.int32), np.zeros(3, np.int32),
            np.array([0, 1, 0], np.int32), np.array([0, 1, 1], np.int32), np.ones(3), np.array([1.0, 1.0, 0.0]))
    print_case(test="block_rank_orthogonal", rank=rank)
    prob = L.Problem.general_blocks(*args, block_rank=[rank]).upload(ctx)
    rc, res, R, y = gpu_solve(ctx, prob, init_factor(2, 2, 9), L.F64, 3, max_outer=30)
    print(res.as_dict())
    if rank == 1:
        assert rc != L.OK and res.err1 > 0.05
    else:
        assert rc == L.OK and res.obj == pytest.approx(1.5, rel=1e-5)


@pytest.mark.parametrize("case,storage", [("random_small", L.C_SPARSE), ("theta_dense", L.C_DENSE),
                                          ("random_small", L.C_DENSE)])
def test_admm_step_parity(ctx, case, storage):
    # splitting iterations (Section 2.2) on a general problem: CG half-steps with
    # C V formed once per half-step, against the oracle's CG on eq. 2.2, both to
    # 1e-12 of the right-hand side
    import torch
    from oracle.alm import admm_step
    prob, op, r = setup(ctx, case, storage)
    print_case(test="gen_admm", case=case, storage=storage)
    rng = np.random.default_rng(51)
    U = 0.3 * rng.standard_normal((op.n, r))
    V = U + 0.03 * rng.standard_normal((op.n, r))
    y = 0.1 * rng.standard_normal(op.m)
    sigma = 2.0
    Ud, Vd = dev_factor(U, L.F64), dev_factor(V, L.F64)
    yd = torch.from_numpy(y.copy()).cuda()
    L.k_admm(ctx, prob, L.F64, Ud, Vd, yd, sigma, 2, cg_tol=1e-12, cg_max=2000)
    torch.cuda.synchronize()
    Uo, Vo, yo = U, V, y
    for _ in range(2):
        Uo, Vo, yo = admm_step(op, Uo, Vo, yo, sigma, cg_tol=1e-12, cg_iters=2000)
    scale = 1.0 + np.abs(Uo).max()
    print("max |dU|", np.max(np.abs(host(Ud, r) - Uo)), "max |dy|", np.max(np.abs(yd.cpu().numpy() - yo)))
    assert np.max(np.abs(host(Ud, r) - Uo)) <= 1e-9 * scale
    assert np.max(np.abs(host(Vd, r) - Vo)) <= 1e-9 * scale
    assert np.max(np.abs(yd.cpu().numpy() - yo)) <= 1e-9 * (1.0 + np.abs(yo).max()) * scale
    assert np.all(host(Ud)[:, r:] == 0.0)


@pytest.mark.parametrize("case", ["petersen", "random_small"])
def test_solve_phase2_matches_oracle(ctx, case):
    # ALM, then the splitting phase, to 1e-7 on both sides.  The random instance
    # has several stationary points and the two sides' L-BFGS paths part after a
    # few hundred iterations, so it switches after the first ALM step (err1 <=
    # 0.1; four L-BFGS iterations, equal on both sides up to rounding) and the
    # splitting phases start from the same point.
    if case == "petersen":
        u, v = petersen_edges()
        n, t, r = 10, theta_triplets(10, u, v), 6
        switch = 1e-3
    else:
        n, t, r = case_data(case)
        switch = 1e-1
    prob = L.Problem.general(n, *t).upload(ctx)
    op = general_problem(n, *t)
    print_case(test="gen_solve_phase2", case=case)
    R0 = init_factor(n, r, 4)
    rc, res, R, y = gpu_solve(ctx, prob, R0, L.F64, op.m, tol=1e-7, phase2=1, switch_err1=switch)
    ores = alm_solve(op, R0, opts=OOptions(tol=1e-7, phase2=True, switch_err1=switch))
    print(res.as_dict(), "oracle", ores.obj, ores.converged, ores.admm_iters, ores.admm_fallbacks)
    assert rc == L.OK and ores.converged
    assert res.admm_iters > 0 and res.admm_fallbacks == ores.admm_fallbacks == 0
    assert abs(res.obj - ores.obj) <= 1e-5 * abs(ores.obj)
    if case == "petersen":
        assert res.obj == pytest.approx(-4.0, rel=1e-6)
    m = K.alm_measures(op, R, y)
    assert m["err1"] <= 1e-7 and abs(m["err3"]) <= 1e-7
