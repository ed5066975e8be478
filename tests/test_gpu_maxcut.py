"""GPU parity of the MaxCut hot path against the FP64 oracle.

Per kernel (same inputs on both sides): float64 results agree to 1e-10 of the
sum of absolute values of the terms that make each output (a bound that does
not divide by the result, which can cancel to zero); float32 storage is
checked against the oracle evaluated on the float32-rounded inputs with a
float32-sized bound.  End to end: the solve reaches err1 <= 1e-5 and
|err3| <= 1e-5 and its objective matches the oracle's solve to 1e-5 relative.
"""

import numpy as np
import pytest

from oracle import certify
from oracle import kernels as K
from oracle.alm import Options as OOptions
from oracle.alm import alm_solve
from oracle.lbfgs import two_loop
from oracle.problem import maxcut_problem
from synth import chung_lu_edges, erdos_renyi_edges, init_factor, pm1_weights

from paper_2407_15049_amd import lrsdp as L
from gpu_util import dev_factor, dev_vec, host, rounded

pytestmark = pytest.mark.gpu

TOL = {L.F64: 1e-10, L.F32: 1e-4}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.Context(0)


def graph(case):
    """(n, u, v, w, r): ragged sizes, heavy rows, weights, isolated nodes, empty."""
    if case == "er_1k":
        u, v = erdos_renyi_edges(1000, 5000, 15049)
        return 1000, u, v, None, 10
    if case == "pm1_ragged":
        u, v = erdos_renyi_edges(777, 3001, 3)
        return 777, u, v, pm1_weights(3001, 4), 20
    if case == "general":
        u, v = erdos_renyi_edges(501, 2000, 5)
        return 501, u, v, np.random.default_rng(6).uniform(-2, 3, 2000), 8
    if case == "cl_heavy":
        u, v = chung_lu_edges(20000, 100000, 2.5, 7)
        return 20000, u, v, None, 24
    if case == "isolated":
        u, v = erdos_renyi_edges(100, 400, 8)
        return 300, u, v, None, 6
    if case == "empty":
        return 10, np.zeros(0, np.int32), np.zeros(0, np.int32), None, 4
    if case == "wide32":
        u, v = erdos_renyi_edges(333, 1500, 9)
        return 333, u, v, None, 32
    if case == "degree_ladder":
        return degree_ladder(general=False)
    if case == "ladder_general":
        return degree_ladder(general=True)
    raise KeyError(case)


def degree_ladder(general):
    """Hub rows of every degree around the gather's batch and lane-group sizes
    (0-40, 63-65, 127-130 around the 128-entry segment length, 255-257) joined
    to distinct leaves drawn from a pool of other nodes; +-1 weights (or real
    weights in [-2, 3) when `general`), rank 20."""
    rng = np.random.default_rng(20)
    degrees = list(range(0, 41)) + [63, 64, 65, 127, 128, 129, 130, 255, 256, 257]
    hubs = len(degrees)
    n = hubs + 2000
    us, vs = [], []
    for h, d in enumerate(degrees):
        leaves = hubs + rng.choice(n - hubs, size=d, replace=False)
        us.append(np.full(d, h))
        vs.append(leaves)
    u = np.concatenate(us).astype(np.int32)
    v = np.concatenate(vs).astype(np.int32)
    perm = rng.permutation(n).astype(np.int32)      # spread the hubs over the work-list windows
    w = rng.uniform(-2, 3, len(u)) if general else pm1_weights(len(u), 21)
    return n, perm[u], perm[v], w, 20


CASES = ["er_1k", "pm1_ragged", "general", "cl_heavy", "isolated", "empty", "wide32", "degree_ladder", "ladder_general"]


def setup(ctx, case):
    n, u, v, w, r = graph(case)
    prob = L.Problem.maxcut(n, u, v, w).upload(ctx)
    oprob = maxcut_problem(n, u, v, w)
    return n, r, prob, oprob


def print_case(**kw):
    print("CASE", kw, flush=True)


@pytest.mark.parametrize("prec", [L.F64, L.F32])
@pytest.mark.parametrize("case", CASES)
def test_spmm_parity(ctx, case, prec):
    import torch
    n, r, prob, op = setup(ctx, case)
    if prec == L.F32 and r * 4 > 256:
        pytest.skip("rank too wide for float32 rows")
    print_case(test="spmm", case=case, prec=prec, n=n, r=r)
    rng = np.random.default_rng(11)
    V = rounded(rng.standard_normal((n, r)), prec)
    ytil = rng.standard_normal(n)
    Vd = dev_factor(V, prec)
    Yd = torch.full_like(Vd, np.nan)
    L.k_spmm(ctx, prob, prec, Vd, dev_vec(ytil), Yd)
    torch.cuda.synchronize()
    Y = host(Yd)
    assert np.all(Y[:, r:] == 0.0), "pad columns must stay zero"
    Yo = K.spmm(op, ytil, V)
    bound = abs(op.C) @ np.abs(V) + np.abs(ytil)[:, None] * np.abs(V)
    err = np.abs(Y[:, :r] - Yo)
    assert np.all(err <= TOL[prec] * bound + 1e-300), f"max ratio {np.max(err / (bound + 1e-300))}"
    # no shift
    L.k_spmm(ctx, prob, prec, Vd, None, Yd)
    torch.cuda.synchronize()
    Y0 = host(Yd, r)
    b0 = abs(op.C) @ np.abs(V)
    assert np.all(np.abs(Y0 - K.spmm(op, None, V)) <= TOL[prec] * b0 + 1e-300)
    # deterministic: bitwise equal on a second run
    Y2d = torch.empty_like(Vd)
    L.k_spmm(ctx, prob, prec, Vd, None, Y2d)
    torch.cuda.synchronize()
    assert torch.equal(Y2d, Yd)


@pytest.mark.parametrize("prec", [L.F64, L.F32])
@pytest.mark.parametrize("case", ["er_1k", "pm1_ragged", "cl_heavy", "empty"])
def test_constraint_map_parity(ctx, case, prec):
    import torch
    n, r, prob, op = setup(ctx, case)
    print_case(test="constraint", case=case, prec=prec)
    rng = np.random.default_rng(12)
    U = rounded(rng.standard_normal((n, r)), prec)
    V = rounded(rng.standard_normal((n, r)), prec)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    L.k_constraint(ctx, prob, prec, dev_factor(U, prec), dev_factor(V, prec), out)
    torch.cuda.synchronize()
    ref = K.constraint_map(op, U, V)
    bound = np.sum(np.abs(U) * np.abs(V), axis=1)
    assert np.all(np.abs(out.cpu().numpy() - ref) <= 1e-12 * bound + 1e-300)
    L.k_constraint(ctx, prob, prec, dev_factor(U, prec), None, out)
    torch.cuda.synchronize()
    assert np.allclose(out.cpu().numpy(), np.sum(U * U, axis=1), rtol=1e-12, atol=0)


@pytest.mark.parametrize("prec", [L.F64, L.F32])
@pytest.mark.parametrize("case", ["er_1k", "pm1_ragged", "general", "cl_heavy", "isolated", "degree_ladder", "ladder_general"])
def test_linesearch_coeffs_parity(ctx, case, prec):
    import torch
    n, r, prob, op = setup(ctx, case)
    if prec == L.F32 and r * 4 > 256:
        pytest.skip("rank too wide")
    print_case(test="ls_coeffs", case=case, prec=prec)
    rng = np.random.default_rng(13)
    R = rounded(rng.standard_normal((n, r)) / np.sqrt(r), prec)
    D = rounded(rng.standard_normal((n, r)) * 0.1, prec)
    y = rng.standard_normal(n)
    sigma = 2.7
    Rd, Dd = dev_factor(R, prec), dev_factor(D, prec)
    ld = Rd.shape[1]
    esz = 8 if prec == L.F64 else 4
    work = torch.empty(2 * n * ld * esz + 8 * n, dtype=torch.uint8, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    q1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    q2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    L.k_ls_coeffs(ctx, prob, prec, Rd, Dd, dev_vec(y), sigma, work, out, q1, q2)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    c = K.linesearch_coeffs(op, R, D, y, sigma)
    ytil = y + sigma * c["q0"]
    absC = abs(op.C)
    aR, aD = np.abs(R), np.abs(D)
    bq1 = 2 * np.sum(aR * aD, axis=1)
    bq2 = np.sum(aD * aD, axis=1)
    bp1 = 2 * np.sum((absC @ aR) * aD)
    bp2 = np.sum((absC @ aD) * aD)
    tol = 1e-10 if prec == L.F64 else 1e-4
    assert np.all(np.abs(q1.cpu().numpy() - c["q1"]) <= 1e-12 * bq1 + 1e-300)
    assert np.all(np.abs(q2.cpu().numpy() - c["q2"]) <= 1e-12 * bq2 + 1e-300)
    bounds = {
        "a1": 0.5 * sigma * np.sum(bq2 * bq2),
        "a2": sigma * np.sum(bq1 * bq2),
        "a3": bp2 + np.sum(np.abs(ytil) * bq2) + 0.5 * sigma * np.sum(bq1 * bq1),
        "a4": bp1 + np.sum(np.abs(ytil) * bq1),
        "p1": bp1, "p2": bp2,
    }
    for idx, name in enumerate(["a1", "a2", "a3", "a4", "p1", "p2"]):
        assert abs(g[idx] - c[name]) <= tol * bounds[name], (name, g[idx], c[name])


def test_cubic_parity(ctx):
    import torch
    rng = np.random.default_rng(14)
    cases = []
    for _ in range(300):
        a1 = abs(rng.standard_normal()) * 10 ** rng.uniform(-6, 3)
        a2, a3 = rng.standard_normal(2) * 10 ** rng.uniform(-3, 3, 2)
        a4 = -abs(rng.standard_normal()) * 10 ** rng.uniform(-6, 3)
        cases.append((a1, a2, a3, a4))
    cases += [(0.0, 0.0, 2.0, -3.0), (1.0, 0.0, 1.0, 0.5), (0.0, 0.0, 0.0, 0.0), (1.0, -4.0, 4.0, -0.1),
              (0.0, 1.0, -1.0, -0.5), (0.0, -1.0, 2.0, -0.5), (1e-30, 1.0, 2.0, -1.0), (2.0, 0.0, 0.0, -1.0)]
    a = torch.tensor(cases, dtype=torch.float64, device="cuda")
    taus = torch.zeros(len(cases), dtype=torch.float64, device="cuda")
    for i in range(len(cases)):
        L.k_cubic(ctx, a[i], taus[i:i + 1])
    torch.cuda.synchronize()
    tg = taus.cpu().numpy()
    for (a1, a2, a3, a4), t in zip(cases, tg):
        to = K.exact_step(a1, a2, a3, a4)
        fo, fg = K.quartic((a1, a2, a3, a4), to), K.quartic((a1, a2, a3, a4), t)
        scale = abs(a4) * max(to, t) + 1e-300
        assert abs(fg - fo) <= 1e-9 * (abs(fo) + scale), ((a1, a2, a3, a4), t, to)
        if to > 0:
            assert abs(t - to) <= 1e-7 * to, ((a1, a2, a3, a4), t, to)
        else:
            assert t == 0.0


@pytest.mark.parametrize("prec", [L.F64, L.F32])
@pytest.mark.parametrize("case", ["er_1k", "pm1_ragged", "cl_heavy", "isolated"])
def test_alm_step_parity(ctx, case, prec):
    import torch
    n, r, prob, op = setup(ctx, case)
    if prec == L.F32 and r * 4 > 256:
        pytest.skip("rank too wide")
    print_case(test="alm", case=case, prec=prec)
    rng = np.random.default_rng(15)
    R = rounded(init_factor(n, r, 3) * (1 + 0.05 * rng.standard_normal((n, 1))), prec)
    y = rng.standard_normal(n)
    sigma = 1.3
    Rd = dev_factor(R, prec)
    yd = dev_vec(y)
    work = torch.empty_like(Rd)
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    L.k_alm(ctx, prob, prec, Rd, yd, sigma, work, out)
    torch.cuda.synchronize()
    ynew = K.multiplier_estimate(op, R, y, sigma)
    m = K.alm_measures(op, R, ynew)
    assert np.allclose(yd.cpu().numpy(), ynew, rtol=0, atol=1e-13 * (1 + np.abs(y).max() + sigma))
    g = out.cpu().numpy()
    bobj = np.sum((abs(op.C) @ np.abs(R)) * np.abs(R))
    assert abs(g[0] - m["obj"]) <= TOL[prec] * bobj + 1e-300
    assert abs(g[1] - m["dual"]) <= 1e-12 * np.abs(ynew).sum()
    assert abs(g[2] - m["res_norm"]) <= 1e-9 * (1 + m["res_norm"])
    assert abs(g[3] - m["err1"]) <= 1e-9 * (1 + m["err1"])
    assert abs(g[5] - m["err3"]) <= 1e-9


@pytest.mark.parametrize("prec", [L.F64, L.F32])
@pytest.mark.parametrize("k", [0, 1, 3, 4, 8])
def test_lbfgs_direction_parity(ctx, prec, k):
    import torch
    n, r = 2053, 12
    rng = np.random.default_rng(16 + k)
    # pairs from a separable SPD quadratic: y = H s with positive diagonal H
    h = rng.uniform(0.5, 5.0, (n, r))
    S = [rounded(rng.standard_normal((n, r)), prec) for _ in range(k)]
    Y = [rounded(h * s, prec) for s in S]
    G = rounded(rng.standard_normal((n, r)), prec)
    Dd = dev_factor(np.zeros((n, r)), prec)
    L.k_lbfgs_dir(ctx, prec, dev_factor(G, prec), [dev_factor(s, prec) for s in S],
                  [dev_factor(y, prec) for y in Y], Dd)
    torch.cuda.synchronize()
    Dg = host(Dd, r)
    Do = two_loop(G, list(zip(S, Y)))
    tol = 1e-10 if prec == L.F64 else 2e-6
    assert np.linalg.norm(Dg - Do) <= tol * np.linalg.norm(Do)


def gpu_solve(ctx, n, u, v, w, R0, prec, **kw):
    import torch
    r = R0.shape[1]
    prob = L.Problem.maxcut(n, u, v, w).upload(ctx)
    rank = kw.pop("rank", r)          # R0 may carry zero columns beyond the rank (dynamic rank)
    opts = L.default_options(prec=prec, rank=rank, ld=L.padded_ld(r, L.F64 if prec == L.F64 else L.F32), **kw)
    Rd = dev_factor(R0, prec)
    yd = torch.zeros(n, dtype=torch.float64, device="cuda")
    rc, res = L.solve(ctx, prob, Rd, yd, opts)
    torch.cuda.synchronize()
    return rc, res, host(Rd, r), yd.cpu().numpy()


def test_solve_er_1k_matches_oracle(ctx):
    n, u, v, w, r = graph("er_1k")
    print_case(test="solve", case="er_1k", prec="f64", r=r)
    R0 = init_factor(n, r, 15050)
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, L.F64)
    op = maxcut_problem(n, u, v, w)
    ores = alm_solve(op, R0, opts=OOptions())
    assert rc == L.OK and ores.converged
    assert res.err1 <= 1e-5 and abs(res.err3) <= 1e-5
    assert abs(res.obj - ores.obj) <= 1e-5 * abs(ores.obj)
    # the library's reported measures agree with the oracle's recomputation
    m = K.alm_measures(op, R, y)
    assert abs(m["obj"] - res.obj) <= 1e-10 * abs(res.obj)
    assert abs(m["err1"] - res.err1) <= 1e-10 + 1e-8 * res.err1


def test_solve_er_1k_rank16_certified(ctx):
    n, u, v, w, _ = graph("er_1k")
    print_case(test="solve", case="er_1k", prec="f64", r=16)
    R0 = init_factor(n, 16, 15051)
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, L.F64)
    op = maxcut_problem(n, u, v, w)
    bound = certify.maxcut_dual_bound(op, y)
    assert rc == L.OK
    assert (res.obj - bound) / (1 + abs(bound)) <= 2e-5
    assert bound <= res.obj + 1e-9 * abs(res.obj)


@pytest.mark.parametrize("case", ["pm1_ragged", "cl_heavy", "isolated"])
def test_solve_small_cases_converge(ctx, case):
    n, u, v, w, r = graph(case)
    r = min(r, 16)
    print_case(test="solve", case=case, prec="f64", r=r)
    R0 = init_factor(n, r, 99)
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, L.F64)
    op = maxcut_problem(n, u, v, w)
    assert rc == L.OK, res.as_dict()
    m = K.alm_measures(op, R, y)
    assert m["err1"] <= 1e-5 and abs(m["err3"]) <= 1e-5


def test_solve_f32_er_1k(ctx):
    n, u, v, w, _ = graph("er_1k")
    print_case(test="solve", case="er_1k", prec="f32", r=12)
    R0 = init_factor(n, 12, 15052)
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, L.F32)
    rc64, res64, _, _ = gpu_solve(ctx, n, u, v, w, R0, L.F64)
    op = maxcut_problem(n, u, v, w)
    m = K.alm_measures(op, R, y)       # float64 recomputation of the float32 result
    print("F32", res.as_dict(), "F64", res64.as_dict(), "oracle-measured", m)
    assert rc == L.OK
    assert m["err1"] <= 1e-5 and abs(m["err3"]) <= 1e-5
    assert abs(res.obj - res64.obj) <= 1e-5 * abs(res64.obj)


def test_solve_reports_limits(ctx):
    n, u, v, w, r = graph("er_1k")
    R0 = init_factor(n, r, 5)
    rc, res, _, _ = gpu_solve(ctx, n, u, v, w, R0, L.F64, max_outer=1)
    assert rc == L.NOT_CONVERGED and res.outer == 1 and res.err1 > 0


@pytest.mark.parametrize("case", ["er_1k", "pm1_ragged", "general", "cl_heavy", "isolated", "degree_ladder", "ladder_general"])
def test_spmm_bf16_input_parity(ctx, case):
    # bfloat16 gathered operand, float32 accumulation and output
    import torch
    n, r, prob, op = setup(ctx, case)
    print_case(test="spmm_bf16", case=case, n=n, r=r)
    ld = L.padded_ld(r, L.F32)
    ldb = (ld + 7) // 8 * 8
    rng = np.random.default_rng(17)
    Vb = torch.from_numpy(rng.standard_normal((n, r)).astype(np.float32)).to(torch.bfloat16)
    V = Vb.to(torch.float64).numpy()                 # exact values the device holds
    Vd = torch.zeros((n, ldb), dtype=torch.bfloat16, device="cuda")
    Vd[:, :r] = Vb.cuda()
    ytil = rng.standard_normal(n)
    Yd = torch.full((n, ld), np.nan, dtype=torch.float32, device="cuda")
    L._check(L.load().lrsdp_k_spmm(ctx.handle, prob.handle, L.F32_BF16IN, L._ptr(Vd), ld,
                                   L._ptr(dev_vec(ytil)), L._ptr(Yd)))
    torch.cuda.synchronize()
    Y = host(Yd)
    assert np.all(Y[:, r:] == 0.0)
    Yo = K.spmm(op, ytil, V)
    bound = abs(op.C) @ np.abs(V) + np.abs(ytil)[:, None] * np.abs(V)
    assert np.all(np.abs(Y[:, :r] - Yo) <= 1e-4 * bound + 1e-300)


def test_solve_bf16_input_er_1k(ctx):
    n, u, v, w, _ = graph("er_1k")
    print_case(test="solve", case="er_1k", prec="bf16in", r=12)
    R0 = init_factor(n, 12, 15052)
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, L.F32_BF16IN, refresh_every=25)
    rc64, res64, _, _ = gpu_solve(ctx, n, u, v, w, R0, L.F64)
    op = maxcut_problem(n, u, v, w)
    m = K.alm_measures(op, R, y)
    print("BF16IN", res.as_dict(), "F64", res64.as_dict(), "oracle-measured", m)
    assert rc == L.OK
    assert m["err1"] <= 1e-5 and abs(m["err3"]) <= 1e-5
    assert abs(res.obj - res64.obj) <= 1e-4 * abs(res64.obj)


def test_solve_refresh_every_matches(ctx):
    n, u, v, w, r = graph("er_1k")
    R0 = init_factor(n, r, 15050)
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, L.F64, refresh_every=16)
    ores = alm_solve(maxcut_problem(n, u, v, w), R0, opts=OOptions())
    assert rc == L.OK
    assert abs(res.obj - ores.obj) <= 1e-5 * abs(ores.obj)


@pytest.mark.parametrize("case", ["er_1k", "pm1_ragged", "cl_heavy", "isolated"])
def test_admm_step_parity(ctx, case):
    # splitting iterations: per-row exact solves on the GPU vs CG (Algorithm 2) in the oracle
    import torch
    from oracle.alm import admm_step
    n, r, prob, op = setup(ctx, case)
    r = min(r, 16)
    print_case(test="admm", case=case)
    rng = np.random.default_rng(18)
    U = init_factor(n, r, 19) + 0.01 * rng.standard_normal((n, r))
    V = U + 0.01 * rng.standard_normal((n, r))
    y = -np.abs(rng.standard_normal(n))
    # A penalty above the default initial one (4 sum|C_ij| / m = 20 on the
    # Chung-Lu graph): at sigma = 3 the iteration diverges on its hub rows and
    # rounding differences grow ~100x per step.
    sigma = 30.0
    Ud, Vd, yd = dev_factor(U, L.F64), dev_factor(V, L.F64), dev_vec(y)
    L.k_admm(ctx, prob, L.F64, Ud, Vd, yd, sigma, 3)
    torch.cuda.synchronize()
    Uo, Vo, yo = U, V, y
    for _ in range(3):
        Uo, Vo, yo = admm_step(op, Uo, Vo, yo, sigma)
    scale = 1.0 + np.abs(Uo).max()
    assert np.max(np.abs(host(Ud, r) - Uo)) <= 1e-9 * scale
    assert np.max(np.abs(host(Vd, r) - Vo)) <= 1e-9 * scale
    assert np.max(np.abs(yd.cpu().numpy() - yo)) <= 1e-9 * (1 + np.abs(yo).max())
    # several iterations in one call equal the same number of single calls
    U2, V2, y2 = dev_factor(U, L.F64), dev_factor(V, L.F64), dev_vec(y)
    L.k_admm(ctx, prob, L.F64, U2, V2, y2, sigma, 3)
    torch.cuda.synchronize()
    U1, V1, y1 = dev_factor(U, L.F64), dev_factor(V, L.F64), dev_vec(y)
    for _ in range(3):
        L.k_admm(ctx, prob, L.F64, U1, V1, y1, sigma, 1)
    torch.cuda.synchronize()
    assert torch.equal(U1, U2) and torch.equal(V1, V2) and torch.equal(y1, y2)


def test_solve_phase2_matches_oracle(ctx):
    n, u, v, w, r = graph("er_1k")
    R0 = init_factor(n, 16, 15051)
    print_case(test="solve_phase2", case="er_1k")
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, L.F64, phase2=1, switch_err1=1e-3)
    ores = alm_solve(maxcut_problem(n, u, v, w), R0, opts=OOptions(phase2=True, switch_err1=1e-3))
    rc0, res0, _, _ = gpu_solve(ctx, n, u, v, w, R0, L.F64)
    print("phase2", res.as_dict(), "oracle", ores.obj, ores.inner, ores.history[-1], "alm only", res0.as_dict())
    assert rc == L.OK and ores.converged and res.admm_iters > 0
    assert abs(res.obj - ores.obj) <= 1e-5 * abs(ores.obj)
    m = K.alm_measures(maxcut_problem(n, u, v, w), R, y)
    assert m["err1"] <= 1e-5 and abs(m["err3"]) <= 1e-5


def test_phase2_forced_fallback_equals_alm_only(ctx):
    # a splitting phase that cannot finish (max_admm = 10 from an early switch) is
    # abandoned; the solve then equals the ALM alone bit for bit, and the oracle's
    # solve with the same options
    n, u, v, w, r = graph("er_1k")
    R0 = init_factor(n, 16, 15051)
    print_case(test="phase2_fallback", case="er_1k")
    rc0, res0, R0g, y0g = gpu_solve(ctx, n, u, v, w, R0, L.F64)
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, L.F64, phase2=1, switch_err1=1e-1, max_admm=10, admm_check=10)
    print(res.as_dict())
    assert rc == L.OK and rc0 == L.OK
    assert res.admm_fallbacks == 1 and res.admm_iters == 10
    assert res.obj == res0.obj and res.inner == res0.inner and res.outer == res0.outer
    assert np.array_equal(R, R0g) and np.array_equal(y, y0g)
    ores = alm_solve(maxcut_problem(n, u, v, w), R0,
                     opts=OOptions(phase2=True, switch_err1=1e-1, max_admm=10, admm_check=10))
    assert ores.admm_fallbacks == 1
    assert abs(res.obj - ores.obj) <= 1e-5 * abs(ores.obj)


def test_phase2_hub_graph_never_fails(ctx):
    # on hub rows the splitting iteration at the switch penalty can diverge; the
    # solve must fall back to the ALM and still converge
    n, u, v, w, r = graph("cl_heavy")
    R0 = init_factor(n, 16, 17)
    print_case(test="phase2_hub", case="cl_heavy")
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, L.F64, phase2=1, switch_err1=1e-3)
    print(res.as_dict())
    assert rc == L.OK, res.as_dict()
    m = K.alm_measures(maxcut_problem(n, u, v, w), R, y)
    assert m["err1"] <= 1e-5 and abs(m["err3"]) <= 1e-5
    if res.admm_fallbacks:
        rc0, res0, _, _ = gpu_solve(ctx, n, u, v, w, R0, L.F64)
        assert res.obj == res0.obj


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("case", ["er_1k", "cl_heavy", "isolated", "general"])
def test_precond_iterates_match_oracle(ctx, case, mode):
    # row-block H0: after a few L-BFGS iterations of the first subproblem the
    # GPU iterate equals the oracle's (same directions, steps and pairs)
    import torch
    n, u, v, w, r = graph(case)
    r = min(r, 16)
    print_case(test="precond_iterates", case=case)
    R0 = init_factor(n, r, 23)
    op = maxcut_problem(n, u, v, w)
    kw = dict(precond=mode, max_outer=1, max_inner=6, eta0=1e-14)
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, L.F64, **kw)
    ores = alm_solve(op, R0, opts=OOptions(precond=mode, max_outer=1, max_inner=6, eta0=1e-14))
    print(res.as_dict(), ores.inner)
    assert res.inner == ores.inner == 6
    scale = 1.0 + np.abs(ores.R).max()
    assert np.max(np.abs(R - ores.R)) <= 1e-9 * scale
    assert np.max(np.abs(y - ores.y)) <= 1e-9 * (1.0 + np.abs(ores.y).max())


def test_precond_solve_matches_oracle(ctx):
    n, u, v, w, _ = graph("er_1k")
    R0 = init_factor(n, 16, 15051)
    print_case(test="precond_solve", case="er_1k")
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, L.F64, precond=1)
    ores = alm_solve(maxcut_problem(n, u, v, w), R0, opts=OOptions(precond=True))
    rc0, res0, _, _ = gpu_solve(ctx, n, u, v, w, R0, L.F64)
    print("precond", res.as_dict(), "oracle", ores.obj, ores.inner, "plain", res0.as_dict())
    assert rc == L.OK and ores.converged
    assert abs(res.obj - ores.obj) <= 1e-5 * abs(ores.obj)
    assert abs(res.obj - res0.obj) <= 2e-5 * abs(res0.obj)       # same certified optimum
    assert res.inner < res0.inner


@pytest.mark.parametrize("prec", [L.F64, L.F32])
def test_precond_hub_graph_converges_faster(ctx, prec):
    n, u, v, w, _ = graph("cl_heavy")
    R0 = init_factor(n, 16, 29)
    print_case(test="precond_hub", prec=prec)
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, R0, prec, precond=1)
    rc0, res0, _, _ = gpu_solve(ctx, n, u, v, w, R0, prec)
    print("precond", res.as_dict(), "plain", res0.as_dict())
    assert rc == L.OK and rc0 == L.OK
    m = K.alm_measures(maxcut_problem(n, u, v, w), R, y)
    assert m["err1"] <= 1e-5 and abs(m["err3"]) <= 1e-5
    assert res.inner < res0.inner


def test_rank_growth_columns_match_the_oracle_generator(ctx):
    # growth after the first ALM step: the new columns are the generator's values
    n, u, v, w, _ = graph("pm1_ragged")
    R0 = init_factor(n, 10, 31)
    print_case(test="rank_growth_columns", case="pm1_ragged")
    kw = dict(max_outer=1, max_inner=50, rank_max=16, rank_trigger=5, rank_scale=0.03, rank_seed=777)
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, np.hstack([R0, np.zeros((n, 6))]), L.F64, rank=10, **kw)
    ores = alm_solve(maxcut_problem(n, u, v, w), R0, opts=OOptions(**kw))
    print(res.as_dict(), ores.rank_final)
    assert res.rank_final == ores.rank_final == 15
    assert np.max(np.abs(R[:, 10:15] - ores.R[:, 10:15])) <= 1e-14
    assert np.all(R[:, 15:] == 0.0)
    assert np.max(np.abs(R[:, :10] - ores.R[:, :10])) <= 1e-9 * (1 + np.abs(ores.R).max())


def test_rank_growth_solve_matches_oracle(ctx):
    # rank 10 start on the 1k-node graph (non-global stationary point at rank 10)
    n, u, v, w, _ = graph("er_1k")
    R0 = init_factor(n, 10, 15050)
    print_case(test="rank_growth_solve", case="er_1k")
    # the schedule this case was built on (penalty x2, 2000 iterations, two pairs),
    # on both sides: whether a subproblem reaches rank_trigger decides the growth
    kw = dict(rank_max=16, rank_trigger=100, sigma_factor=2.0, max_inner=2000, lbfgs_mem=2)
    rc, res, R, y = gpu_solve(ctx, n, u, v, w, np.hstack([R0, np.zeros((n, 6))]), L.F64, rank=10, **kw)
    ores = alm_solve(maxcut_problem(n, u, v, w), R0, opts=OOptions(**kw))
    print(res.as_dict(), "oracle", ores.obj, ores.rank_final)
    assert rc == L.OK and ores.converged
    assert res.rank_final == ores.rank_final
    assert abs(res.obj - ores.obj) <= 1e-5 * abs(ores.obj)
    assert res.obj < -3906.0                    # below the rank-10 stationary value -3905.98
