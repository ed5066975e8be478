"""MaxCut problems relabelled by degree inside the library (LRSDP_ORDER_DEGREE).

Relabelling is a symmetric permutation of C, so the problem is the same: the
solve, the certificate, the warm start and rank growth take and return every
per-node array in the caller's labels, and their results are the oracle's on
the caller's problem up to the order of summation.  Cases: the first L-BFGS
iterates against the oracle's (bound 1e-9, as for the other iterate tests),
a full solve re-measured by the oracle, growth columns equal to the oracle
generator's, the certificate and the warm start against the input-order
problem, and the per-kernel entry points refusing such a problem.
"""

import numpy as np
import pytest

from oracle import kernels as K
from oracle.alm import Options as OOptions
from oracle.alm import alm_solve
from oracle.problem import maxcut_problem
from synth import init_factor

from paper_2407_15049_amd import lrsdp as L
from gpu_util import dev_factor, host
from test_gpu_maxcut import graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.Context(0)


def print_case(**kw):
    print("CASE", kw, flush=True)


def solve_ordered(ctx, n, u, v, w, R0, prec, node_order, **kw):
    import torch
    r = R0.shape[1]
    prob = L.Problem.maxcut(n, u, v, w, node_order=node_order).upload(ctx)
    rank = kw.pop("rank", r)
    opts = L.default_options(prec=prec, rank=rank, ld=L.padded_ld(r, L.F64 if prec == L.F64 else L.F32), **kw)
    Rd = dev_factor(R0, prec)
    yd = torch.zeros(n, dtype=torch.float64, device="cuda")
    rc, res = L.solve(ctx, prob, Rd, yd, opts)
    torch.cuda.synchronize()
    return prob, rc, res, host(Rd, r), yd.cpu().numpy()


def test_degree_order_is_recorded(ctx):
    n, u, v, w, _ = graph("cl_heavy")
    assert L.Problem.maxcut(n, u, v, w).info.node_order == L.ORDER_INPUT
    assert L.Problem.maxcut(n, u, v, w, node_order=L.ORDER_DEGREE).info.node_order == L.ORDER_DEGREE


@pytest.mark.parametrize("case", ["cl_heavy", "pm1_ragged", "general", "degree_ladder", "isolated"])
def test_degree_order_iterates_match_oracle(ctx, case):
    n, u, v, w, r = graph(case)
    r = min(r, 16)
    print_case(test="order_iterates", case=case)
    R0 = init_factor(n, r, 41)
    kw = dict(max_outer=1, max_inner=6, eta0=1e-14)
    _, rc, res, R, y = solve_ordered(ctx, n, u, v, w, R0, L.F64, L.ORDER_DEGREE, **kw)
    ores = alm_solve(maxcut_problem(n, u, v, w), R0, opts=OOptions(**kw))
    print(res.as_dict(), ores.inner)
    assert res.inner == ores.inner == 6
    assert np.max(np.abs(R - ores.R)) <= 1e-9 * (1.0 + np.abs(ores.R).max())
    assert np.max(np.abs(y - ores.y)) <= 1e-9 * (1.0 + np.abs(ores.y).max())


@pytest.mark.parametrize("prec", [L.F64, L.F32])
def test_degree_order_solve_remeasured_by_oracle(ctx, prec):
    n, u, v, w, r = graph("cl_heavy")
    print_case(test="order_solve", case="cl_heavy", prec=prec)
    R0 = init_factor(n, r, 43)
    _, rc, res, R, y = solve_ordered(ctx, n, u, v, w, R0, prec, L.ORDER_DEGREE)
    _, rc0, res0, _, _ = solve_ordered(ctx, n, u, v, w, R0, prec, L.ORDER_INPUT)
    print("degree", res.as_dict(), "input", res0.as_dict())
    assert rc == L.OK and rc0 == L.OK
    # the returned (R, y) are in the caller's labels: the oracle's measures of
    # them are the library's report (float32 storage: the SpMM behind the
    # library's objective accumulates in float32)
    tol = 1e-10 if prec == L.F64 else 1e-6
    m = K.alm_measures(maxcut_problem(n, u, v, w), R, y)
    assert abs(m["obj"] - res.obj) <= tol * abs(res.obj)
    assert abs(m["err3"] - res.err3) <= tol
    assert m["err1"] <= 1e-5 and abs(m["err3"]) <= 1e-5
    # both orders stop at stationary points of the same problem
    assert abs(res.obj - res0.obj) <= 1e-3 * abs(res0.obj)


def test_degree_order_rank_growth_columns(ctx):
    # the new columns are keyed by the caller's node labels: the oracle generator's values
    n, u, v, w, _ = graph("pm1_ragged")
    R0 = init_factor(n, 10, 31)
    print_case(test="order_rank_growth", case="pm1_ragged")
    kw = dict(max_outer=1, max_inner=50, rank_max=16, rank_trigger=5, rank_scale=0.03, rank_seed=777)
    _, rc, res, R, y = solve_ordered(ctx, n, u, v, w, np.hstack([R0, np.zeros((n, 6))]), L.F64, L.ORDER_DEGREE,
                                     rank=10, **kw)
    ores = alm_solve(maxcut_problem(n, u, v, w), R0, opts=OOptions(**kw))
    print(res.as_dict(), ores.rank_final)
    assert res.rank_final == ores.rank_final == 15
    assert np.max(np.abs(R[:, 10:15] - ores.R[:, 10:15])) <= 1e-14
    assert np.all(R[:, 15:] == 0.0)
    assert np.max(np.abs(R[:, :10] - ores.R[:, :10])) <= 1e-9 * (1 + np.abs(ores.R).max())


def test_degree_order_certificate_matches_input_order(ctx):
    import torch
    n, u, v, w, r = graph("er_1k")
    print_case(test="order_certify", case="er_1k")
    R0 = init_factor(n, r, 47)
    p_in, rc, res, R, y = solve_ordered(ctx, n, u, v, w, R0, L.F64, L.ORDER_INPUT)
    assert rc == L.OK
    p_deg = L.Problem.maxcut(n, u, v, w, node_order=L.ORDER_DEGREE).upload(ctx)
    yd = torch.from_numpy(y).cuda()
    c_in = L.certify(ctx, p_in, yd, max_iter=400, tol=1e-9)
    c_deg = L.certify(ctx, p_deg, yd, max_iter=400, tol=1e-9)
    print("input", c_in.as_dict(), "degree", c_deg.as_dict())
    assert c_in.status == 0 and c_deg.status == 0
    assert abs(c_in.lambda_min - c_deg.lambda_min) <= 1e-8 * (1.0 + abs(c_in.lambda_min))
    assert abs(c_in.by - c_deg.by) <= 1e-12 * abs(c_in.by)
    # the caller's y, unchanged
    assert torch.equal(yd.cpu(), torch.from_numpy(y))


def test_degree_order_warm_start_matches_input_order(ctx):
    import torch
    from paper_2407_15049_amd.warmstart import load_model, warm_start
    model = load_model(ctx.torch_device)
    if model is None:
        pytest.skip("no committed warm-start model")
    n, u, v, w, _ = graph("cl_heavy")
    print_case(test="order_warm_start", case="cl_heavy")
    p_in = L.Problem.maxcut(n, u, v, w).upload(ctx)
    p_deg = L.Problem.maxcut(n, u, v, w, node_order=L.ORDER_DEGREE).upload(ctx)
    y_in, s_in = warm_start(ctx, p_in, model)
    y_deg, s_deg = warm_start(ctx, p_deg, model)
    torch.cuda.synchronize()
    a, b = y_in.cpu().numpy(), y_deg.cpu().numpy()
    print("sigma0", s_in, s_deg, "max |dy|", np.abs(a - b).max())
    # features are float32 sums over the neighbours taken in the other order
    assert np.max(np.abs(a - b)) <= 1e-4 * (1.0 + np.abs(a).max())
    assert abs(s_in - s_deg) <= 1e-4 * s_in


def test_degree_order_kernel_entry_points_refuse(ctx):
    import torch
    n, u, v, w, r = graph("er_1k")
    print_case(test="order_refuse", case="er_1k")
    prob = L.Problem.maxcut(n, u, v, w, node_order=L.ORDER_DEGREE).upload(ctx)
    ld = L.padded_ld(r, L.F64)
    V = torch.zeros((n, ld), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(V)
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LrsdpError) as e:
        L.k_spmm(ctx, prob, L.F64, V, y, Y)
    assert e.value.code == L.EUNSUPPORTED
    with pytest.raises(L.LrsdpError) as e:
        L.k_constraint(ctx, prob, L.F64, V, V, out)
    assert e.value.code == L.EUNSUPPORTED
    with pytest.raises(L.LrsdpError) as e:
        L.k_alm_noalloc(ctx, prob, L.F64, V, y, 1.0, torch.zeros(8, dtype=torch.float64, device="cuda"))
    assert e.value.code == L.EUNSUPPORTED
