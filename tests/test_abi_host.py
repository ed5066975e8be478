"""Host-side checks of the C-ABI library (no GPU needed).

* the built library exports every function include/lrsdp.h declares;
* the host problem builder validates its input and reports the same problem
  constants as the oracle's own build;
* the default solver options carry the same schedule numbers as the oracle.
"""

import os
import re

import numpy as np
import pytest

from oracle.alm import Options as OracleOptions
from oracle.problem import completion_problem, maxcut_problem
from synth import chung_lu_edges, completion_instance, erdos_renyi_edges, pm1_weights

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

L = pytest.importorskip("paper_2407_15049_amd.lrsdp")


@pytest.fixture(scope="module")
def lib():
    return L.load()


def header_functions():
    text = open(os.path.join(ROOT, "include", "lrsdp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lrsdp_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.exported_symbols())


def test_version(lib):
    assert b"gfx950" in lib.lrsdp_version()


@pytest.mark.parametrize("u,v,msg", [
    ([0, 1], [1, 5], "outside"),
    ([0, 2], [1, 2], "self loop"),
    ([0, 1], [1, 0], "more than once"),
    ([-1], [2], "outside"),
])
def test_maxcut_rejects_malformed_edges(u, v, msg):
    with pytest.raises(L.LrsdpError) as e:
        L.Problem.maxcut(5, u, v)
    assert e.value.code == L.EINVAL and msg in str(e.value)


@pytest.mark.parametrize("u,v,msg", [
    ([0, 1], [1, 5], "outside"),
    ([0, 2], [1, 2], "self loop"),
    ([0, 1], [1, 0], "more than once"),
])
def test_degree_order_rejects_malformed_edges(u, v, msg):
    with pytest.raises(L.LrsdpError) as e:
        L.Problem.maxcut(5, u, v, node_order=L.ORDER_DEGREE)
    assert e.value.code == L.EINVAL and msg in str(e.value)


def test_degree_order_names_caller_labels_and_keeps_constants():
    # node 3 has the largest degree, so it is internal node 0; a repeated edge is
    # reported in the caller's labels
    u = [3, 3, 3, 0, 3]
    v = [0, 1, 2, 1, 4]
    p = L.Problem.maxcut(6, u, v, node_order=L.ORDER_DEGREE)
    q = L.Problem.maxcut(6, u, v)
    assert p.info.node_order == L.ORDER_DEGREE and q.info.node_order == L.ORDER_INPUT
    for f in ("n", "m", "nnz", "weights", "max_row_nnz", "c_l1", "b_l1", "b_inf"):
        assert getattr(p.info, f) == getattr(q.info, f), f
    with pytest.raises(L.LrsdpError) as e:
        L.Problem.maxcut(6, u + [4], v + [3], node_order=L.ORDER_DEGREE)
    assert e.value.code == L.EINVAL and "(3, 4)" in str(e.value)
    with pytest.raises(L.LrsdpError) as e:
        L.Problem.maxcut(6, u, v, node_order=7)
    assert e.value.code == L.EINVAL


def test_maxcut_rejects_nonfinite_weight():
    with pytest.raises(L.LrsdpError):
        L.Problem.maxcut(4, [0, 1], [1, 2], [1.0, np.nan])


def test_completion_rejects_bad_samples():
    with pytest.raises(L.LrsdpError):
        L.Problem.completion(3, 3, [0, 0], [1, 1], [1.0, 2.0])      # repeated
    with pytest.raises(L.LrsdpError):
        L.Problem.completion(3, 3, [0, 3], [1, 1], [1.0, 2.0])      # out of range
    with pytest.raises(L.LrsdpError):
        L.Problem.completion(3, 3, [0], [1], [np.inf])


@pytest.mark.parametrize("kind", ["unit", "pm1", "general", "cl"])
def test_maxcut_constants_match_oracle(kind):
    n, m = 300, 1200
    if kind == "cl":
        u, v = chung_lu_edges(n, m, 2.5, 5)
    else:
        u, v = erdos_renyi_edges(n, m, 4)
    w = None
    if kind == "pm1":
        w = pm1_weights(m, 9)
    elif kind == "general":
        w = np.random.default_rng(2).uniform(-2, 3, m)
    p = L.Problem.maxcut(n, u, v, w)
    o = maxcut_problem(n, u, v, w)
    info = p.info
    assert info.kind == L.MAXCUT and info.n == n and info.m == n
    assert info.nnz == 2 * m
    assert info.weights == {"unit": 0, "cl": 0, "pm1": 1, "general": 2}[kind]
    assert np.isclose(info.c_l1, o.c_l1, rtol=1e-12)
    assert info.b_l1 == n and info.b_inf == 1.0
    deg = np.bincount(np.concatenate([u, v]), minlength=n)
    assert info.max_row_nnz == deg.max()


def test_completion_constants_match_oracle():
    i, j, Mij, _, _ = completion_instance(40, 30, 3, 6, seed=3)
    p = L.Problem.completion(40, 30, i, j, Mij)
    o = completion_problem(40, 30, i, j, Mij)
    info = p.info
    assert info.kind == L.COMPLETION and info.n == 70 and info.m == len(i)
    assert np.isclose(info.b_l1, np.abs(o.b).sum()) and np.isclose(info.b_inf, np.abs(o.b).max())
    assert np.isclose(info.c_l1, o.c_l1)


def test_default_options_share_oracle_schedule():
    o = L.default_options()
    ref = OracleOptions()
    for name in ["tol", "lbfgs_mem", "max_outer", "max_inner", "max_iter_total", "sigma_factor",
                 "sigma_max_ratio", "feas_decrease", "eta0", "eta_factor", "eta_min"]:
        assert getattr(o, name) == getattr(ref, name), name
    assert o.sigma0 == ref.sigma0 == 0.0


def test_workspace_validation():
    u, v = erdos_renyi_edges(50, 100, 1)
    p = L.Problem.maxcut(50, u, v)
    with pytest.raises(L.LrsdpError):
        L.workspace_bytes(p, L.default_options(rank=10, ld=10, prec=L.F32))   # 40 B rows
    with pytest.raises(L.LrsdpError):
        L.workspace_bytes(p, L.default_options(rank=10, ld=10, lbfgs_mem=9))
    b4 = L.workspace_bytes(p, L.default_options(rank=10, ld=10, lbfgs_mem=4))
    b2 = L.workspace_bytes(p, L.default_options(rank=10, ld=10, lbfgs_mem=2))
    assert b4 > b2 >= (2 * 2 + 2) * 50 * 10 * 8


def test_padded_ld():
    assert L.padded_ld(20, L.F64) == 20 and L.padded_ld(26, L.F32) == 28 and L.padded_ld(10, L.F32) == 12


def test_precond_option_validation():
    u, v = erdos_renyi_edges(50, 120, 1)
    p = L.Problem.maxcut(50, u, v)
    o = L.default_options(prec=L.F64, rank=4, ld=4, precond=1, lbfgs_mem=3)
    with pytest.raises(L.LrsdpError) as e:
        L.workspace_bytes(p, o)
    assert e.value.code == L.EINVAL and "lbfgs_mem" in str(e.value)
    o.lbfgs_mem = 2
    base = L.workspace_bytes(p, L.default_options(prec=L.F64, rank=4, ld=4))
    assert L.workspace_bytes(p, o) >= base + 4 * 50 * 8      # (T + 1) rho rows and kap
    i, j, M, _, _ = completion_instance(10, 8, 2, 3, seed=1)
    c = L.Problem.completion(10, 8, i, j, M)
    with pytest.raises(L.LrsdpError) as e:
        L.workspace_bytes(c, L.default_options(prec=L.F64, rank=4, ld=4, precond=1))
    assert e.value.code == L.EUNSUPPORTED


def test_reopt_option_validation():
    u, v = erdos_renyi_edges(50, 120, 1)
    p = L.Problem.maxcut(50, u, v)
    for bad in (dict(reopt=3), dict(reopt=1, reopt_factor=1.0), dict(reopt=1, reopt_factor=0.0),
                dict(reopt=1, max_reopt=-1), dict(reopt=2, cert_iters=0)):
        with pytest.raises(L.LrsdpError) as e:
            L.workspace_bytes(p, L.default_options(prec=L.F64, rank=4, ld=4, **bad))
        assert e.value.code == L.EINVAL, bad
    base = L.workspace_bytes(p, L.default_options(prec=L.F64, rank=4, ld=4))
    assert L.workspace_bytes(p, L.default_options(prec=L.F64, rank=4, ld=4, reopt=1)) == base
    # strict level: the multipliers of the original problem and the certificate's workspace
    cert = L.certify_workspace_bytes(p, 300)
    assert L.workspace_bytes(p, L.default_options(prec=L.F64, rank=4, ld=4, reopt=2)) >= base + cert + 50 * 8


def test_general_problem_build_and_validation():
    from oracle.problem import general_problem
    from synth import random_general_triplets
    cr, cc, cv, m, ak, ar, ac, av, W = random_general_triplets(40, 25, 3, 60, 2, 9)
    b = np.arange(m, dtype=np.float64) - 3.0
    p = L.Problem.general(40, cr, cc, cv, m, ak, ar, ac, av, b)
    op = general_problem(40, cr, cc, cv, m, ak, ar, ac, av, b)
    info = p.info
    assert info.kind == L.GENERAL and info.n == 40 and info.m == m
    # symmetric pattern of Omega: the positions of C's and the constraints' triplets
    pos = {(min(a, c), max(a, c)) for a, c in zip(list(cr) + list(ar), list(cc) + list(ac))}
    assert info.nnz == sum(1 if a == c else 2 for a, c in pos)
    assert info.c_l1 == pytest.approx(op.c_l1, rel=1e-14)
    assert info.b_l1 == pytest.approx(np.abs(b).sum()) and info.b_inf == pytest.approx(np.abs(b).max())
    bad = [
        dict(c_row=[40]), dict(a_row=[-1]), dict(a_con=[m]), dict(c_val=[np.nan]), dict(b=np.full(m, np.inf)),
    ]
    for kw in bad:
        args = dict(c_row=cr, c_col=cc, c_val=cv, a_con=ak, a_row=ar, a_col=ac, a_val=av, b=b)
        for k, v in kw.items():
            if k == "b":
                args[k] = v
            else:
                a = np.array(args[k], copy=True)
                a[0] = v[0]
                args[k] = a
        with pytest.raises(L.LrsdpError) as e:
            L.Problem.general(40, args["c_row"], args["c_col"], args["c_val"], m, args["a_con"], args["a_row"],
                              args["a_col"], args["a_val"], args["b"])
        assert e.value.code == L.EINVAL, kw
    with pytest.raises(L.LrsdpError) as e:
        L.workspace_bytes(p, L.default_options(prec=L.F64, rank=4, ld=4, precond=1))
    assert e.value.code == L.EUNSUPPORTED
    assert L.workspace_bytes(p, L.default_options(prec=L.F64, rank=4, ld=4, reopt=2)) > 0
    # the splitting phase adds its CG scratch: six n x ld arrays and three m-vectors (256-byte rounded) and R's copy
    base = L.workspace_bytes(p, L.default_options(prec=L.F64, rank=4, ld=4))
    ph2 = L.workspace_bytes(p, L.default_options(prec=L.F64, rank=4, ld=4, phase2=1))
    arr, vec = (40 * 4 * 8 + 255) // 256 * 256, (m * 8 + 255) // 256 * 256
    assert ph2 - base >= 6 * arr + 3 * vec + 40 * 4 * 8
    assert L.admm_workspace_bytes(p, L.F64, 4) == 6 * arr + 3 * vec


def test_general_blocks_build_and_validation():
    from oracle.problem import general_blocks_problem
    from test_oracle_general import two_theta_blocks
    args = two_theta_blocks()
    p = L.Problem.general_blocks(*args)
    op = general_blocks_problem(*args)
    assert p.info.n == 15 and p.info.m == op.m
    assert p.info.c_l1 == pytest.approx(op.c_l1, rel=1e-14)
    block_n, c_blk, c_row, c_col, c_val, m, a_con, a_blk, a_row, a_col, a_val, b = args
    bad_blk = np.array(c_blk, copy=True)
    bad_blk[0] = 2
    with pytest.raises(L.LrsdpError) as e:
        L.Problem.general_blocks(block_n, bad_blk, c_row, c_col, c_val, m, a_con, a_blk, a_row, a_col, a_val, b)
    assert e.value.code == L.EINVAL
    bad_row = np.array(a_row, copy=True)
    bad_row[0] = 5                                  # block 0 has order 5
    with pytest.raises(L.LrsdpError) as e:
        L.Problem.general_blocks(block_n, c_blk, c_row, c_col, c_val, m, a_con, a_blk, bad_row, a_col, a_val, b)
    assert e.value.code == L.EINVAL


def test_block_ranks_validation():
    from test_oracle_general import two_theta_blocks
    p = L.Problem.general_blocks(*two_theta_blocks())
    p.set_block_ranks([2, 3])
    with pytest.raises(ValueError):
        p.set_block_ranks([2])
    with pytest.raises(L.LrsdpError) as e:
        p.set_block_ranks([0, 3])
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LrsdpError) as e:
        L.Problem.maxcut(4, [0, 1], [1, 2]).set_block_ranks([1])
    assert e.value.code == L.EUNSUPPORTED


def test_general_dense_storage_choice_and_validation():
    from synth import random_general_triplets, theta_triplets
    from synth import petersen_edges
    u, v = petersen_edges()
    t = theta_triplets(10, u, v)                       # C = -J: every position nonzero
    auto = L.Problem.general(10, *t)
    sparse = L.Problem.general(10, *t, c_storage=L.C_SPARSE)
    dense = L.Problem.general(10, *t, c_storage=L.C_DENSE)
    assert auto.info.c_dense == 1 and dense.info.c_dense == 1 and sparse.info.c_dense == 0
    # dense storage: Omega keeps the constraint positions only (trace: 10 diagonal, edges: 15),
    # and the device image holds the n x n matrix
    assert dense.info.nnz == 10 + 2 * 15 and sparse.info.nnz == 10 * 10
    assert dense.device_bytes() >= sparse.device_bytes() - 8 * 100 + 8 * 10 * 10
    assert dense.info.c_l1 == sparse.info.c_l1
    cr, cc, cv, m, ak, ar, ac, av, W = random_general_triplets(40, 25, 3, 60, 2, 9)
    b = np.zeros(m)
    assert L.Problem.general(40, cr, cc, cv, m, ak, ar, ac, av, b).info.c_dense == 0   # 60 of 820
    with pytest.raises(L.LrsdpError) as e:
        L.Problem.general(40, cr, cc, cv, m, ak, ar, ac, av, b, c_storage=7)
    assert e.value.code == L.EINVAL
    big = 16385
    with pytest.raises(L.LrsdpError) as e:
        L.Problem.general(big, [0], [1], [1.0], 1, [0], [0], [0], [1.0], [1.0], c_storage=L.C_DENSE)
    assert e.value.code == L.EINVAL and "dense" in str(e.value)
