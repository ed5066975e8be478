"""Oracle general problems (one block, sparse C and A_k from triplets) against
independent references.

* The MaxCut and completion SDPs written as general triplets give the same
  constraint map, adjoint and objective as their dedicated constructors.
* Triplet convention: an off-diagonal entry may be given in either triangle,
  and repeated entries add up.
* Closed forms of the Lovasz theta number (Lovasz 1979): the theta SDP's
  optimum is -theta, with theta(C_n) = n cos(pi/n) / (1 + cos(pi/n)) for odd n
  (sqrt 5 for the pentagon), theta(Petersen) = 4, theta(K_n) = 1 and
  theta of the edgeless graph = n.
* A random feasible instance solves to a point whose dual slack
  C - A*(y) is psd up to the tolerance (a certified optimum).
"""

import math

import numpy as np
import pytest

from oracle import certify
from oracle.alm import Options, alm_solve
from oracle.problem import completion_problem, general_problem, maxcut_problem
from synth import (completion_instance, cycle_edges, erdos_renyi_edges, init_factor, petersen_edges,
                   random_general_triplets, theta_triplets)


def maxcut_triplets(n, u, v, w):
    deg = np.zeros(n)
    np.add.at(deg, u, w)
    np.add.at(deg, v, w)
    c_row = np.concatenate([u, np.arange(n)])
    c_col = np.concatenate([v, np.arange(n)])
    c_val = np.concatenate([0.25 * w, -0.25 * deg])     # C = -L/4
    k = np.arange(n)
    return c_row, c_col, c_val, n, k, k, k, np.ones(n), np.ones(n)


def same_problem(p, q, rng):
    U = rng.standard_normal((p.n, 4))
    V = rng.standard_normal((p.n, 4))
    y = rng.standard_normal(p.m)
    assert np.allclose(p.A_of(U, V), q.A_of(U, V), rtol=1e-13, atol=1e-12)
    assert np.allclose((p.A_adj(y) @ V), (q.A_adj(y) @ V), rtol=1e-13, atol=1e-12)
    assert p.objective(U, V) == pytest.approx(q.objective(U, V), rel=1e-13)
    assert p.c_l1 == pytest.approx(q.c_l1, rel=1e-14)
    assert np.array_equal(p.b, q.b)


def test_maxcut_as_general():
    u, v = erdos_renyi_edges(70, 300, 3)
    w = np.random.default_rng(4).uniform(-1, 2, 300)
    same_problem(general_problem(70, *maxcut_triplets(70, u, v, w)), maxcut_problem(70, u, v, w),
                 np.random.default_rng(5))


def test_completion_as_general():
    n1, n2 = 20, 15
    i, j, M, _, _ = completion_instance(n1, n2, 2, 5, seed=6)
    n = n1 + n2
    m = len(i)
    c_row = c_col = np.arange(n)
    g = general_problem(n, c_row, c_col, np.ones(n), m, np.arange(m), i, n1 + j, np.ones(m), 2 * M)
    same_problem(g, completion_problem(n1, n2, i, j, M), np.random.default_rng(7))


def test_triplet_convention():
    rng = np.random.default_rng(8)
    n, m = 12, 3
    a_con = np.array([0, 1, 1, 2])
    a_row = np.array([3, 0, 5, 7])
    a_col = np.array([9, 0, 2, 7])
    a_val = np.array([1.5, 2.0, -1.0, 0.5])
    b = np.array([1.0, 2.0, 3.0])
    p = general_problem(n, [1, 4], [4, 4], [2.0, -1.0], m, a_con, a_row, a_col, a_val, b)
    # the other triangle, and an entry split into two triplets that add up
    q = general_problem(n, [4, 4, 4], [1, 1, 4], [0.5, 1.5, -1.0], m, a_con, a_col, a_row, a_val, b)
    same_problem(p, q, rng)
    # <A_0, X> = 1.5 (X_39 + X_93) for X = U V^T
    U, V = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    X = U @ V.T
    assert p.A_of(U, V)[0] == pytest.approx(1.5 * (X[3, 9] + X[9, 3]), rel=1e-14)
    assert p.A_of(U, V)[1] == pytest.approx(2.0 * X[0, 0] - (X[5, 2] + X[2, 5]), rel=1e-13)


def theta(n, u, v, rank, tol=1e-8):
    op = general_problem(n, *theta_triplets(n, u, v))
    res = alm_solve(op, init_factor(n, rank, 3), opts=Options(tol=tol))
    assert res.converged
    return -res.obj


@pytest.mark.parametrize("n", [5, 7, 9])
def test_theta_odd_cycle(n):
    u, v = cycle_edges(n)
    c = math.cos(math.pi / n)
    assert theta(n, u, v, 6) == pytest.approx(n * c / (1 + c), rel=1e-6)


def test_theta_petersen_complete_and_empty():
    u, v = petersen_edges()
    assert theta(10, u, v, 6) == pytest.approx(4.0, rel=1e-6)
    iu = np.triu_indices(6, 1)
    assert theta(6, iu[0], iu[1], 6) == pytest.approx(1.0, rel=1e-6)
    assert theta(8, np.zeros(0, np.int32), np.zeros(0, np.int32), 3) == pytest.approx(8.0, rel=1e-6)


def test_random_general_reaches_a_certified_optimum():
    cr, cc, cv, m, ak, ar, ac, av, W = random_general_triplets(60, 40, 4, 120, 3, 5)
    op = general_problem(60, cr, cc, cv, m, ak, ar, ac, av, np.zeros(m))
    op = general_problem(60, cr, cc, cv, m, ak, ar, ac, av, op.A_of(W))
    res = alm_solve(op, init_factor(60, 10, 4), opts=Options())
    assert res.converged and res.err1 <= 1e-5 and abs(res.err3) <= 1e-5
    assert certify.lambda_min(op, res.y) >= -1e-5 * (1 + op.c_l1)


def two_theta_blocks():
    """Blocks: theta SDP of C5 (order 5) and of the Petersen graph (order 10),
    each with its own trace constraint; optimum -(sqrt 5 + 4)."""
    t1 = theta_triplets(5, *cycle_edges(5))
    t2 = theta_triplets(10, *petersen_edges())
    c_blk = np.concatenate([np.zeros(len(t1[0]), np.int32), np.ones(len(t2[0]), np.int32)])
    c_row = np.concatenate([t1[0], t2[0]])
    c_col = np.concatenate([t1[1], t2[1]])
    c_val = np.concatenate([t1[2], t2[2]])
    m1 = t1[3]
    a_con = np.concatenate([t1[4], m1 + t2[4]])
    a_blk = np.concatenate([np.zeros(len(t1[4]), np.int32), np.ones(len(t2[4]), np.int32)])
    a_row = np.concatenate([t1[5], t2[5]])
    a_col = np.concatenate([t1[6], t2[6]])
    a_val = np.concatenate([t1[7], t2[7]])
    b = np.concatenate([t1[8], t2[8]])
    return [5, 10], c_blk, c_row, c_col, c_val, m1 + t2[3], a_con, a_blk, a_row, a_col, a_val, b


def theta_with_slack_block():
    """Blocks: X (order 5, theta of C5) and a scalar s >= 0 (order 1):
    tr X + s = 1 and the edge constraints; optimum -sqrt 5 with s = 0."""
    c_row, c_col, c_val, m, a_con, a_row, a_col, a_val, b = theta_triplets(5, *cycle_edges(5))
    a_con = np.concatenate([a_con, [0]])
    a_blk = np.concatenate([np.zeros(len(a_row), np.int32), [1]])
    a_row = np.concatenate([a_row, [0]])
    a_col = np.concatenate([a_col, [0]])
    a_val = np.concatenate([a_val, [1.0]])
    return [5, 1], np.zeros(len(c_row), np.int32), c_row, c_col, c_val, m, a_con, a_blk, a_row, a_col, a_val, b


def test_blocks_equal_offset_indices():
    from oracle.problem import general_blocks_problem
    args = two_theta_blocks()
    p = general_blocks_problem(*args)
    block_n, c_blk, c_row, c_col, c_val, m, a_con, a_blk, a_row, a_col, a_val, b = args
    off = np.array([0, 5])
    q = general_problem(15, off[c_blk] + c_row, off[c_blk] + c_col, c_val, m, a_con, off[a_blk] + a_row,
                        off[a_blk] + a_col, a_val, b)
    same_problem(p, q, np.random.default_rng(11))


def test_two_theta_blocks_closed_form():
    from oracle.problem import general_blocks_problem
    op = general_blocks_problem(*two_theta_blocks())
    res = alm_solve(op, init_factor(15, 6, 3), opts=Options(tol=1e-8))
    assert res.converged
    assert -res.obj == pytest.approx(math.sqrt(5) + 4.0, rel=1e-6)


def test_scalar_slack_block():
    from oracle.problem import general_blocks_problem
    op = general_blocks_problem(*theta_with_slack_block())
    res = alm_solve(op, init_factor(6, 4, 3), opts=Options(tol=1e-8))
    assert res.converged
    assert -res.obj == pytest.approx(math.sqrt(5), rel=1e-6)
    assert np.sum(res.R[5] ** 2) <= 1e-6          # the slack ends at 0


def trace_blocks(sizes, seed):
    """Blocks X_j (orders `sizes`) with random symmetric C_j and tr X_j = 1 each:
    min <C_j, X_j> over psd X_j of trace 1 is lambda_min(C_j), reached by a
    rank-one X_j (v v^T for a unit eigenvector v)."""
    rng = np.random.default_rng(seed)
    c_blk, c_row, c_col, c_val, mats = [], [], [], [], []
    a_con, a_blk, a_row, a_col, a_val = [], [], [], [], []
    for j, nj in enumerate(sizes):
        M = rng.standard_normal((nj, nj))
        M = 0.5 * (M + M.T)
        mats.append(M)
        r, c = np.triu_indices(nj)
        c_blk.append(np.full(len(r), j))
        c_row.append(r)
        c_col.append(c)
        c_val.append(M[r, c])
        a_con.append(np.full(nj, j))
        a_blk.append(np.full(nj, j))
        a_row.append(np.arange(nj))
        a_col.append(np.arange(nj))
        a_val.append(np.ones(nj))
    cat = lambda xs, t=np.int32: np.concatenate(xs).astype(t)
    args = (list(sizes), cat(c_blk), cat(c_row), cat(c_col), cat(c_val, np.float64), len(sizes), cat(a_con),
            cat(a_blk), cat(a_row), cat(a_col), cat(a_val, np.float64), np.ones(len(sizes)))
    return args, mats


def test_block_rank_masks_the_gradient():
    from oracle import kernels as K
    from oracle.problem import general_blocks_problem
    args, _ = trace_blocks([4, 6], 5)
    full = general_blocks_problem(*args)
    part = general_blocks_problem(*args, block_rank=[1, 3])
    rng = np.random.default_rng(6)
    R = rng.standard_normal((10, 3))
    y = rng.standard_normal(2)
    G, Gm = K.gradient(full, R, y, 3.0), K.gradient(part, R, y, 3.0)
    assert np.all(Gm[:4, 1:] == 0.0)                       # block 0 keeps column 0 only
    assert np.array_equal(Gm[:4, :1], G[:4, :1]) and np.array_equal(Gm[4:], G[4:])


def test_block_rank_one_reaches_lambda_min():
    # a rank-one block reaches min <C_j, X_j> = lambda_min(C_j) over trace-one psd X_j
    from oracle.problem import general_blocks_problem
    args, mats = trace_blocks([4, 6], 7)
    op = general_blocks_problem(*args, block_rank=[1, 3])
    res = alm_solve(op, init_factor(10, 3, 8), opts=Options(tol=1e-9))
    want = sum(np.linalg.eigvalsh(M)[0] for M in mats)
    assert res.converged
    assert res.obj == pytest.approx(want, rel=1e-6, abs=1e-7)
    assert np.all(res.R[:4, 1:] == 0.0)


def test_block_rank_one_cannot_hold_two_orthogonal_unit_rows():
    # X_00 = X_11 = 1 and X_01 = 0 need rank 2: a rank-one factor (a, b) has
    # X_01 = ab with a^2 = b^2 = 1, so the constraints cannot all hold
    from oracle.problem import general_blocks_problem
    args = ([2], np.array([0, 0], np.int32), np.array([0, 1], np.int32), np.array([0, 1], np.int32),
            np.array([1.0, 0.5]), 3, np.array([0, 1, 2], np.int32), np.zeros(3, np.int32),
            np.array([0, 1, 0], np.int32), np.array([0, 1, 1], np.int32), np.ones(3), np.array([1.0, 1.0, 0.0]))
    R0 = init_factor(2, 2, 9)
    one = alm_solve(general_blocks_problem(*args, block_rank=[1]), R0, opts=Options(max_outer=30))
    two = alm_solve(general_blocks_problem(*args, block_rank=[2]), R0, opts=Options(max_outer=30))
    assert not one.converged and one.err1 > 0.05
    assert two.converged and two.obj == pytest.approx(1.5, rel=1e-5)   # <C, X> = X_00 + 0.5 X_11
