"""End-to-end pins of the oracle's Burer-Monteiro ALM solve.

Closed forms (complete graph, odd cycle, bipartite graph), the two-sided
brute-force bound (max cut <= SDP <= max cut / 0.87856 for w >= 0), the dual
certificate (minimum eigenvalue of C - A*(y)), invariances, and for completion
the nuclear norm of a fully observed matrix and exact recovery of a planted one.
"""

import numpy as np
import pytest

from oracle import certify
from oracle.alm import Options, alm_solve
from oracle.problem import completion_problem, maxcut_problem
from synth import completion_instance, erdos_renyi_edges, init_factor

GW = 0.87856


def solve_maxcut(n, u, v, w=None, r=4, seed=0, tol=1e-8):
    prob = maxcut_problem(n, u, v, w)
    res = alm_solve(prob, init_factor(n, r, seed), opts=Options(tol=tol))
    return prob, res


def test_complete_graph_closed_form():
    # K_n: SDP optimum (min form) = -n^2/4, y* = -(n/4) 1
    n = 9
    u, v = np.triu_indices(n, 1)
    prob, res = solve_maxcut(n, u, v, r=3)
    assert res.converged
    assert np.isclose(res.obj, -n * n / 4.0, rtol=1e-6)
    assert np.allclose(res.y, -n / 4.0, rtol=1e-4)


@pytest.mark.parametrize("n", [5, 7, 9, 11])
def test_odd_cycle_closed_form(n):
    # C_n (n odd): optimum -(n/2)(1 + cos(pi/n)), y*_i = -(1 + cos(pi/n))/2
    u = np.arange(n)
    v = (u + 1) % n
    prob, res = solve_maxcut(n, u, v, r=3)
    assert res.converged
    expect = -(n / 2.0) * (1.0 + np.cos(np.pi / n))
    assert np.isclose(res.obj, expect, rtol=1e-6)
    assert np.allclose(res.y, -(1.0 + np.cos(np.pi / n)) / 2.0, rtol=1e-4)


def test_bipartite_closed_form():
    # bipartite graph, w >= 0: every edge is cut, optimum -sum(w)
    rng = np.random.default_rng(1)
    a, b = 6, 7
    pairs = [(i, a + j) for i in range(a) for j in range(b) if rng.random() < 0.5]
    u = np.array([p[0] for p in pairs]); v = np.array([p[1] for p in pairs])
    w = rng.uniform(0.5, 2.0, len(u))
    prob, res = solve_maxcut(a + b, u, v, w, r=3)
    assert res.converged
    assert np.isclose(res.obj, -w.sum(), rtol=1e-6)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_two_sided_bound(seed):
    n, m = 14, 30
    u, v = erdos_renyi_edges(n, m, 100 + seed)
    w = np.random.default_rng(seed).uniform(0.2, 1.0, m)
    prob, res = solve_maxcut(n, u, v, w, r=6)
    assert res.converged
    sdp = -res.obj
    mc = certify.brute_force_maxcut(n, u, v, w)
    assert mc <= sdp * (1 + 1e-6)
    assert mc >= GW * sdp
    # certified lower bound from the dual: primal and certificate agree
    bound = -certify.maxcut_dual_bound(prob, res.y)
    assert sdp <= bound + 1e-6 * abs(bound)
    assert (bound - sdp) / (1 + abs(sdp)) < 1e-5
    assert certify.err2(prob, res.y) < 1e-6


def test_relabel_and_scale_invariance():
    n, m = 40, 120
    u, v = erdos_renyi_edges(n, m, 7)
    _, base = solve_maxcut(n, u, v, r=8)
    perm = np.random.default_rng(3).permutation(n)
    _, rel = solve_maxcut(n, perm[u], perm[v], r=8, seed=5)
    _, scl = solve_maxcut(n, u, v, 3.0 * np.ones(m), r=8, seed=6)
    assert np.isclose(rel.obj, base.obj, rtol=1e-6)
    assert np.isclose(scl.obj, 3.0 * base.obj, rtol=1e-6)


def test_disjoint_union_additive():
    u1, v1 = erdos_renyi_edges(12, 25, 8)
    u2, v2 = erdos_renyi_edges(9, 15, 9)
    _, r1 = solve_maxcut(12, u1, v1, r=6)
    _, r2 = solve_maxcut(9, u2, v2, r=6)
    _, ru = solve_maxcut(21, np.concatenate([u1, u2 + 12]), np.concatenate([v1, v2 + 12]), r=6)
    assert np.isclose(ru.obj, r1.obj + r2.obj, rtol=1e-6)


def test_er_1k_rank_gap_is_certified():
    # On the 1k-node Erdos-Renyi workload, rank 10 stalls at a non-global
    # stationary point that the certificate exposes; rank 16 closes the gap.
    from synth import maxcut_instance
    inst = maxcut_instance("er_1k")
    prob = maxcut_problem(inst["n"], inst["u"], inst["v"], inst["w"])
    r10 = alm_solve(prob, init_factor(inst["n"], 10, 1), opts=Options(tol=1e-7))
    r16 = alm_solve(prob, init_factor(inst["n"], 16, 1), opts=Options(tol=1e-7))
    b10 = certify.maxcut_dual_bound(prob, r10.y)
    b16 = certify.maxcut_dual_bound(prob, r16.y)
    assert r10.converged and r16.converged
    assert r16.obj < r10.obj                       # rank 16 reaches a lower objective
    assert (r16.obj - b16) / (1 + abs(b16)) < 1e-6  # and is certified optimal
    assert (r10.obj - b10) / (1 + abs(b10)) > 1e-4  # rank 10 is not
    assert b10 <= r16.obj + 1e-6 * abs(r16.obj)     # every dual bound is a lower bound


def test_completion_fully_observed_nuclear_norm():
    # every entry observed: the optimum is 2 ||M||_*
    n1, n2, k = 8, 6, 2
    i, j, Mij, U, V = completion_instance(n1, n2, k, n2, seed=11)
    prob = completion_problem(n1, n2, i, j, Mij)
    R0 = init_factor(n1 + n2, 5, 3)
    res = alm_solve(prob, R0, opts=Options(tol=1e-8))
    M = U @ V.T
    nuc = np.linalg.svd(M, compute_uv=False).sum()
    assert res.converged
    assert np.isclose(res.obj, 2.0 * nuc, rtol=1e-5)
    bound = certify.completion_dual_bound(prob, n1, n2, i, j, res.y)
    assert bound <= res.obj + 1e-6 * res.obj
    assert (res.obj - bound) / (1 + res.obj) < 1e-5


def test_completion_planted_exact_recovery():
    n1 = n2 = 30
    i, j, Mij, U, V = completion_instance(n1, n2, 2, 20, seed=12)
    prob = completion_problem(n1, n2, i, j, Mij)
    res = alm_solve(prob, init_factor(n1 + n2, 6, 4), opts=Options(tol=1e-8))
    X12 = res.R[:n1] @ res.R[n1:].T
    M = U @ V.T
    assert res.converged
    assert np.linalg.norm(X12 - M) / np.linalg.norm(M) < 1e-4
    assert np.isclose(res.obj, 2.0 * np.linalg.svd(M, compute_uv=False).sum(), rtol=1e-5)
