"""Pins of the oracle's dynamic rank (appendix A.1): the SplitMix64 generator
against its published first outputs, the Box-Muller columns' moments, and a
rank-10 start on the 1k-node graph (a non-global stationary point at rank 10,
certified) that reaches the certified optimum once the rank grows."""

import numpy as np

from oracle import certify
from oracle.alm import Options, alm_solve, new_columns, splitmix64_at
from oracle.problem import maxcut_problem
from synth import erdos_renyi_edges, init_factor


def test_splitmix64_published_outputs():
    # the SplitMix64 sequence seeded with 0 starts 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4
    out = splitmix64_at(0, np.arange(2))
    assert int(out[0]) == 0xE220A8397B1DCDAF
    assert int(out[1]) == 0x6E789E6AA1B965F4


def test_new_columns_are_standard_normal_and_positional():
    Z = new_columns(50000, 3, 7, 15049)
    assert Z.shape == (50000, 4)
    assert abs(Z.mean()) < 0.01 and abs(Z.var() - 1.0) < 0.02
    # entry (i, c) depends only on (i, c, seed): a different column range overlaps
    W = new_columns(50000, 5, 9, 15049)
    assert np.array_equal(Z[:, 2:], W[:, :2])
    assert not np.array_equal(new_columns(10, 3, 4, 1), new_columns(10, 3, 4, 2))


def test_rank_growth_escapes_the_rank10_stationary_point():
    u, v = erdos_renyi_edges(1000, 5000, 15049)
    prob = maxcut_problem(1000, u, v)
    R0 = init_factor(1000, 10, 15050)
    fixed = alm_solve(prob, R0, opts=Options())
    grown = alm_solve(prob, R0, opts=Options(rank_max=16, rank_trigger=100))
    assert fixed.converged and grown.converged
    assert grown.rank_final == 15 or grown.rank_final == 16
    lam_fixed = certify.lambda_min(prob, fixed.y)
    lam_grown = certify.lambda_min(prob, grown.y)
    assert lam_fixed < -1e-3                    # rank 10 stops at a non-global point
    assert lam_grown > lam_fixed / 5            # the grown solve is much closer to dual feasible
    assert grown.obj < fixed.obj - 0.1          # and has the lower (better) objective
