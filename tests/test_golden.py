"""Stored expected values (tests/golden/, written by make_golden.py from the
oracle only) against the oracle as it stands and against the closed forms."""

import json
import os

import pytest

from oracle.alm import Options, alm_solve

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_oracle_reproduces_the_stored_solves():
    from golden.make_golden import instances
    stored = load("oracle_solves.json")["solves"]
    for name, (op, R0, tol) in instances().items():
        res = alm_solve(op, R0, opts=Options(tol=tol))
        want = stored[name]
        assert res.converged and want["converged"], name
        assert res.outer == want["outer"] and res.inner == want["inner"], name
        assert res.obj == pytest.approx(want["obj"], rel=1e-12), name


def test_stored_solves_reach_the_closed_forms():
    s = load("oracle_solves.json")["solves"]
    c = load("closed_forms.json")["values"]
    assert s["maxcut_c9_rank2"]["obj"] == pytest.approx(c["maxcut_c9_min_form"]["value"], rel=1e-7)
    assert s["theta_c5_rank6"]["obj"] == pytest.approx(c["theta_c5_min_form"]["value"], rel=1e-7)
    assert s["theta_petersen_rank6"]["obj"] == pytest.approx(c["theta_petersen_min_form"]["value"], rel=1e-7)
    for v in c.values():
        assert v["source"]
