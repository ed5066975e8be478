"""GPU solves of the golden instances against the stored oracle values
(tests/golden/oracle_solves.json, written by make_golden.py from the oracle)."""

import json
import os

import numpy as np
import pytest

from paper_2407_15049_amd import lrsdp as L
from gpu_util import dev_factor

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.Context(0)


def stored():
    with open(os.path.join(GOLDEN, "oracle_solves.json")) as f:
        return json.load(f)["solves"]


def build(rec):
    if rec["kind"] == "maxcut":
        return L.Problem.maxcut(*rec["data"])
    if rec["kind"] == "completion":
        return L.Problem.completion(*rec["data"])
    return L.Problem.general(*rec["data"])


@pytest.mark.parametrize("name", sorted(stored()))
def test_gpu_solve_matches_stored_oracle_value(ctx, name):
    import torch
    from golden.make_golden import recipes
    rec = recipes()[name]
    want = stored()[name]
    print("CASE", dict(test="golden", name=name), flush=True)
    prob = build(rec).upload(ctx)
    R0 = rec["R0"]
    r = R0.shape[1]
    opts = L.default_options(prec=L.F64, rank=r, ld=L.padded_ld(r, L.F64), tol=rec["tol"])
    Rd = dev_factor(R0, L.F64)
    yd = torch.zeros(prob.info.m, dtype=torch.float64, device="cuda")
    rc, res = L.solve(ctx, prob, Rd, yd, opts)
    torch.cuda.synchronize()
    print(res.as_dict(), "stored", want)
    assert rc == L.OK
    assert res.err1 <= rec["tol"] and abs(res.err3) <= rec["tol"]
    assert abs(res.obj - want["obj"]) <= max(10 * rec["tol"], 1e-6) * (1 + abs(want["obj"]))
