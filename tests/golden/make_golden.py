"""Writes the stored expected values under tests/golden/ by calling only the
oracle (and the seeded input generators).  Run from the repository root:

    python tests/golden/make_golden.py

oracle_solves.json: the oracle's FP64 solves of small seeded instances to
err1, |err3| <= tol (objective, ALM steps, L-BFGS iterations), so that GPU
tests compare against fixed numbers and a change of the oracle's arithmetic
shows up as a diff of this file.

closed_forms.json: textbook optimal values the solves must reach, with their
sources: the MaxCut SDP of the odd cycle C_n, (n/2)(1 + cos(pi/n)) (Delorme and
Poljak 1993; Goemans and Williamson 1995), of K_n, n^2/4, and the Lovasz theta
numbers theta(C_n) = n cos(pi/n) / (1 + cos(pi/n)) for odd n and
theta(Petersen) = 4 (Lovasz 1979).
"""

import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.alm import Options, alm_solve  # noqa: E402
from oracle.problem import completion_problem, general_problem, maxcut_problem  # noqa: E402
from synth import (completion_instance, cycle_edges, erdos_renyi_edges, init_factor, petersen_edges,  # noqa: E402
                   theta_triplets)


def recipes():
    """name -> dict(kind, data, R0, tol): the seeded instances (raw data, so that
    the GPU tests build the same problems through the library)."""
    out = {}
    u, v = erdos_renyi_edges(1000, 5000, 15049)
    out["maxcut_er_1k_rank10"] = dict(kind="maxcut", data=(1000, u, v, None), R0=init_factor(1000, 10, 15050),
                                      tol=1e-5)
    u, v = cycle_edges(9)
    out["maxcut_c9_rank2"] = dict(kind="maxcut", data=(9, u, v, None), R0=init_factor(9, 2, 5), tol=1e-8)
    i, j, M, _, _ = completion_instance(40, 31, 2, 10, seed=21)
    out["completion_40x31_rank2"] = dict(kind="completion", data=(40, 31, i, j, M), R0=init_factor(71, 2, 7),
                                         tol=1e-7)
    out["theta_c5_rank6"] = dict(kind="general", data=(5,) + tuple(theta_triplets(5, *cycle_edges(5))),
                                 R0=init_factor(5, 6, 3), tol=1e-8)
    out["theta_petersen_rank6"] = dict(kind="general", data=(10,) + tuple(theta_triplets(10, *petersen_edges())),
                                       R0=init_factor(10, 6, 3), tol=1e-8)
    return out


def oracle_problem(rec):
    build = {"maxcut": maxcut_problem, "completion": completion_problem, "general": general_problem}[rec["kind"]]
    return build(*rec["data"])


def instances():
    """name -> (oracle problem, starting factor, tol)."""
    return {k: (oracle_problem(r), r["R0"], r["tol"]) for k, r in recipes().items()}


def main():
    solves = {}
    for name, (op, R0, tol) in instances().items():
        res = alm_solve(op, R0, opts=Options(tol=tol))
        solves[name] = dict(obj=res.obj, dual=res.dual, err1=res.err1, err3=res.err3, outer=res.outer,
                            inner=res.inner, converged=bool(res.converged), tol=tol)
        print(name, solves[name])
    with open(os.path.join(HERE, "oracle_solves.json"), "w") as f:
        json.dump({"generator": "python tests/golden/make_golden.py", "solves": solves}, f, indent=1)
    closed = {
        "maxcut_c9_min_form": dict(value=-(9 / 2) * (1 + math.cos(math.pi / 9)),
                                   source="MaxCut SDP of the odd cycle C_n: (n/2)(1 + cos(pi/n)) "
                                          "(Delorme and Poljak 1993; Goemans and Williamson 1995)"),
        "maxcut_k7_min_form": dict(value=-49 / 4, source="MaxCut SDP of K_n: n^2/4"),
        "theta_c5_min_form": dict(value=-math.sqrt(5), source="Lovasz theta of the pentagon, sqrt 5 (Lovasz 1979)"),
        "theta_c7_min_form": dict(value=-7 * math.cos(math.pi / 7) / (1 + math.cos(math.pi / 7)),
                                  source="Lovasz theta of the odd cycle C_n: n cos(pi/n) / (1 + cos(pi/n)) "
                                         "(Lovasz 1979)"),
        "theta_petersen_min_form": dict(value=-4.0, source="Lovasz theta of the Petersen graph, 4 (Lovasz 1979)"),
    }
    with open(os.path.join(HERE, "closed_forms.json"), "w") as f:
        json.dump({"generator": "python tests/golden/make_golden.py", "values": closed}, f, indent=1)


if __name__ == "__main__":
    main()
