"""Seeded synthetic instance generators.

This module is shared by the CPU oracle and the GPU path.  It only draws random
graphs, weights, planted matrices and starting factors; it holds none of the
solver's arithmetic (no Laplacian, no constraint map, no objective).
"""

from .graphs import (  # noqa: F401
    erdos_renyi_edges,
    chung_lu_edges,
    pm1_weights,
    init_factor,
    completion_instance,
    maxcut_instance,
    MAXCUT_CONFIGS,
)
from .general import (cycle_edges, petersen_edges, random_box_triplets, random_general_triplets,  # noqa: F401
                      theta_triplets)
