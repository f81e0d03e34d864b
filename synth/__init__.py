"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the method: it only produces lattice
geometries (bond lists), seeded random numbers (start vectors, batch draws,
network initialisation, minibatch draws) and the named workload recipes.
Both the oracle (``oracle/``) and the device path read their inputs from here
and from nowhere else, so neither side can feed the other.
"""

from .lattice import (ring_bonds, torus_bonds, two_site_bonds, complete_bonds, site_index,
                      checkerboard_bonds, checkerboard_terms)
from .draws import (
    start_vector,
    start_vector_complex,
    batch_instances,
    mlp_init,
    minibatch_uniforms,
    MLP_SIZES,
)
from .workloads import WORKLOADS, Workload, workload

__all__ = [
    "ring_bonds", "torus_bonds", "two_site_bonds", "complete_bonds", "site_index",
    "checkerboard_bonds", "checkerboard_terms",
    "start_vector", "start_vector_complex", "batch_instances", "mlp_init", "minibatch_uniforms", "MLP_SIZES",
    "WORKLOADS", "Workload", "workload",
]
