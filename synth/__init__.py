"""Seeded synthetic inputs for the ISDF path (orbitals, K-means seeds, loss field).

This module only *generates* inputs.  It holds none of the ISDF arithmetic
(no weight function, no clustering, no Gram blocks, no fit): both the CPU
oracle and the GPU library consume what it produces.
"""
from .orbitals import (  # noqa: F401
    WORKLOADS,
    Workload,
    make_workload,
    make_orbitals_large,
    make_orbitals,
    init_centroids,
    loss_field,
    random_orthonormal,
)
