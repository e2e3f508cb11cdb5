"""Seeded synthetic inputs shared by the product path, the tests and the oracle.

This package holds input recipes only: mesh node positions of the periodic
box, the neighbour table, material fields, initial conditions, random states
and source positions.  It contains none of the discontinuous Galerkin
arithmetic (no quadrature, no basis, no operator); both the HIP library and
the oracle compute everything else from these inputs on their own.
"""
from .generators import (  # noqa: F401
    box_nodes,
    box_neighbors,
    FourierMaterial,
    ConstantMaterial,
    standing_wave_2d,
    plane_wave_3d,
    gaussian_pulse,
    random_state,
    random_points,
    c2_workload,
)
