"""Seeded synthetic inputs shared by the product path, the tests and the oracle.

This package holds input recipes only: mesh node positions of the unit box,
the neighbour table (periodic, or with wall / absorbing boundary codes),
material fields, initial conditions and closed-form solutions, random states
and source positions.  It contains none of the discontinuous Galerkin
arithmetic (no quadrature, no basis, no operator); both the HIP library and
the oracle compute everything else from these inputs on their own.
"""
from .generators import (  # noqa: F401
    box_nodes,
    box_neighbors,
    cube_rotations,
    lattice_permutation,
    face_orientation,
    rotated_box,
    BC_WALL,
    BC_ABSORBING,
    BC_PRESCRIBED,
    PlaneWaves,
    c3_literal_plane_wave,
    FourierMaterial,
    GradedMedium,
    ConstantMaterial,
    standing_wave_2d,
    plane_wave_3d,
    gaussian_pulse,
    membrane_mode,
    travelling_pulse_x,
    random_state,
    random_points,
    c2_workload,
)
