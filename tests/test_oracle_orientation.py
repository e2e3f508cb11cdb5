"""Pins of general face orientations (unstructured hexes, rest of the
boundary/orientation row): the same physical mesh with some cells renumbered
by reference-cell rotations (faces then meet other face indices in other
orientations, workloads.rotated_box) must give the same operator and the
same ADER step once the state is renumbered the same way.  The renumbering
is pure index arithmetic, independent of the oracle's face code; a wrong
orientation (a flipped tangential coordinate, a wrong neighbour face)
breaks the equality."""
import numpy as np
import pytest

import workloads as W
from oracle import Mesh, apply_operator, ader, norms


def _meshes(dim, nc, k, seed):
    mat = W.FourierMaterial(7, dim=dim)
    nodes, nb, fo, rot = W.rotated_box(dim, nc, k, 0.05, seed)
    m_rot = Mesh(dim, k, nodes, nb, mat, face_orient=fo)
    m_std = Mesh(dim, k, W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc), mat)
    perms = [W.lattice_permutation(dim, k, r) for r in rot]
    return m_std, m_rot, perms, fo


def _renumber(U, perms):
    return np.stack([U[c][:, perms[c]] for c in range(U.shape[0])])


@pytest.mark.parametrize("dim,nc,k,flux", [(2, 3, 3, "upwind"), (2, 3, 2, "central"), (3, 3, 2, "upwind"),
                                           (3, 2, 3, "central")])
def test_operator_invariant_under_cell_renumbering(dim, nc, k, flux):
    m_std, m_rot, perms, fo = _meshes(dim, nc, k, seed=3 + k)
    # the renumbering really produces non-standard faces
    std = np.array([8 * (f ^ 1) for f in range(2 * dim)])
    assert np.any(fo != std[None, :])
    U = W.random_state(21, (m_std.nc, dim + 1, m_std.np_))
    want = _renumber(apply_operator(m_std, U, flux=flux), perms)
    got = apply_operator(m_rot, _renumber(U, perms), flux=flux)
    assert norms.rel_l2(got, want) < 1e-12


def test_ader_step_invariant_under_cell_renumbering():
    dim, nc, k = 3, 2, 3
    m_std, m_rot, perms, _ = _meshes(dim, nc, k, seed=11)
    U = W.random_state(22, (m_std.nc, dim + 1, m_std.np_))
    dt = 0.01
    want = _renumber(ader.ader_step(m_std, U, dt), perms)
    got = ader.ader_step(m_rot, _renumber(U, perms), dt)
    assert norms.rel_l2(got, want) < 1e-12


def test_wrong_orientation_is_detected():
    dim, nc, k = 3, 2, 2
    m_std, m_rot, perms, fo = _meshes(dim, nc, k, seed=5)
    U = W.random_state(23, (m_std.nc, dim + 1, m_std.np_))
    want = _renumber(apply_operator(m_std, U), perms)
    bad = fo.copy()
    c, f = np.argwhere(bad % 8 != 0)[0]
    bad[c, f] ^= 1                                  # reverse one tangential coordinate of one face
    m_bad = Mesh(dim, k, m_rot.geo_nodes, m_rot.neighbors, m_rot.material, face_orient=bad)
    assert norms.rel_l2(apply_operator(m_bad, _renumber(U, perms)), want) > 1e-6


def test_face_orientation_codes():
    assert W.face_orientation((0.2, 0.7), (0.2, 0.7)) == 0
    assert W.face_orientation((0.2, 0.7), (0.8, 0.7)) == 1
    assert W.face_orientation((0.2, 0.7), (0.2, 0.3)) == 2
    assert W.face_orientation((0.2, 0.7), (0.7, 0.2)) == 4
    assert W.face_orientation((0.2, 0.7), (0.3, 0.8)) == 7
    assert W.face_orientation((0.3,), (0.7,)) == 1
    assert len(W.cube_rotations(3)) == 24 and len(W.cube_rotations(2)) == 4
