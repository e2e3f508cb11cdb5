"""Pins of the oracle with a density and a sound speed that vary inside the
cells (Sec. 2, eq. general-hyp-pde: rho and c are functions of x).

Sec. 2.1 keeps the coefficients inside S with an unweighted mass; for rho
varying inside a cell that literal form evaluates grad(p/rho) and
div(rho c^2 v) instead of grad(p)/rho and rho c^2 div(v).  The oracle takes
the weighted-mass reading (rho- and (rho c^2)^-1-weighted mass matrices).
These pins tell the two apart and check every place the density enters:

* a closed-form wave in a medium graded along the direction of propagation
  (both rho and c vary inside every cell, the impedance rho c is constant):
  the literal placement converges to another solution, the weighted one at
  order k+1, for LSRK(5,4) and ADER;
* the discrete energy identity on affine cells with rho(x), c(x) from the
  seeded Fourier fields, with the energy form obtained from the physical
  norm by polarization (so the oracle's mass matrices are not reused);
* a single periodic cell assembled column by column: with the mass matrix
  from the same polarization, M L is skew (central flux, affine cell) and
  has a negative semidefinite symmetric part (upwind);
* a constant state is steady with rho(x).
"""
import numpy as np
import pytest

import workloads as W
from oracle import Mesh, ader, apply_operator, basis, norms
from oracle import timestep as ts


def make(dim, nc, k, amp, mat):
    return Mesh(dim, k, W.box_nodes(dim, nc, k, amp), W.box_neighbors(dim, nc), mat)


def varying(dim, seed=11):
    return W.FourierMaterial(seed, dim=dim, rho_amp=0.3)


def test_density_field_varies_inside_cells():
    m = make(3, 2, 3, 0.05, varying(3))
    cd = m.cell_data(np.arange(m.nc))
    assert np.ptp(cd["rho"], axis=1).min() > 1e-2
    assert 0.7 <= cd["rho"].min() and cd["rho"].max() <= 1.3
    # c is the same field as with a constant density
    assert np.array_equal(cd["c"], W.FourierMaterial(11, dim=3).c(cd["x"]))


def _energy_form(m, U, V):
    """E(U, V) = (||U + V||^2 - ||U - V||^2) / 4 with the physical energy norm."""
    return 0.25 * (norms.energy_norm2(m, U + V) - norms.energy_norm2(m, U - V))


def _jump_dissipation(m, U, mat):
    """-sum over faces of (Z/2 [v_n]^2 + [p]^2 / (2 Z)), each face once, with
    the traces evaluated from the GL tables and Z = rho c from the material at
    the face points."""
    d = m.dim
    tot = 0.0
    for f in range(1, 2 * d, 2):
        fd = m.face_data(np.arange(m.nc), f)
        um = np.einsum("qi,cvi->cvq", basis.tensor_basis(m.xgl, m.face_ref[f]), U)
        up = np.einsum("qi,cvi->cvq", basis.tensor_basis(m.xgl, m.face_ref[f ^ 1]), U[fd["nb"]])
        area = np.linalg.norm(fd["a"], axis=-1)
        nrm = fd["a"] / area[..., None]
        jv = np.einsum("cqa,caq->cq", nrm, um[:, :d] - up[:, :d])
        jp = um[:, d] - up[:, d]
        rho, c = mat(fd["x"])
        Z = rho * c
        tot -= np.sum(area * (0.5 * Z * jv ** 2 + jp ** 2 / (2 * Z)))
    return tot


@pytest.mark.parametrize("dim,nc,k", [(2, 3, 3), (2, 2, 5), (3, 2, 2)])
def test_energy_identity_affine_variable_density(dim, nc, k):
    mat = varying(dim)
    m = make(dim, nc, k, 0.0, mat)
    U = W.random_state(5 + k, (m.nc, dim + 1, m.np_))
    Lc = apply_operator(m, U, flux="central")
    Lu = apply_operator(m, U, flux="upwind")
    scale = np.sqrt(norms.energy_norm2(m, U) * norms.energy_norm2(m, Lu))
    assert abs(_energy_form(m, U, Lc)) < 1e-13 * scale
    diss = _jump_dissipation(m, U, mat)
    assert diss < 0 and abs(_energy_form(m, U, Lu) - diss) < 1e-12 * abs(diss)


def test_energy_identity_fails_for_a_misplaced_density():
    """The same identity with the density of the energy form inverted (a
    plausible slip) is violated: the pin can see where rho goes."""
    dim, nc, k = 2, 3, 3
    mat = varying(dim)
    m = make(dim, nc, k, 0.0, mat)

    class Inverted:
        def __call__(self, x):
            r, c = mat(x)
            return 1.0 / r, c * r  # same impedance, density inverted

    mi = make(dim, nc, k, 0.0, Inverted())
    U = W.random_state(8, (m.nc, dim + 1, m.np_))
    Lu = apply_operator(m, U, flux="central")
    scale = np.sqrt(norms.energy_norm2(m, U) * norms.energy_norm2(m, Lu))
    assert abs(_energy_form(mi, U, Lu)) > 1e-3 * scale


def _dense(m, fn, N):
    A = np.empty((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        A[:, j] = fn(e.reshape(m.nc, m.dim + 1, m.np_)).ravel()
    return A


@pytest.mark.parametrize("dim,k,amp", [(2, 3, 0.0), (2, 2, 0.05), (3, 2, 0.0)])
def test_single_cell_brute_force_variable_density(dim, k, amp):
    m = make(dim, 1, k, amp, varying(dim, seed=21))
    N = (dim + 1) * m.np_
    eye = np.eye(N)
    M = np.array([[_energy_form(m, eye[i].reshape(1, dim + 1, m.np_), eye[j].reshape(1, dim + 1, m.np_))
                   for j in range(N)] for i in range(N)])
    A = M @ _dense(m, lambda u: apply_operator(m, u, flux="upwind"), N)
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.max() < 1e-12 * np.abs(ev).max()
    assert ev.min() < -1e-3 * np.abs(ev).max()
    if amp == 0.0:
        Bc = M @ _dense(m, lambda u: apply_operator(m, u, flux="central"), N)
        assert np.abs(Bc + Bc.T).max() < 1e-12 * np.abs(Bc).max()


@pytest.mark.parametrize("dim,amp", [(2, 0.05), (3, 0.05)])
def test_constant_state_steady_variable_density(dim, amp):
    m = make(dim, 2, 3, amp, varying(dim))
    U = np.zeros((m.nc, dim + 1, m.np_))
    U[:] = np.linspace(0.3, 1.4, dim + 1)[None, :, None]
    scale = np.abs(apply_operator(m, W.random_state(3, U.shape))).max()
    assert np.abs(apply_operator(m, U)).max() < 1e-12 * scale


def test_graded_medium_wave_solves_the_pde():
    """The closed form (p, v) of the graded medium satisfies the PDE: finite
    differences of the recipe, independent of any DG code."""
    g = W.GradedMedium()
    x = W.random_points(4, 50, 2)
    h = 1e-5
    rho, c = g(x)
    dt = (g.wave(x, 0.3 + h) - g.wave(x, 0.3 - h)) / (2 * h)
    dx = (g.wave(x + [h, 0], 0.3) - g.wave(x - [h, 0], 0.3)) / (2 * h)
    dy = (g.wave(x + [0, h], 0.3) - g.wave(x - [0, h], 0.3)) / (2 * h)
    assert np.abs(rho * dt[:, 0] + dx[:, 2]).max() < 1e-8
    assert np.abs(rho * dt[:, 1] + dy[:, 2]).max() < 1e-8
    assert np.abs(dt[:, 2] + rho * c ** 2 * (dx[:, 0] + dy[:, 1])).max() < 1e-8
    assert np.ptp(rho) > 0.5 and np.ptp(c) > 0.5


def _graded_error(dim, nc, k, scheme, T=0.15):
    g = W.GradedMedium()
    m = make(dim, nc, k, 0.05, g)
    U = m.interpolate(lambda x: g.wave(x, 0.0))
    dt, ns = ts.dt_from_courant(m, 0.15, T)
    for s in range(ns):
        if scheme == "lsrk":
            U = ts.lsrk_step(lambda u, t: apply_operator(m, u), U, s * dt, dt)
        else:
            U = ader.ader_step(m, U, dt)
    return norms.l2_error(m, U, g.wave, T)


@pytest.mark.parametrize("k,scheme", [(2, "lsrk"), (3, "lsrk"), (3, "ader")])
def test_graded_medium_convergence(k, scheme):
    """Order k+1 against the closed form on the curved 2D box with rho and c
    varying inside every cell."""
    e1 = _graded_error(2, 4, k, scheme)
    e2 = _graded_error(2, 8, k, scheme)
    rate_p = np.log2(e1[0] / e2[0])
    rate_v = np.log2(e1[1] / e2[1])
    assert rate_p > k + 1 - 0.4 and rate_v > k + 1 - 0.4, (e1, e2)


def test_graded_medium_convergence_3d():
    e1 = _graded_error(3, 3, 2, "lsrk", T=0.1)
    e2 = _graded_error(3, 6, 2, "lsrk", T=0.1)
    assert np.log2(e1[0] / e2[0]) > 2.6 and np.log2(e1[1] / e2[1]) > 2.6, (e1, e2)
