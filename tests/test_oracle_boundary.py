"""Pins of the oracle's boundary faces (rigid wall, first-order absorbing).

The paper asks for boundary conditions without fixing any (Sec. 2); the
reading is the mirror state for a wall and the zero exterior state for an
absorbing face, both through the interior flux (oracle/operator.py).  Pins:
the closed-form solutions themselves satisfy the PDE and the conditions; the
semi-discrete energy rate (U, M L U) = (U, -K U) vanishes with the central
flux and walls, is negative with upwind; the wall box carries the
standing membrane mode and the absorbing box lets a plane pulse leave, both
converging at order k+1 against the closed form.  A wrong sign in the mirror
state or an exterior impedance from a non-existent neighbour fails them."""
import numpy as np
import pytest

import workloads as W
from oracle import Mesh, BC_WALL, BC_ABSORBING, apply_operator, norms, timestep as ts
from oracle.operator import residual


def _fd_check(fn, dim):
    """Central differences: p_t = -div v, v_t = -grad p (rho = c = 1)."""
    rng = np.random.default_rng(3)
    x = rng.uniform(0.05, 0.95, size=(20, dim))
    t, h = 0.37, 1e-5
    ut = (fn(x, t + h) - fn(x, t - h)) / (2 * h)
    div = np.zeros(len(x))
    grad = np.zeros((len(x), dim))
    for a in range(dim):
        e = np.zeros(dim)
        e[a] = h
        dp = (fn(x + e, t) - fn(x - e, t)) / (2 * h)
        div += dp[:, a]
        grad[:, a] = dp[:, dim]
    assert np.max(np.abs(ut[:, dim] + div)) < 1e-6
    assert np.max(np.abs(ut[:, :dim] + grad)) < 1e-6


@pytest.mark.parametrize("dim", [2, 3])
def test_membrane_mode_solves_the_wall_problem(dim):
    fn = lambda x, t: W.membrane_mode(x, t, m=[1, 2, 1][:dim])
    _fd_check(fn, dim)
    # v.n = 0 on every wall
    rng = np.random.default_rng(4)
    for a in range(dim):
        for side in (0.0, 1.0):
            x = rng.uniform(0, 1, size=(10, dim))
            x[:, a] = side
            assert np.max(np.abs(fn(x, 0.3)[:, a])) < 1e-14


def test_travelling_pulse_solves_the_pde():
    _fd_check(lambda x, t: W.travelling_pulse_x(x, t, x0=0.5, width=0.1), 2)


def test_box_neighbors_boundary_codes():
    nb = W.box_neighbors(2, 3, bc=("wall", "absorbing"))
    # cell 0 is at x index 0, y index 0; cell 8 at (2, 2)
    assert nb[0, 0] == BC_WALL and nb[0, 2] == BC_ABSORBING and nb[0, 1] == 1 and nb[0, 3] == 3
    assert nb[8, 1] == BC_WALL and nb[8, 3] == BC_ABSORBING and nb[8, 0] == 7 and nb[8, 2] == 5
    assert (nb >= 0).sum() == 2 * 2 * 3 * 2  # interior faces seen from both sides
    with pytest.raises(ValueError):
        Mesh(2, 2, W.box_nodes(2, 3, 2, 0.0), np.where(nb < 0, -4, nb), W.ConstantMaterial())


def _energy_rate(m, U, flux):
    r = residual(m, U, np.arange(m.nc), flux=flux)
    return float(np.sum(U * r)), float(np.sum(U * U))


@pytest.mark.parametrize("dim,bc", [(2, ("wall", "wall")), (3, ("wall", "periodic", "wall"))])
def test_energy_rate_with_walls(dim, bc):
    """Affine cells: the Gauss rule integrates the volume terms exactly, so
    (U, -K U) reduces to face terms, which cancel between neighbours and
    vanish on walls for the central flux (on curved cells the quadrature of
    the metric terms leaves a rounding-free but nonzero remainder)."""
    k, nc = 3, 3
    m = Mesh(dim, k, W.box_nodes(dim, nc, k, 0.0), W.box_neighbors(dim, nc, bc), W.FourierMaterial(5, dim=dim))
    U = W.random_state(11, (m.nc, dim + 1, m.np_))
    rate, scale = _energy_rate(m, U, "central")
    assert abs(rate) < 1e-12 * scale
    rate_up, _ = _energy_rate(m, U, "upwind")
    assert rate_up < -1e-6 * scale
    # a wrong mirror (v+ = v-) would let energy through the walls
    m_p = Mesh(dim, k, W.box_nodes(dim, nc, k, 0.0), W.box_neighbors(dim, nc), W.FourierMaterial(5, dim=dim))
    rate_p, _ = _energy_rate(m_p, U, "central")
    assert abs(rate_p) < 1e-12 * scale


def test_energy_rate_absorbing_is_dissipative():
    dim, k, nc = 2, 3, 3
    m = Mesh(dim, k, W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc, ("absorbing", "periodic")),
             W.FourierMaterial(6, dim=dim))
    U = W.random_state(12, (m.nc, dim + 1, m.np_))
    rate, scale = _energy_rate(m, U, "upwind")
    assert rate < -1e-6 * scale


def test_energy_rate_boundary_terms_affine():
    """Affine cells, central flux inside: (U, -K U) is the sum of the boundary
    terms p v.n - p* v.n - p v*_n, i.e. 0 on a wall with central flux and
    -(p^2 + Z^2 (v.n)^2) / (2Z) on an absorbing face with upwind flux.  Checked
    on a state that vanishes near every face but the -x ones (interior
    faces then carry nothing)."""
    dim, k, nc = 2, 3, 2
    m = Mesh(dim, k, W.box_nodes(dim, nc, k, 0.0), W.box_neighbors(dim, nc, ("absorbing", "periodic")),
             W.ConstantMaterial(rho=1.0, c=2.0))
    # v_x = s, p = 0.3 s with s = (x - 1/2)^2 cos(2 pi y) at the GL nodes of the
    # cells at x index 0 (s vanishes at their +x face and is continuous across
    # their y faces, so no interior face sees a jump)
    x = m.node_points()
    U = np.zeros((m.nc, dim + 1, m.np_))
    for c in range(m.nc):
        if m.neighbors[c, 0] < 0:
            s = (x[c, :, 0] - 0.5) ** 2 * np.cos(2 * np.pi * x[c, :, 1])
            U[c, 0] = s
            U[c, dim] = 0.3 * s
    rate, _ = _energy_rate(m, U, "upwind")
    # the -x face x = 0: trace s = 0.25 g(y), g the cubic interpolant of
    # cos(2 pi y) at the 4 GL nodes of each cell; v.n = -s, p = 0.3 s, Z = 2
    gl = np.array([-1.0, -1 / np.sqrt(5.0), 1 / np.sqrt(5.0), 1.0])
    yq, wq = np.polynomial.legendre.leggauss(20)
    want = 0.0
    for y0 in (0.0, 0.5):
        yn = y0 + 0.25 * (gl + 1)
        coef = np.polyfit(yn, np.cos(2 * np.pi * yn), 3)
        y = y0 + 0.25 * (yq + 1)
        sv = 0.25 * np.polyval(coef, y)
        want -= np.sum(0.25 * wq * ((0.3 * sv) ** 2 + 4.0 * sv ** 2) / 4.0)
    assert abs(rate - want) < 1e-12 * abs(want)


def _run_lsrk(m, U0, T, cr):
    h = 1.0 / round(m.nc ** (1.0 / m.dim))
    dt = cr * h / m.k ** 1.5
    n = int(np.ceil(T / dt))
    dt = T / n
    U = U0
    for s in range(n):
        U = ts.lsrk_step(lambda x, t: apply_operator(m, x), U, s * dt, dt)
    return U


@pytest.mark.parametrize("amp", [0.0, 0.05])
def test_wall_box_membrane_mode_converges(amp):
    """2D box with walls on all sides, k = 3: the (1, 1) membrane mode at
    T = 0.3 against the closed form on 3^2 and 6^2 cells."""
    k, T = 3, 0.3
    errs = []
    for nc in (3, 6):
        m = Mesh(2, k, W.box_nodes(2, nc, k, amp), W.box_neighbors(2, nc, ("wall", "wall")), W.ConstantMaterial())
        U = _run_lsrk(m, m.interpolate(lambda x: W.membrane_mode(x, 0.0)), T, 0.2)
        errs.append(norms.l2_error(m, U, W.membrane_mode, T)[0])
    assert errs[1] < (1e-5 if amp == 0.0 else 1e-4)
    assert errs[0] / errs[1] > 2 ** (k + 1) * 0.6


def test_absorbing_box_lets_the_pulse_leave():
    """2D box, absorbing x faces, periodic y, k = 3: a right-going pulse half
    way through the +x face at T = 0.3 against the closed form, and no
    reflection left behind once it has gone."""
    k, T = 3, 0.3
    exact = lambda x, t: W.travelling_pulse_x(x, t, x0=0.6, width=0.08)
    errs = []
    for nc in (6, 12):
        m = Mesh(2, k, W.box_nodes(2, nc, k, 0.0), W.box_neighbors(2, nc, ("absorbing", "periodic")),
                 W.ConstantMaterial())
        U = _run_lsrk(m, m.interpolate(lambda x: exact(x, 0.0)), T, 0.2)
        errs.append(norms.l2_error(m, U, exact, T)[0])
    assert errs[1] < 5e-4
    assert errs[0] / errs[1] > 2 ** (k + 1) * 0.5
    # after the pulse has left: the energy left is small
    U = _run_lsrk(m, m.interpolate(lambda x: exact(x, 0.0)), 0.75, 0.2)
    assert norms.energy_norm2(m, U) < 1e-6 * norms.energy_norm2(m, m.interpolate(lambda x: exact(x, 0.0)))
