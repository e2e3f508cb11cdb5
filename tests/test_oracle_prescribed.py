"""Pins of the oracle's prescribed exterior state (boundary faces that take
given data u_ext, a reading: the paper leaves boundary conditions open,
Sec. 2).  The data are plane waves (workloads.PlaneWaves), which are also
the closed-form solution: the waves solve the PDE and their integral is the
time integral; a zero exterior equals the absorbing condition exactly; LSRK
(exterior at the stage times) and ADER (exterior integrated over the step)
converge to the plane wave at order k+1 on a non-periodic box, curved cells
included.  A wrong sign in the exterior velocity, the exterior taken at the
wrong time or a missing time integral in ADER fails one of them."""
import numpy as np
import pytest

import workloads as W
from oracle import Mesh, apply_operator, ader, norms, timestep as ts


def _wave(dim):
    k = 2 * np.pi * np.array([1.0, 0.6, 0.3])[:dim]
    kn = np.linalg.norm(k)
    # rho = 1, c = 1.3: omega = c |k|, Z = rho c
    return W.PlaneWaves([[1.0, *np.pad(k, (0, 3 - dim)), 1.3 * kn, 0.4, 1.3]])


@pytest.mark.parametrize("dim", [2, 3])
def test_plane_waves_solve_the_pde_and_integrate(dim):
    pw = _wave(dim)
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, size=(15, dim))
    t, h = 0.3, 1e-5
    ut = (pw(x, t + h) - pw(x, t - h)) / (2 * h)
    div = np.zeros(len(x))
    grad = np.zeros((len(x), dim))
    for a in range(dim):
        e = np.zeros(dim)
        e[a] = h
        du = (pw(x + e, t) - pw(x - e, t)) / (2 * h)
        div += du[:, a]
        grad[:, a] = du[:, dim]
    # rho = 1, c = 1.3: p_t = -rho c^2 div v, v_t = -grad p / rho
    assert np.max(np.abs(ut[:, dim] + 1.69 * div)) < 1e-5
    assert np.max(np.abs(ut[:, :dim] + grad)) < 1e-5
    s, w = np.polynomial.legendre.leggauss(30)
    t0, dt = 0.2, 0.07
    quad = sum(0.5 * dt * wi * pw(x, t0 + 0.5 * dt * (si + 1)) for si, wi in zip(s, w))
    assert np.max(np.abs(pw.integral(x, t0, dt) - quad)) < 1e-13


def test_zero_exterior_is_absorbing():
    dim, k, nc = 2, 3, 3
    mat = W.FourierMaterial(6, dim=dim)
    nodes = W.box_nodes(dim, nc, k, 0.05)
    m_p = Mesh(dim, k, nodes, W.box_neighbors(dim, nc, ("prescribed", "periodic")), mat)
    m_a = Mesh(dim, k, nodes, W.box_neighbors(dim, nc, ("absorbing", "periodic")), mat)
    U = W.random_state(31, (m_p.nc, dim + 1, m_p.np_))
    zero = lambda x: np.zeros(x.shape[:-1] + (dim + 1,))
    assert np.array_equal(apply_operator(m_p, U, exterior=zero), apply_operator(m_a, U))
    with pytest.raises(ValueError):
        apply_operator(m_p, U)


class _Mat:
    """rho = 1, c = 1.3 everywhere."""

    def __call__(self, x):
        x = np.asarray(x)
        return np.ones(x.shape[:-1]), np.full(x.shape[:-1], 1.3)


def _errors(dim, k, amp, scheme, T=0.25, ncs=(3, 6)):
    pw = _wave(dim)
    errs = []
    for nc in ncs:
        m = Mesh(dim, k, W.box_nodes(dim, nc, k, amp), W.box_neighbors(dim, nc, ("prescribed",) * dim), _Mat())
        dt0 = 0.15 / nc / 1.3 / k ** 1.5
        n = int(np.ceil(T / dt0))
        dt = T / n
        U = m.interpolate(lambda x: pw(x, 0.0))
        for s in range(n):
            if scheme == "lsrk":
                U = ts.lsrk_step(lambda u, t: apply_operator(m, u, exterior=lambda x: pw(x, t)), U, s * dt, dt)
            else:
                U = ader.ader_step(m, U, dt, exterior_integral=lambda x: pw.integral(x, s * dt, dt))
        errs.append(norms.l2_error(m, U, lambda x, t: pw(x, t), T)[0])
    return errs


@pytest.mark.parametrize("scheme,amp", [("lsrk", 0.0), ("lsrk", 0.05), ("ader", 0.05)])
def test_prescribed_box_converges_to_the_plane_wave(scheme, amp):
    k = 3
    e = _errors(2, k, amp, scheme)
    assert e[1] < (2e-4 if amp == 0.0 else 1e-3)
    assert e[0] / e[1] > 2 ** (k + 1) * 0.6


def test_prescribed_box_3d_plane_wave_converges():
    e = _errors(3, 3, 0.05, "ader", T=0.1, ncs=(2, 4))
    assert e[1] < 5e-3 and e[0] / e[1] > 2 ** 4 * 0.55
    # the exterior integral matters: taking the state at t instead of its
    # integral over the step is wrong by a factor dt and blows the error up
    pw = _wave(3)
    m = Mesh(3, 3, W.box_nodes(3, 2, 3, 0.05), W.box_neighbors(3, 2, ("prescribed",) * 3), _Mat())
    U = m.interpolate(lambda x: pw(x, 0.0))
    dt = 0.01
    good = ader.ader_step(m, U, dt, exterior_integral=lambda x: pw.integral(x, 0.0, dt))
    bad = ader.ader_step(m, U, dt, exterior_integral=lambda x: pw(x, 0.0))
    exact = m.interpolate(lambda x: pw(x, dt))
    assert norms.rel_l2(good, exact) < 0.05 * norms.rel_l2(bad, exact)
