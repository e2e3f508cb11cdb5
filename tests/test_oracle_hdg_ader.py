"""Pins of the oracle's HDG-ADER variant (Sec. 2.4, eq. hdg-ader): the first
element-local derivative of the TCK sum is replaced by the DG derivative.

* For a GL interpolant of a smooth periodic field the traces of neighbours
  coincide (GL nodes include the face nodes), so every flux returns the own
  trace; on affine cells with constant material and exact quadrature the DG
  derivative then equals the element-local one, and HDG-ADER must give the
  ADER step to rounding (both with and without the degree reduction).  A
  wrong coefficient shift or a missing dt U term fails it.
* On a discontinuous state the two differ, at second order in dt (the first
  differing term is dt^2/2 L(L U + S U)).
* Joint space-time convergence against the closed-form standing wave at
  order k+1 and bounded energy over many steps at Cr 0.1."""
import numpy as np
import pytest

import workloads as W
from oracle import Mesh, ader, norms, timestep as ts


@pytest.mark.parametrize("dim,k,reduce", [(2, 3, True), (2, 4, False), (3, 3, True)])
def test_hdg_equals_ader_on_continuous_states(dim, k, reduce):
    nc = 3
    m = Mesh(dim, k, W.box_nodes(dim, nc, k, 0.0), W.box_neighbors(dim, nc), W.ConstantMaterial(rho=1.3, c=0.8))
    U = m.interpolate(lambda x: W.gaussian_pulse(x, [0.4] * dim, 0.2) +
                      0.3 * np.stack([np.sin(2 * np.pi * x[..., a]) for a in range(dim)] +
                                     [np.cos(2 * np.pi * x[..., 0])], axis=-1))
    dt = 0.1 / nc / k ** 1.5
    a = ader.ader_step(m, U, dt, reduce=reduce)
    h = ader.hdg_ader_step(m, U, dt, reduce=reduce)
    assert norms.rel_l2(h - U, a - U) < 1e-11


def test_hdg_differs_from_ader_at_second_order():
    dim, k, nc = 2, 3, 3
    m = Mesh(dim, k, W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc), W.FourierMaterial(2, dim=dim))
    U = W.random_state(4, (m.nc, dim + 1, m.np_))
    diffs = []
    for dt in (1e-3, 5e-4):
        diffs.append(np.linalg.norm(ader.hdg_ader_step(m, U, dt) - ader.ader_step(m, U, dt)))
    assert diffs[0] > 1e-10
    assert 3.5 < diffs[0] / diffs[1] < 4.5


def test_hdg_ader_joint_convergence():
    k, T = 3, 0.2
    errs = []
    for nc in (8, 16):
        m = Mesh(2, k, W.box_nodes(2, nc, k, 0.05), W.box_neighbors(2, nc), W.ConstantMaterial())
        dt, n = ts.dt_from_courant(m, 0.1, T)
        U = m.interpolate(lambda x: W.standing_wave_2d(x, 0.0))
        for s in range(n):
            U = ader.hdg_ader_step(m, U, dt)
        errs.append(norms.l2_error(m, U, W.standing_wave_2d, n * dt)[0])
    assert errs[1] < 2e-5
    assert errs[0] / errs[1] > 2 ** (k + 1) * 0.6


def test_hdg_ader_energy_bounded():
    dim, k, nc = 2, 4, 3
    m = Mesh(dim, k, W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc), W.FourierMaterial(3, dim=dim))
    dt, n = ts.dt_from_courant(m, 0.1, 0.5)
    U = m.interpolate(lambda x: W.gaussian_pulse(x, [0.5, 0.5], 0.15))
    e0 = norms.energy_norm2(m, U)
    for s in range(n):
        U = ader.hdg_ader_step(m, U, dt)
    assert norms.energy_norm2(m, U) <= e0 * (1 + 1e-10)
