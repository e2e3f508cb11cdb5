"""Pins of the oracle's point-source pieces (not from the paper; the injection
itself is "parity unpinned"): the Ricker derivatives and antiderivative
against finite differences and quadrature, and the point location by Newton
iteration against the map."""
import numpy as np
import pytest
from scipy.integrate import quad

import workloads as W
from oracle import Mesh, sources


def test_ricker_closed_forms():
    r = sources.Ricker(f=8.0, amp=1.7)
    assert abs(r(0.0)) < 1e-4 * 1.7
    assert abs(r(r.t0) - 1.7) < 1e-15
    h = 1e-5
    for t in (0.05, 0.13, 0.2, 0.31):
        for l in range(4):
            fd = (r.deriv(t + h, l) - r.deriv(t - h, l)) / (2 * h)
            assert abs(r.deriv(t, l + 1) - fd) < 1e-6 * max(1.0, abs(fd))
        val, _ = quad(r, 0.0, t, epsabs=1e-13, epsrel=1e-13)
        assert abs(r.integral(0.0, t) - val) < 1e-11


def test_locate_point():
    m = Mesh(3, 3, W.box_nodes(3, 3, 3, 0.05), W.box_neighbors(3, 3), W.ConstantMaterial())
    for xs in W.random_points(3, 5, 3):
        cell, xi = sources.locate(m, xs)
        x, _ = m.map_points([cell], xi[None, :])
        assert np.max(np.abs(x[0, 0] - xs)) < 1e-12
        assert np.all(xi >= 0) and np.all(xi <= 1)
