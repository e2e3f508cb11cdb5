"""Loose pin of the oracle's time steppers against the paper's printed
critical Courant numbers (Sec. 4.6, Table 2; golden file
tests/golden/table2_critical_courant.txt).

Stability is judged as a run would: the amplification over one unit of time,
max |lambda|^(1/dt), must stay below 2 (the Taylor polynomials behind ADER
grow by ~1e-7 per step on undamped modes for some k, which no run notices).
The LSRK4(5) coefficients here are a reading (the paper's reference is not
reproduced) and the mesh is a small periodic box, so the check is that
Cr_crit lies within 0.8-1.2 times the printed value."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import Mesh, apply_operator, ader

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_critical_courant.txt")


def table2():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            d, k, rk45, rk59, ad = line.split()
            out[(int(d), int(k))] = dict(lsrk=float(rk45), ader=float(ad))
    return out


def _dense(m, fn, shape):
    N = int(np.prod(shape))
    return np.column_stack([fn(e.reshape(shape)).ravel() for e in np.eye(N)])


def _setup(dim, nc, k):
    m = Mesh(dim, k, W.box_nodes(dim, nc, k, 0.0), W.box_neighbors(dim, nc), W.ConstantMaterial())
    shape = (m.nc, dim + 1, m.np_)
    L = _dense(m, lambda u: apply_operator(m, u), shape)
    return m, L


def _stable(ev, dt):
    return np.max(np.abs(ev)) ** (1.0 / dt) <= 2.0


def _lsrk_stable(lam, dt):
    z = dt * lam
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24 + z ** 5 / 200
    return _stable(R, dt)


def _ader_stable(m, L, dt):
    # the TCK sum is cell-local and identical on every cell of the Cartesian box
    nloc = (m.dim + 1) * m.np_

    def one_cell(e):
        U = np.zeros((m.nc, m.dim + 1, m.np_))
        U[0] = e.reshape(m.dim + 1, m.np_)
        return ader.tck(m, U, dt, cells=[0])[0]
    B = _dense(m, one_cell, (nloc,))
    T = np.kron(np.eye(m.nc), B)
    return _stable(np.linalg.eigvals(np.eye(L.shape[0]) + L @ T), dt)


@pytest.mark.parametrize("dim,nc,k", [(2, 4, 1), (2, 4, 4), (2, 3, 7), (3, 3, 1)])
def test_critical_courant_numbers(dim, nc, k):
    ref = table2()[(dim, k)]
    m, L = _setup(dim, nc, k)
    lam = np.linalg.eigvals(L)
    h = 1.0 / nc
    dt = lambda cr: cr * h / k ** 1.5
    assert _lsrk_stable(lam, dt(0.8 * ref["lsrk"]))
    assert not _lsrk_stable(lam, dt(1.2 * ref["lsrk"]))
    assert _ader_stable(m, L, dt(0.8 * ref["ader"]))
    assert not _ader_stable(m, L, dt(1.2 * ref["ader"]))
