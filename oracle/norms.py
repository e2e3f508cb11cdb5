"""Energy norm, errors against closed-form solutions and parity measures (oracle).

The physical norm is the acoustic energy (twice it):
||u||^2 = sum_K (v, rho v)_K + (p, p/(rho c^2))_K, by Gauss quadrature on
n = k+1 points per direction, the rule the paper uses throughout (Sec. 3).
"""
from __future__ import annotations

import numpy as np

from .operator import tables


def values_at_gauss(mesh, U, cells=None):
    cells = np.arange(mesh.nc) if cells is None else cells
    T = tables(mesh)
    return np.einsum("qi,cvi->cvq", T.phi, np.asarray(U)[cells] if len(U) == mesh.nc else U)


def energy_norm2(mesh, U):
    d = mesh.dim
    cd = mesh.cell_data(np.arange(mesh.nc))
    uq = values_at_gauss(mesh, U)
    ev = np.sum(cd["wdet"] * cd["rho"] * np.sum(uq[:, :d] ** 2, axis=1))
    ep = np.sum(cd["wdet"] / (cd["rho"] * cd["c"] ** 2) * uq[:, d] ** 2)
    return float(ev + ep)


def energy_rel_diff(mesh, A, B):
    """||A - B|| / ||B|| in the energy norm."""
    return float(np.sqrt(energy_norm2(mesh, np.asarray(A) - np.asarray(B)) / energy_norm2(mesh, B)))


def rel_l2(a, b):
    """Plain coefficient 2-norm relative difference ||a - b|| / ||b||."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def l2_error(mesh, U, exact, t):
    """(L2 error of p, L2 error of v) against exact(x, t) -> [..., d+1] at the
    Gauss points of the mapped cells."""
    d = mesh.dim
    cd = mesh.cell_data(np.arange(mesh.nc))
    uq = values_at_gauss(mesh, U)                    # [C][d+1][Q]
    ue = np.moveaxis(exact(cd["x"], t), -1, 1)       # [C][d+1][Q]
    e = uq - ue
    ep = np.sqrt(np.sum(cd["wdet"] * e[:, d] ** 2))
    ev = np.sqrt(np.sum(cd["wdet"] * np.sum(e[:, :d] ** 2, axis=1)))
    return float(ep), float(ev)
