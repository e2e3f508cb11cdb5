"""Low-storage Runge-Kutta time stepping and the time-step size (oracle).

Paper, Sec. 2.2: explicit Runge-Kutta in Butcher form and the two-register
low-storage schemes of Kennedy, Carpenter and Lewis (LSRK4(5): five stages,
order four).  The coefficients of that reference are not reproduced in the
paper; the reading taken here is the five-stage fourth-order 2N-storage
scheme of Carpenter and Kennedy (NASA TM-109112, 1994) in Williamson form

    du <- A_i du + dt F(u, t + c_i dt);   u <- u + B_i du,   i = 1..5.

Sec. 2.3 gives the Courant number Cr = c dt k^1.5 / h; "a characteristic
element size h" is read as the smallest singular value of the Jacobian over
the cell's Gauss points (1/n on the uniform n^d box), c as its largest value
over those points.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

LSRK54_A = [Fraction(0), Fraction(-567301805773, 1357537059087),
            Fraction(-2404267990393, 2016746695238), Fraction(-3550918686646, 2091501179385),
            Fraction(-1275806237668, 842570457699)]
LSRK54_B = [Fraction(1432997174477, 9575080441755), Fraction(5161836677717, 13612068292357),
            Fraction(1720146321549, 2090206949498), Fraction(3134564353537, 4481467310338),
            Fraction(2277821191437, 14882151754819)]
LSRK54_C = [Fraction(0), Fraction(1432997174477, 9575080441755),
            Fraction(2526269341429, 6820363962896), Fraction(2006345519317, 3224310063776),
            Fraction(2802321613138, 2924317926251)]


def lsrk_butcher(A=LSRK54_A, B=LSRK54_B):
    """Butcher tableau (a, b, c) of a 2N-storage scheme, in exact rationals.

    With du_i = A_i du_{i-1} + dt k_i and u_i = u_{i-1} + B_i du_i, the stage
    increment du_i = dt sum_{j<=i} (prod_{l=j+1..i} A_l) k_j, so
    b_j = sum_{i>=j} B_i prod_{l=j+1..i} A_l and a_{ij} for stage i+1 sums the
    B's of the stages before it in the same way.
    """
    s = len(A)
    coef = [[Fraction(0)] * s for _ in range(s)]  # coef[i][j]: weight of k_j in du_i
    for i in range(s):
        for j in range(i + 1):
            w = Fraction(1)
            for l in range(j + 1, i + 1):
                w *= A[l]
            coef[i][j] = w
    b = [sum(B[i] * coef[i][j] for i in range(j, s)) for j in range(s)]
    a = [[Fraction(0)] * s for _ in range(s)]
    for i in range(1, s):
        for j in range(i):
            a[i][j] = sum(B[m] * coef[m][j] for m in range(j, i))
    c = [sum(row) for row in a]
    return a, b, c


def lsrk_step(rhs, U, t, dt, A=LSRK54_A, B=LSRK54_B, C=LSRK54_C):
    """One 2N-storage step: rhs(U, t) -> dU/dt.  Returns the new state."""
    u = np.array(U, dtype=np.float64, copy=True)
    du = np.zeros_like(u)
    for Ai, Bi, Ci in zip(A, B, C):
        du = float(Ai) * du + dt * rhs(u, t + float(Ci) * dt)
        u = u + float(Bi) * du
    return u


def cell_h_and_c(mesh, cells=None):
    """(h_K, c_K) per cell: min over the Gauss points of the smallest singular
    value of J, and max over the Gauss points of c."""
    cells = np.arange(mesh.nc) if cells is None else cells
    cd = mesh.cell_data(cells)
    sv = np.linalg.svd(cd["J"], compute_uv=False)   # [C][Q][d]
    return sv[..., -1].min(axis=1), cd["c"].max(axis=1)


def dt_from_courant(mesh, cr, t_end=None):
    """dt = Cr min_K(h_K / c_K) / k^1.5, rounded down so that dt = T / ceil(T/dt)."""
    h, c = cell_h_and_c(mesh)
    dt = cr * float(np.min(h / c)) / mesh.k ** 1.5
    if t_end is None:
        return dt, None
    nsteps = int(math.ceil(t_end / dt - 1e-12))
    return t_end / nsteps, nsteps
