"""Low-storage Runge-Kutta time stepping and the time-step size (oracle).

Paper, Sec. 2.2: explicit Runge-Kutta in Butcher form and the two-register
low-storage schemes of Kennedy, Carpenter and Lewis (LSRK4(5): five stages,
order four).  The coefficients of that reference are not reproduced in the
paper; the reading taken here is the five-stage fourth-order 2N-storage
scheme of Carpenter and Kennedy (NASA TM-109112, 1994) in Williamson form

    du <- A_i du + dt F(u, t + c_i dt);   u <- u + B_i du,   i = 1..5.

LSRK5(9) (the paper's second scheme: nine stages, order five, two
registers; its coefficients are not reproduced either).  Reading: the
two-register (2R) form, whose Butcher tableau has a_ij = b_j for j < i-1 and
a free subdiagonal a_{i,i-1} = alpha_i, so nine stages leave 8 + 9 = 17 free
coefficients for the 17 conditions of order five.  These have a finite set
of real solutions; the one taken is named by the 10-digit key
LSRK59_KEY_ALPHA / LSRK59_KEY_B and refined to full precision by Newton's
method on the conditions (it has all c_i in [0, 1] and |coefficients| <=
0.62).  The step is the plain explicit Runge-Kutta step of that tableau.

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


LSRK59_KEY_ALPHA = [0.1702644982, -0.09676474868, 0.0244514839, 0.1382907685, 0.2294641842, 0.5748250612,
                    -0.1211285367, 0.09183392377]
LSRK59_KEY_B = [0.1804864076, 0.622352667, -0.4110536782, -0.01125784998, 0.009612188747, 0.1576014651,
                0.1129031225, 0.08522852155, 0.2541271558]


def tableau_2r(alpha, b):
    """Butcher (a, b, c) of a two-register scheme: a_ij = b_j (j < i-1), a_{i,i-1} = alpha_i."""
    s = len(b)
    a = np.zeros((s, s), dtype=np.result_type(np.asarray(alpha), np.asarray(b)))
    for i in range(1, s):
        a[i, :i - 1] = b[:i - 1]
        a[i, i - 1] = alpha[i - 1]
    b = np.asarray(b)
    return a, b, a.sum(axis=1)


def order5_conditions(a, b):
    """The 17 order conditions of order five, sum_j b_j Phi_j(tree) - 1/gamma(tree),
    for the rooted trees with up to five vertices (order 1: 1, 2: 1, 3: 2, 4: 4, 5: 9)."""
    c = a.sum(axis=1)
    ac, ac2, ac3 = a @ c, a @ c ** 2, a @ c ** 3
    aac = a @ ac
    return np.array([
        b.sum() - 1, b @ c - 1 / 2,
        b @ c ** 2 - 1 / 3, b @ ac - 1 / 6,
        b @ c ** 3 - 1 / 4, b @ (c * ac) - 1 / 8, b @ ac2 - 1 / 12, b @ aac - 1 / 24,
        b @ c ** 4 - 1 / 5, b @ (c ** 2 * ac) - 1 / 10, b @ (c * ac2) - 1 / 15, b @ (c * aac) - 1 / 30,
        b @ (ac * ac) - 1 / 20, b @ ac3 - 1 / 20, b @ (a @ (c * ac)) - 1 / 40, b @ (a @ ac2) - 1 / 60,
        b @ (a @ aac) - 1 / 120])


_LSRK59 = []


def lsrk59_tableau(iters=20):
    """(a, b, c) of LSRK5(9): Newton on the 17 conditions from the key
    (derivatives by complex steps, exact for these polynomials)."""
    if _LSRK59:
        return _LSRK59[0]
    # residuals in extended precision (the root is conditioned ~1e3, so a
    # double residual would leave ~1e-13 in the coefficients), Jacobian in
    # double: the iteration converges to the root to double precision
    x = np.array(LSRK59_KEY_ALPHA + LSRK59_KEY_B, dtype=np.longdouble)

    def res(v):
        return order5_conditions(*tableau_2r(v[:8], v[8:])[:2])
    for _ in range(iters):
        r = res(x)
        if np.max(np.abs(r)) < 1e-18:
            break
        J = np.empty((17, 17))
        for j in range(17):
            e = x.astype(np.float64).astype(np.complex128)
            e[j] += 1e-30j
            J[:, j] = res(e).imag / 1e-30
        x = x - np.linalg.solve(J, r.astype(np.float64)).astype(np.longdouble)
    a, b, c = tableau_2r(x[:8], x[8:])
    _LSRK59.append((a.astype(np.float64), b.astype(np.float64), c.astype(np.float64)))
    return _LSRK59[0]


def rk_step(rhs, U, t, dt, a, b, c):
    """One explicit Runge-Kutta step of Butcher tableau (a, b, c) (Sec. 2.2):
    k_i = rhs(U + dt sum_{j<i} a_ij k_j, t + c_i dt), U + dt sum_i b_i k_i."""
    u = np.asarray(U, dtype=np.float64)
    k = []
    for i in range(len(b)):
        y = u.copy()
        for j in range(i):
            if a[i][j] != 0.0:
                y = y + dt * float(a[i][j]) * k[j]
        k.append(rhs(y, t + float(c[i]) * dt))
    out = u.copy()
    for i in range(len(b)):
        out = out + dt * float(b[i]) * k[i]
    return out


def lsrk59_step(rhs, U, t, dt):
    """One LSRK5(9) step (see the module docstring)."""
    return rk_step(rhs, U, t, dt, *lsrk59_tableau())


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
