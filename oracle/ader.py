"""ADER time stepping with the Taylor-Cauchy-Kowalevski (TCK) sum (oracle).

Paper, Sec. 2.3 (eq. ader-U and eq. ader): u_{n+1} = u_n - M^-1 K M^-1
sum_{j=0}^{k+1} dt^{j+1}/(j+1)! (-1)^j int N^T S^j N u_n, i.e.
u_{n+1} = u_n + L_h(I) with I the time integral of the local Taylor
expansion.  Sec. 3.2 (flexible basis change, Alg. 2) evaluates the j-th
derivatives by repeated first derivatives at Gauss points; Sec. 3.3
(degree reduction, Alg. 3) projects every second derivative to a degree two
lower on the reference element.

Reading of Alg. 3 (its loop index and the text's degree formula disagree):
the m-th time derivative ut^m lives at n_m Gauss points per direction with
n_0 = k+1, n_m = n_{m-1} - 2 when m is even and n_m = n_{m-1} when m is odd,
so that deg ut^m = k - 2 floor(m/2).  For m = 1..k+1:

    w      = -S_loc ut^{m-1}                  (at the n_{m-1} Gauss points)
    ut^m   = P_{n -> n-2} w  if m even,  else w
    I     += dt^{m+1}/(m+1)! * E_{n_m -> k+1} ut^m,     I starts at dt ut^0,

with S_loc u = ((1/rho) grad p, rho c^2 div v) evaluated pointwise from the
level's Lagrange interpolant and the Jacobian at the level's points, P the
L2 projection on the reference cell and E the evaluation of the level
interpolant at the k+1 Gauss points.  A projection to fewer than one point
per direction (and every later term) is zero.  With `reduce=False`
(Alg. 2 only) every level has k+1 points and nothing is projected.

Reduction period (the ablation of Sec. 3.3): the text first describes a
projection P_{k-i+1}^{k-i} after every derivative and then proposes every
second one (Alg. 3).  With period R the derivative m is projected by R
points when m is a multiple of R, so deg ut^m = k - R floor(m/R): R = 1 is
the every-step variant (deg k - m), R = 2 Alg. 3, R = 3 every third.

Everything is built from dense d-dimensional tables evaluated directly.
"""
from __future__ import annotations

import math

import numpy as np

from . import basis
from .operator import apply_operator, tables


def levels(k, reduce=True, period=2):
    """Points per direction n_m of the time derivatives m = 0..k+1 (0 = vanished)."""
    out = [k + 1]
    for m in range(1, k + 2):
        n = out[-1]
        if reduce and m % period == 0:
            n = n - period
        out.append(max(n, 0))
    return out


def projection_table(n, d, drop=2):
    """Dense L2 projection (reference cell, unit weight) from Q_{n-1} (values at the
    n^d Gauss points) onto Q_{n-1-drop} (values at the (n-drop)^d Gauss points):
    solve the normal equations with mass matrix int l_a l_b and right-hand side
    int l_a l_j, both by an over-integrating Gauss rule."""
    xs, _ = basis.gauss(n)
    xr, _ = basis.gauss(n - drop)
    xo, wo = basis.gauss(n + 2)
    pts = basis.tensor_points(xo, d)
    w = basis.tensor_weights(wo, d)
    lr = basis.tensor_basis(xr, pts)          # [Qo][(n-2)^d]
    ls = basis.tensor_basis(xs, pts)          # [Qo][n^d]
    M = lr.T @ (w[:, None] * lr)
    Bm = lr.T @ (w[:, None] * ls)
    return np.linalg.solve(M, Bm)


class AderTables:
    def __init__(self, mesh, reduce=True, period=2):
        d, k = mesh.dim, mesh.k
        self.levels = levels(k, reduce, period)
        self.reduce = reduce
        self.period = period
        self.pts = {}
        self.D = {}
        self.E = {}
        self.from_gl = {}
        for n in sorted(set(l for l in self.levels if l > 0)):
            x, _ = basis.gauss(n)
            p = basis.tensor_points(x, d)
            self.pts[n] = p
            self.D[n] = basis.tensor_basis_grad(x, p) if n > 1 else [np.zeros((1, 1))] * d
            self.E[n] = basis.tensor_basis(x, mesh.cell_ref)          # level n -> k+1 Gauss points
            self.from_gl[n] = basis.tensor_basis(mesh.xgl, p)           # GL coefficients -> level points
        self.P = {n: projection_table(n, d, period) for n in self.pts if n - period >= 1}


def ader_tables(mesh, reduce=True, period=2):
    key = ("ader", reduce, period)
    t = mesh._cache.get(key)
    if t is None:
        t = AderTables(mesh, reduce, period)
        mesh._cache[key] = t
    return t


def level_data(mesh, cells, n):
    """J^-1, rho and c at the n^d Gauss points of each cell (the level's own points)."""
    key = ("level", n)
    full = mesh._cache.get(key)
    if full is not None:
        return {kk: v[cells] for kk, v in full.items()}
    T = ader_tables(mesh)
    pts = T.pts[n] if n in T.pts else basis.tensor_points(basis.gauss(n)[0], mesh.dim)

    def compute(cs):
        x, J = mesh.map_points(cs, pts)
        rho, c = mesh.material(x)
        return dict(Jinv=np.linalg.inv(J), rho=np.asarray(rho, float), c=np.asarray(c, float))

    if mesh._cacheable():
        full = compute(np.arange(mesh.nc))
        mesh._cache[key] = full
        return {kk: v[cells] for kk, v in full.items()}
    return compute(cells)


def minus_s_local(mesh, cells, ut, n, T):
    """-S_loc ut at the level's n^d Gauss points: collocation derivatives of
    the level-n Lagrange interpolant, J^-1, rho and c at those points."""
    d = mesh.dim
    ld = level_data(mesh, cells, n)
    Jinv = ld["Jinv"]                                    # [C][Q][b][a]
    grads = [np.einsum("qj,cvj->cvq", T.D[n][b], ut) for b in range(d)]  # d/dxi_b of each comp
    w = np.empty_like(ut)
    for a in range(d):
        w[:, a] = -(1.0 / ld["rho"]) * sum(Jinv[:, :, b, a] * grads[b][:, d] for b in range(d))
    div = sum(Jinv[:, :, b, a] * grads[b][:, a] for a in range(d) for b in range(d))
    w[:, d] = -ld["rho"] * ld["c"] ** 2 * div
    return w


def tck(mesh, U, dt, cells=None, reduce=True, source_terms=None, period=2):
    """Time-integrated Taylor sum I (GL coefficients, float64[C][d+1][np]).

    source_terms: optional callable (cells, m, n) -> additive p-values at the
    level-n points of the (m-1)-th recursion step, float64[C][n^d] (the
    point-source injection); None for no source.  period: the reduction
    period (module docstring).
    """
    d, k = mesh.dim, mesh.k
    T = ader_tables(mesh, reduce, period)
    Tb = tables(mesh)
    cells = np.arange(mesh.nc) if cells is None else np.atleast_1d(np.asarray(cells, dtype=np.int64))
    ut = np.einsum("qi,cvi->cvq", Tb.phi, np.asarray(U)[cells])   # ut^0 at the k+1 Gauss points
    I = dt * ut.copy()
    lev = T.levels
    for m in range(1, k + 2):
        n = lev[m - 1]
        if n <= 0:
            break
        w = minus_s_local(mesh, cells, ut, n, T)
        if source_terms is not None:
            w[:, d] += source_terms(cells, m, n)
        if reduce and m % period == 0:
            if n - period < 1:
                break
            ut = np.einsum("rq,cvq->cvr", T.P[n], w)
        else:
            ut = w
        nm = lev[m]
        I += dt ** (m + 1) / math.factorial(m + 1) * np.einsum("pq,cvq->cvp", T.E[nm], ut)
    # GL coefficients of the Gauss-point values (dense solve with the GL table)
    Ig = np.linalg.solve(Tb.phi[None, :, :], np.swapaxes(I, -1, -2))
    return np.ascontiguousarray(np.swapaxes(Ig, -1, -2))


def ader_step(mesh, U, dt, flux="upwind", reduce=True, source=None, t=0.0, period=2, exterior_integral=None):
    """One ADER step u + L_h(I) (+ the exact time integral of the source).
    Prescribed boundary faces take exterior_integral(x), the time integral of
    the exterior state over [t, t + dt], as the exterior state of I."""
    st = None if source is None else source.tck_terms(mesh, t)
    I = tck(mesh, U, dt, reduce=reduce, source_terms=st, period=period)
    out = np.asarray(U, dtype=np.float64) + apply_operator(mesh, I, flux=flux, exterior=exterior_integral)
    if source is not None:
        out = out + source.integral(t, t + dt) * source.vector_full(mesh)
    return out


def hdg_tck(mesh, U, W, dt, cells=None, reduce=True):
    """Time-integrated sum of the HDG-ADER variant (Sec. 2.4, eq. hdg-ader),
    GL coefficients float64[C][d+1][np]:

        I = dt U + sum_{j=1}^{k+1} dt^{j+1}/(j+1)! (-S)^(j-1) W,   W = L_h U,

    i.e. the first element-local derivative of the TCK sum is replaced by the
    DG derivative W (faces included); the later ones are element-local as in
    tck, with the degree of the j-th derivative k - 2 floor(j/2) (W is the
    first derivative and keeps the k+1 points)."""
    d, k = mesh.dim, mesh.k
    T = ader_tables(mesh, reduce)
    Tb = tables(mesh)
    cells = np.arange(mesh.nc) if cells is None else np.atleast_1d(np.asarray(cells, dtype=np.int64))
    u0 = np.einsum("qi,cvi->cvq", Tb.phi, np.asarray(U)[cells])
    ut = np.einsum("qi,cvi->cvq", Tb.phi, np.asarray(W)[cells])   # derivative order 1
    lev = T.levels
    I = dt * u0 + dt ** 2 / 2.0 * np.einsum("pq,cvq->cvp", T.E[lev[1]], ut)
    for m in range(2, k + 2):
        n = lev[m - 1]
        if n <= 0:
            break
        w = minus_s_local(mesh, cells, ut, n, T)
        if reduce and m % 2 == 0:
            if n - 2 < 1:
                break
            ut = np.einsum("rq,cvq->cvr", T.P[n], w)
        else:
            ut = w
        I += dt ** (m + 1) / math.factorial(m + 1) * np.einsum("pq,cvq->cvp", T.E[lev[m]], ut)
    Ig = np.linalg.solve(Tb.phi[None, :, :], np.swapaxes(I, -1, -2))
    return np.ascontiguousarray(np.swapaxes(Ig, -1, -2))


def hdg_ader_step(mesh, U, dt, flux="upwind", reduce=True):
    """One HDG-ADER step (Sec. 2.4, eq. hdg-ader): two applications of the DG
    operator, u + L_h(hdg_tck(u, L_h u))."""
    U = np.asarray(U, dtype=np.float64)
    W = apply_operator(mesh, U, flux=flux)
    return U + apply_operator(mesh, hdg_tck(mesh, U, W, dt, reduce=reduce), flux=flux)
