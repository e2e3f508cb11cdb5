"""Point sources with a Ricker wavelet (oracle).

Not part of the paper (its experiments have no sources); the reading used
for batched-source workloads:

* strong form  d/dt p + rho c^2 div v = s(t) delta(x - x_s); in the weighted
  weak form of oracle/operator.py the p right-hand side gains
  s(t) phi(xi_s) / (rho(x_s) c(x_s)^2), so the semi-discrete source is
  s(t) g with g = M_p^-1 phi(xi_s) / (rho c^2), nonzero in one cell;
* x_s is located by Newton iteration on the cell maps; the lowest cell index
  whose closed reference cell contains the point wins;
* Ricker s(t) = amp (1 - 2 a tau^2) exp(-a tau^2), a = (pi f)^2, tau = t - t0;
  its l-th derivative is -amp/(2a) (-sqrt a)^(l+2) H_{l+2}(sqrt(a) tau) exp(-a tau^2)
  (physicists' Hermite H) and its antiderivative amp tau exp(-a tau^2);
* LSRK evaluates s at the stage times; ADER adds s^(m-1)(t) g (g evaluated
  at the level points) inside the Cauchy-Kowalevski recursion and the exact
  time integral of s times g to the update.

Pins: in a homogeneous periodic box the pressure converges at order k+1 to
the retarded solution of p_tt - c^2 lap p = s'(t) delta(x - x_s) (2D, with
the periodic images), for LSRK and ADER; the Ricker closed forms against
finite differences and quadrature; linearity/superposition.  On curved
meshes with variable coefficients no closed form exists; the same code
path serves them.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import hermite as H

from . import basis
from .operator import cholesky_factors, _chol_apply


def locate(mesh, xs, tol=1e-12, iters=50):
    """(cell, xi) with x_cell(xi) = xs; lowest cell index wins."""
    xs = np.asarray(xs, dtype=np.float64)
    for cell in range(mesh.nc):
        xi = np.full(mesh.dim, 0.5)
        ok = False
        for _ in range(iters):
            x, J = mesh.map_points([cell], xi[None, :])
            r = x[0, 0] - xs
            if np.max(np.abs(r)) < tol:
                ok = True
                break
            xi = xi - np.linalg.solve(J[0, 0], r)
            if np.any(np.abs(xi - 0.5) > 2.0):
                break
        if ok and np.all(xi >= -1e-10) and np.all(xi <= 1 + 1e-10):
            return cell, np.clip(xi, 0.0, 1.0)
    raise ValueError("source point not inside the mesh")


class Ricker:
    def __init__(self, f=8.0, t0=None, amp=1.0):
        self.f = float(f)
        self.t0 = 1.2 / self.f if t0 is None else float(t0)
        self.amp = float(amp)
        self.a = (math.pi * self.f) ** 2

    def deriv(self, t, l=0):
        """l-th time derivative of s at t (l = 0 is s itself)."""
        tau = t - self.t0
        sa = math.sqrt(self.a)
        c = np.zeros(l + 3)
        c[l + 2] = 1.0
        return -self.amp / (2 * self.a) * (-sa) ** (l + 2) * H.hermval(sa * tau, c) * math.exp(-self.a * tau * tau)

    def __call__(self, t):
        return self.deriv(t, 0)

    def integral(self, t1, t2):
        F = lambda t: self.amp * (t - self.t0) * math.exp(-self.a * (t - self.t0) ** 2)
        return F(t2) - F(t1)


class PointSource:
    """One point source s(t) delta(x - x_s) acting on the pressure equation."""

    def __init__(self, mesh, xs, wavelet):
        self.cell, self.xi = locate(mesh, xs)
        self.wavelet = wavelet
        d = mesh.dim
        x, _ = mesh.map_points([self.cell], self.xi[None, :])
        rho, c = mesh.material(x)
        phi = basis.tensor_basis(mesh.xgl, self.xi[None, :])[0]        # GL basis at xi_s
        rhs = phi / (float(np.ravel(rho)[0]) * float(np.ravel(c)[0]) ** 2)
        _, Lp = cholesky_factors(mesh, [self.cell])
        self.g = _chol_apply(Lp, rhs[None, None, :])[0, 0]              # GL coefficients, p comp
        self.dim = d

    def vector_full(self, mesh):
        out = np.zeros((mesh.nc, mesh.dim + 1, mesh.np_))
        out[self.cell, mesh.dim] = self.g
        return out

    def rhs(self, mesh, t):
        return self.wavelet(t) * self.vector_full(mesh)

    def integral(self, t1, t2):
        return self.wavelet.integral(t1, t2)

    def tck_terms(self, mesh, t):
        """Callable for oracle.ader.tck: s^(m-1)(t) g at the level-n points."""
        def fn(cells, m, n):
            from .ader import ader_tables
            T = ader_tables(mesh)
            out = np.zeros((len(cells), n ** mesh.dim))
            hit = np.nonzero(np.asarray(cells) == self.cell)[0]
            if len(hit):
                pts = T.pts[n] if n in T.pts else basis.tensor_points(basis.gauss(n)[0], mesh.dim)
                gv = basis.tensor_basis(mesh.xgl, pts) @ self.g
                out[hit] = self.wavelet.deriv(t, m - 1) * gv
            return out
        return fn
