"""Pin of the oracle's point-source injection against the closed form.

Reading (the paper has no sources): d/dt p + rho c^2 div v = s(t) delta(x - x_s),
rho d/dt v + grad p = 0, so p solves p_tt - c^2 lap p = s'(t) delta(x - x_s).
In 2D its retarded solution is

    p(x, t) = 1/(2 pi c^2) int_{-inf}^{t - r/c} s'(tau) / sqrt((t - tau)^2 - r^2/c^2) dtau
            = 1/(2 pi c^2) int_0^inf s'(t - (r/c) cosh u) du          (tau = t - (r/c) cosh u),

summed here over the periodic images of the source (2D waves have tails, so
the images matter at the 1e-3 level).  Homogeneous rho = 1.5, c = 1.2 (a
missing 1/(rho c^2) in the injection is off by a factor 2.16), Ricker
wavelet, source at a cell centre; the pressure at T in the shell
0.15 < r < 0.42 around the source converges to it at order k+1 for LSRK
(source at the stage times) and ADER (source derivatives in the
Cauchy-Kowalevski recursion, exact integral in the update)."""
import numpy as np
import pytest

import workloads as W
from oracle import Mesh, apply_operator, ader, basis, sources as osrc, timestep as ts

RHO, C = 1.5, 1.2


class _Homogeneous:
    def __call__(self, x):
        x = np.asarray(x)
        return np.full(x.shape[:-1], RHO), np.full(x.shape[:-1], C)


def _ricker_dt(f, t0, t):
    """d/dt of (1 - 2 a tau^2) exp(-a tau^2), a = (pi f)^2, tau = t - t0."""
    a = (np.pi * f) ** 2
    tau = t - t0
    return -2 * a * tau * (3 - 2 * a * tau ** 2) * np.exp(-a * tau ** 2)


def _exact_2d(f, t0, r, t):
    u, w = np.polynomial.legendre.leggauss(400)
    umax = 8.0  # cosh(8) r / c far exceeds the wavelet's support
    uu = 0.5 * umax * (u + 1)
    vals = _ricker_dt(f, t0, t - (r[..., None] / C) * np.cosh(uu))
    return (vals * (0.5 * umax * w)).sum(-1) / (2 * np.pi * C * C)


def _shell_error(nc, k, scheme, f=3.0):
    m = Mesh(2, k, W.box_nodes(2, nc, k, 0.0), W.box_neighbors(2, nc), _Homogeneous())
    xs = np.full(2, (nc // 2 + 0.5) / nc)
    wavelet = osrc.Ricker(f=f)
    T = wavelet.t0 + 0.3 / C
    ps = osrc.PointSource(m, xs, wavelet)
    cr = 0.3 if scheme == "lsrk" else 0.15
    n = int(np.ceil(T / (cr / nc / C / k ** 1.5)))
    dt = T / n
    U = np.zeros((m.nc, 3, m.np_))
    for s in range(n):
        if scheme == "lsrk":
            U = ts.lsrk_step(lambda u, t: apply_operator(m, u) + ps.rhs(m, t), U, s * dt, dt)
        else:
            U = ader.ader_step(m, U, dt, source=ps, t=s * dt)
    cd = m.cell_data(np.arange(m.nc))
    pq = np.einsum("qi,ci->cq", basis.tensor_basis(m.xgl, m.cell_ref), U[:, 2])
    x = cd["x"]
    r = np.linalg.norm(x - xs, axis=-1)
    sel = (r > 0.15) & (r < 0.42)
    ex = np.zeros(sel.sum())
    for i in range(-2, 3):
        for j in range(-2, 3):
            ex += _exact_2d(f, wavelet.t0, np.linalg.norm(x[sel] - xs - np.array([i, j]), axis=-1), T)
    w = cd["wdet"][sel]
    return np.sqrt(np.sum(w * (pq[sel] - ex) ** 2) / np.sum(w * ex ** 2))


@pytest.mark.parametrize("scheme", ["lsrk", "ader"])
def test_point_source_converges_to_retarded_solution(scheme):
    k = 3
    e12, e16 = _shell_error(12, k, scheme), _shell_error(16, k, scheme)
    assert e12 < 6e-3 and e16 < 2e-3
    assert e12 / e16 > (16 / 12) ** (k + 1) * 0.7
