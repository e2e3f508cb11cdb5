"""Pins of the oracle's time integrators: LSRK(5,4) order conditions and
stability polynomial in exact rationals, temporal order 4 against the matrix
exponential (Sec. 2.2); the ADER Taylor-Cauchy-Kowalevski sum against the
closed-form time derivatives of polynomial states, with and without the
degree reduction (Sec. 2.3, 3.2, 3.3, Alg. 2-3); ADER order k+1 in space and
time jointly (Sec. 4.6); Courant number (Sec. 2.3) on the uniform box."""
import math
from fractions import Fraction

import numpy as np
import pytest
from numpy.polynomial import polynomial as P
from scipy.linalg import expm

import workloads as W
from oracle import Mesh, apply_operator, ader, basis, norms
from oracle import timestep as ts


def test_lsrk_order_conditions_exact():
    a, b, c = ts.lsrk_butcher()
    s = len(b)
    A = [[a[i][j] for j in range(s)] for i in range(s)]

    def Ac(v):
        return [sum(A[i][j] * v[j] for j in range(s)) for i in range(s)]

    dot = lambda u, v: sum(x * y for x, y in zip(u, v))
    cc = [x * x for x in c]
    conds = [
        (sum(b), Fraction(1)),
        (dot(b, c), Fraction(1, 2)),
        (dot(b, cc), Fraction(1, 3)),
        (dot(b, Ac(c)), Fraction(1, 6)),
        (dot(b, [x ** 3 for x in c]), Fraction(1, 4)),
        (dot(b, [ci * y for ci, y in zip(c, Ac(c))]), Fraction(1, 8)),
        (dot(b, Ac(cc)), Fraction(1, 12)),
        (dot(b, Ac(Ac(c))), Fraction(1, 24)),
    ]
    for got, want in conds:
        assert abs(float(got - want)) < 1e-20
    for ci, want in zip(c, ts.LSRK54_C):
        assert abs(float(ci - want)) < 1e-20


def test_lsrk_stability_polynomial():
    """R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 + gamma_5 z^5, gamma_5 * 5! = 0.6."""
    a, b, c = ts.lsrk_butcher()
    s = len(b)
    v = [Fraction(1)] * s
    gam = []
    for j in range(1, s + 1):
        gam.append(sum(bi * vi for bi, vi in zip(b, v)))
        v = [sum(a[i][l] * v[l] for l in range(s)) for i in range(s)]
    want = [Fraction(1, math.factorial(j)) for j in range(1, 5)]
    for g, w in zip(gam[:4], want):
        assert abs(float(g - w)) < 1e-20
    assert abs(float(gam[4]) * 120 - 0.6) < 1e-6


def test_lsrk_temporal_order_four():
    m = Mesh(2, 2, W.box_nodes(2, 2, 2, 0.05), W.box_neighbors(2, 2), W.FourierMaterial(2, dim=2))
    N = m.nc * 3 * m.np_
    L = np.column_stack([apply_operator(m, e.reshape(m.nc, 3, m.np_)).ravel() for e in np.eye(N)])
    u0 = W.random_state(1, N)
    T = 0.02
    exact = expm(T * L) @ u0
    errs = []
    for ns in (2, 4, 8):
        u = u0.reshape(m.nc, 3, m.np_)
        for s in range(ns):
            u = ts.lsrk_step(lambda x, t: (L @ x.ravel()).reshape(x.shape), u, s * T / ns, T / ns)
        errs.append(np.linalg.norm(u.ravel() - exact))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.8)


def _poly_state(dim, k, rng):
    """Random total-degree-k polynomial coefficient arrays for (v_1..v_d, p)."""
    out = []
    for _ in range(dim + 1):
        cf = np.zeros((k + 1,) * dim)
        for idx in np.ndindex(*cf.shape):
            if sum(idx) <= k:
                cf[idx] = rng.standard_normal()
        out.append(cf)
    return out


def _polyval(cf, x):
    return P.polyval2d(x[..., 0], x[..., 1], cf) if cf.ndim == 2 else P.polyval3d(x[..., 0], x[..., 1], x[..., 2], cf)


def _minus_S(state, dim, rho, c):
    """-S u for constant rho, c on polynomial coefficient arrays."""
    p = state[dim]
    v = [-P.polyder(p, axis=a) / rho for a in range(dim)]
    div = sum(_pad(P.polyder(state[a], axis=a), p.shape) for a in range(dim))
    return [_pad(x, p.shape) for x in v] + [-rho * c * c * div]


def _pad(cf, shape):
    out = np.zeros(shape)
    out[tuple(slice(0, s) for s in cf.shape)] = cf
    return out


@pytest.mark.parametrize("dim,k,reduce,period", [(2, 3, True, 2), (2, 4, True, 2), (2, 4, False, 2), (3, 2, True, 2),
                                                (3, 3, False, 2), (2, 4, True, 1), (3, 3, True, 1), (2, 5, True, 3),
                                                (3, 4, True, 3)])
def test_tck_exact_on_polynomials(dim, k, reduce, period):
    """Affine cells, constant rho, c: for a total-degree-k polynomial state the
    m-th derivative has total degree k-m, so neither the collocated evaluation
    nor the projections lose anything and I must equal the exact Taylor
    integral sum_m dt^{m+1}/(m+1)! (-S)^m u."""
    rho, c = 1.3, 0.7
    m = Mesh(dim, k, W.box_nodes(dim, 2, k, 0.0), W.box_neighbors(dim, 2), W.ConstantMaterial(rho, c))
    rng = np.random.default_rng(4)
    st = _poly_state(dim, k, rng)
    xn = m.node_points()
    U = np.stack([_polyval(cf, xn) for cf in st], axis=1)
    dt = 0.37
    I = ader.tck(m, U, dt, reduce=reduce, period=period)
    want = np.zeros_like(U)
    cur = st
    for j in range(k + 2):
        want += dt ** (j + 1) / math.factorial(j + 1) * np.stack([_polyval(cf, xn) for cf in cur], axis=1)
        cur = _minus_S(cur, dim, rho, c)
    assert np.max(np.abs(I - want)) < 1e-12 * np.max(np.abs(want))


def test_tck_reduction_changes_general_states():
    """With a full Q_k state the reduction is a real approximation (the two
    variants must differ) -- guards against the reduction silently not running."""
    m = Mesh(2, 4, W.box_nodes(2, 2, 4, 0.05), W.box_neighbors(2, 2), W.FourierMaterial(1, dim=2))
    U = W.random_state(2, (m.nc, 3, m.np_))
    a = ader.tck(m, U, 0.05, reduce=True)
    b = ader.tck(m, U, 0.05, reduce=False)
    assert norms.rel_l2(a, b) > 1e-8
    for period in (1, 3):
        c = ader.tck(m, U, 0.05, reduce=True, period=period)
        assert norms.rel_l2(c, a) > 1e-8 and norms.rel_l2(c, b) > 1e-8


def test_ader_levels():
    assert ader.levels(5) == [6, 6, 4, 4, 2, 2, 0]
    assert ader.levels(4) == [5, 5, 3, 3, 1, 1]
    assert ader.levels(7) == [8, 8, 6, 6, 4, 4, 2, 2, 0]
    assert ader.levels(3, reduce=False) == [4] * 5
    assert ader.levels(5, period=1) == [6, 5, 4, 3, 2, 1, 0]
    assert ader.levels(5, period=3) == [6, 6, 6, 3, 3, 3, 0]
    assert ader.levels(7, period=3) == [8, 8, 8, 5, 5, 5, 2, 2, 2]


@pytest.mark.parametrize("drop", [1, 2, 3])
def test_projection_is_legendre_truncation(drop):
    """P_{n->n-drop} keeps Legendre modes below n-drop and removes the highest ones (2D)."""
    n = 6
    xs = basis.gauss(n)[0]
    xr = basis.gauss(n - drop)[0]
    from numpy.polynomial import legendre as Lg
    rng = np.random.default_rng(0)
    coef = rng.standard_normal((n, n))
    f = Lg.legval2d(2 * basis.tensor_points(xs, 2)[:, 0] - 1, 2 * basis.tensor_points(xs, 2)[:, 1] - 1, coef)
    tr = coef.copy()
    tr[n - drop:, :] = 0
    tr[:, n - drop:] = 0
    g = Lg.legval2d(2 * basis.tensor_points(xr, 2)[:, 0] - 1, 2 * basis.tensor_points(xr, 2)[:, 1] - 1, tr)
    got = ader.projection_table(n, 2, drop) @ f
    assert np.allclose(got, g, atol=1e-12)


@pytest.mark.parametrize("k,period", [(2, 2), (3, 2), (3, 1), (3, 3)])
def test_ader_joint_convergence(k, period):
    errs = []
    for nc in (4, 8):
        m = Mesh(2, k, W.box_nodes(2, nc, k, 0.0), W.box_neighbors(2, nc), W.ConstantMaterial())
        U = m.interpolate(lambda x: W.standing_wave_2d(x, 0.0))
        dt, ns = ts.dt_from_courant(m, 0.1, 0.2)
        for s in range(ns):
            U = ader.ader_step(m, U, dt, period=period)
        errs.append(norms.l2_error(m, U, W.standing_wave_2d, 0.2)[0])
    assert np.log2(errs[0] / errs[1]) > k + 1 - 0.3


def test_courant_dt_of_first_workload():
    """2D 8x8 affine box, k = 3, Cr = 0.2: dt = 0.2 (1/8) / 3^1.5."""
    m = Mesh(2, 3, W.box_nodes(2, 8, 3, 0.0), W.box_neighbors(2, 8), W.ConstantMaterial())
    dt, _ = ts.dt_from_courant(m, 0.2)
    assert abs(dt - 0.2 / 8 / 3 ** 1.5) < 1e-16
    assert abs(dt - 4.811252243246881e-3) < 1e-15
