"""Pins of the oracle's 1D rules, Lagrange tables and basis-change identities
against textbook facts (Sec. 3 of the paper: Gauss rule on k+1 points,
G and GL Lagrange bases, inverse mass via the basis change of Sec. 3.1)."""
import numpy as np
import pytest
from scipy.special import roots_jacobi

from oracle import basis


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_exactness(n):
    x, w = basis.gauss(n)
    assert np.all(np.diff(x) > 0) and abs(w.sum() - 1) < 1e-14
    for m in range(2 * n):
        assert abs(np.dot(w, x ** m) - 1.0 / (m + 1)) < 1e-14
    # not exact one degree higher (a wrong rule of higher order would pass above)
    assert abs(np.dot(w, x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12


@pytest.mark.parametrize("n", range(2, 10))
def test_gauss_lobatto(n):
    x, w = basis.gauss_lobatto(n)
    assert x[0] == 0.0 and x[-1] == 1.0 and abs(w.sum() - 1) < 1e-14
    if n > 2:
        # interior GL points are the roots of the Jacobi polynomial P^(1,1)_{n-2}
        r, _ = roots_jacobi(n - 2, 1, 1)
        assert np.max(np.abs(x[1:-1] - 0.5 * (np.sort(r) + 1))) < 1e-14
    for m in range(2 * n - 2):
        assert abs(np.dot(w, x ** m) - 1.0 / (m + 1)) < 1e-14
    assert abs(np.dot(w, x ** (2 * n - 2)) - 1.0 / (2 * n - 1)) > 1e-12


@pytest.mark.parametrize("n", [1, 2, 4, 7, 9])
def test_lagrange_tables(n):
    nodes = basis.gauss_lobatto(n)[0] if n > 1 else np.array([0.5])
    assert np.allclose(basis.lagrange(nodes, nodes), np.eye(n), atol=1e-14)
    xs = np.linspace(-0.1, 1.1, 13)
    L = basis.lagrange(nodes, xs)
    dL = basis.lagrange_deriv(nodes, xs)
    for m in range(n):
        f = nodes ** m
        assert np.allclose(L @ f, xs ** m, atol=1e-12)
        df = m * xs ** (m - 1) if m > 0 else np.zeros_like(xs)
        assert np.allclose(dL @ f, df, atol=1e-10)


def test_tensor_basis_partition_and_gradient():
    nodes = basis.gauss_lobatto(4)[0]
    pts = np.random.default_rng(0).uniform(size=(20, 3))
    phi = basis.tensor_basis(nodes, pts)
    assert np.allclose(phi.sum(axis=1), 1.0, atol=1e-13)
    for g in basis.tensor_basis_grad(nodes, pts):
        assert np.allclose(g.sum(axis=1), 0.0, atol=1e-12)
    # x*y^2*z reproduced with its gradient
    grid = basis.tensor_points(nodes, 3)
    f = grid[:, 0] * grid[:, 1] ** 2 * grid[:, 2]
    assert np.allclose(phi @ f, pts[:, 0] * pts[:, 1] ** 2 * pts[:, 2], atol=1e-13)
    gy = basis.tensor_basis_grad(nodes, pts)[1] @ f
    assert np.allclose(gy, 2 * pts[:, 0] * pts[:, 1] * pts[:, 2], atol=1e-12)


def test_multi_index_is_x_fastest():
    mi = basis.multi_indices(3, 3)
    assert list(mi[1]) == [1, 0, 0] and list(mi[3]) == [0, 1, 0] and list(mi[9]) == [0, 0, 1]


@pytest.mark.parametrize("n", [2, 5, 8])
def test_interpolation_gl_to_g_and_back(n):
    """u_G = u_GL (Sec. 3.2): the G interpolant of the G-point values of a GL
    polynomial is the same polynomial, so S^-1[j, q] = l^G_q(xi^GL_j)."""
    xg = basis.gauss(n)[0]
    xgl = basis.gauss_lobatto(n)[0]
    S = basis.lagrange(xgl, xg)
    Sinv = basis.lagrange(xg, xgl)
    assert np.allclose(S @ Sinv, np.eye(n), atol=1e-12)
    assert np.allclose(Sinv @ S, np.eye(n), atol=1e-12)
