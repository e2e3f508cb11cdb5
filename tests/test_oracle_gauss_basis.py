"""Pins of the oracle's Gauss (collocated) storage basis, Sec. 3.1.

The oracle evaluates the weak form directly with Lagrange polynomials in
the Gauss points (oracle/operator.py, storage="gauss").  Pins independent of
that code path: the mass matrix is diagonal with the quadrature weights
(the property Sec. 3.1 names), the GL -> Gauss map reproduces polynomials
exactly at the reference Gauss points, and, since both bases span the same
space under the same quadrature, the Gauss-basis operator equals
S L_GL S^-1 built from the pinned GL operator.  A transposed S, a wrong node
order or a GL table left in the neighbour trace fails one of them."""
import numpy as np
import pytest

import workloads as W
from oracle import Mesh, apply_operator, basis, norms
from oracle.operator import gl_to_gauss, mass_matrices, tables
from oracle import timestep as ts


def _mesh(dim, nc, k, bc=None, orient=False):
    mat = W.FourierMaterial(19, dim=dim)
    if orient:
        nodes, nb, fo, _ = W.rotated_box(dim, nc, k, 0.05, seed=23)
        return Mesh(dim, k, nodes, nb, mat, face_orient=fo)
    return Mesh(dim, k, W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc, bc), mat)


@pytest.mark.parametrize("dim,k", [(2, 3), (3, 2)])
def test_gauss_mass_is_diagonal(dim, k):
    m = _mesh(dim, 2, k)
    cells = np.arange(m.nc)
    Mv, Mp = mass_matrices(m, cells, "gauss")
    cd = m.cell_data(cells)
    for M, w in ((Mv, cd["wdet"] * cd["rho"]), (Mp, cd["wdet"] / (cd["rho"] * cd["c"] ** 2))):
        assert np.abs(M - np.einsum("cq,qj->cqj", w, np.eye(m.np_))).max() < 1e-14 * w.max()
    # the GL mass is not diagonal: the two bases really differ
    Mgl, _ = mass_matrices(m, cells)
    assert np.abs(Mgl - np.einsum("cii->ci", Mgl)[:, :, None] * np.eye(m.np_)).max() > 1e-3 * np.abs(Mgl).max()


@pytest.mark.parametrize("dim,k", [(2, 4), (3, 3)])
def test_gl_to_gauss_reproduces_polynomials(dim, k):
    """A polynomial of degree k per direction, given by its values at the GL
    nodes, has at the Gauss points exactly its own values (lexicographic
    order, x fastest)."""
    m = _mesh(dim, 1, k)
    rng = np.random.default_rng(5)
    coef = rng.standard_normal((k + 1,) * dim)

    def f(xi):
        out = np.zeros(len(xi))
        for idx in np.ndindex(*coef.shape):
            out += coef[idx] * np.prod([xi[:, a] ** idx[a] for a in range(dim)], axis=0)
        return out

    gl_pts = basis.tensor_points(m.xgl, dim)
    U = np.zeros((1, dim + 1, m.np_))
    U[0, dim] = f(gl_pts)
    assert np.abs(gl_to_gauss(m, U)[0, dim] - f(m.cell_ref)).max() < 1e-12 * np.abs(coef).sum()


CASES = [(2, 3, 3, None, False, "upwind"), (2, 3, 2, ("wall", "absorbing"), False, "central"),
         (3, 2, 2, None, False, "upwind"), (3, 3, 2, None, True, "upwind"),
         (3, 2, 3, ("absorbing", "periodic", "wall"), False, "upwind")]


@pytest.mark.parametrize("dim,nc,k,bc,orient,flux", CASES)
def test_gauss_operator_is_basis_change_of_gl_operator(dim, nc, k, bc, orient, flux):
    m = _mesh(dim, nc, k, bc, orient)
    U = W.random_state(41 + k, (m.nc, dim + 1, m.np_))
    want = gl_to_gauss(m, apply_operator(m, U, flux=flux))
    got = apply_operator(m, gl_to_gauss(m, U), flux=flux, storage="gauss")
    assert norms.rel_l2(got, want) < 1e-11


def test_gauss_basis_constant_state_and_lsrk():
    """A constant state is steady on the periodic mesh; one LSRK step in the
    Gauss basis is the GL step mapped by S."""
    m = _mesh(3, 2, 3)
    U = np.zeros((m.nc, 4, m.np_))
    U[:, 3] = 1.0
    U[:, 0] = 0.5
    r = apply_operator(m, gl_to_gauss(m, U), storage="gauss")
    assert np.abs(r).max() < 1e-9
    U = W.random_state(3, (m.nc, 4, m.np_))
    dt = 1e-3
    want = gl_to_gauss(m, ts.lsrk_step(lambda x, t: apply_operator(m, x), U, 0.0, dt))
    got = ts.lsrk_step(lambda x, t: apply_operator(m, x, storage="gauss"), gl_to_gauss(m, U), 0.0, dt)
    assert norms.rel_l2(got, want) < 1e-12
    assert tables(m, "gauss").phi.shape == (m.np_, m.np_)
