"""Pins of the oracle's geometry and DG operator (Sec. 2.1 weak form, Sec. 2.4
upwind/HDG flux, Sec. 3.1 inverse mass) against facts that do not depend on
the oracle's own code: volume and closed-surface identities of the map,
free-stream preservation, the discrete energy identity, skew-symmetry /
dissipativity of the brute-force assembled operator, the inverse-mass basis
change formula and spatial convergence against closed-form waves."""
import numpy as np
import pytest

import workloads as W
from oracle import Mesh, apply_operator, basis, norms
from oracle import operator as op
from oracle import timestep as ts


def make(dim, nc, k, amp, mat=None, q=None):
    mat = mat or W.FourierMaterial(7, dim=dim)
    return Mesh(dim, k, W.box_nodes(dim, nc, q or k, amp), W.box_neighbors(dim, nc), mat)


def test_neighbor_table_is_an_involution():
    for dim, nc in [(2, 3), (3, 4)]:
        nb = W.box_neighbors(dim, nc)
        for e in range(nb.shape[0]):
            for f in range(2 * dim):
                assert nb[nb[e, f], f ^ 1] == e


def test_affine_geometry():
    m = make(3, 4, 2, 0.0, W.ConstantMaterial())
    cd = m.cell_data(np.arange(m.nc))
    assert np.allclose(cd["J"], np.eye(3) / 4, atol=1e-15)
    assert np.allclose(cd["detJ"], 1 / 64, atol=1e-15)


@pytest.mark.parametrize("dim,nc,k", [(2, 3, 3), (3, 2, 3)])
def test_curved_volume_and_closed_surface(dim, nc, k):
    m = make(dim, nc, k, 0.05)
    # total volume of the periodic box is 1 (over-integrated det J)
    xo, wo = basis.gauss(2 * k + 4)
    _, J = m.map_points(np.arange(m.nc), basis.tensor_points(xo, dim))
    vol = np.sum(np.linalg.det(J) * basis.tensor_weights(wo, dim))
    assert abs(vol - 1.0) < 1e-13
    # closed surface: sum of the face area vectors of each cell vanishes,
    # and neighbouring faces carry opposite area vectors (watertight map)
    tot = np.zeros((m.nc, dim))
    for f in range(2 * dim):
        fd = m.face_data(np.arange(m.nc), f)
        tot += fd["a"].sum(axis=1)
        fo = m.face_data(fd["nb"], f ^ 1)
        assert np.max(np.abs(fd["a"] + fo["a"])) < 1e-15
    assert np.max(np.abs(tot)) < 1e-15


def test_deformation_keeps_positive_jacobian():
    m = make(3, 6, 3, 0.05)
    cd = m.cell_data(np.arange(m.nc))
    # J = I/n + gradient of the displacement; det J * n^3 stays above 1 - 0.1 pi sqrt(3)
    assert cd["detJ"].min() * 216 > 1 - 0.1 * np.pi * np.sqrt(3)


@pytest.mark.parametrize("dim,nc,k,amp", [(2, 3, 3, 0.0), (2, 3, 3, 0.05), (3, 2, 2, 0.0), (3, 2, 3, 0.05)])
def test_constant_state_is_steady(dim, nc, k, amp):
    m = make(dim, nc, k, amp)
    U = np.zeros((m.nc, dim + 1, m.np_))
    U[:] = np.linspace(0.3, 1.4, dim + 1)[None, :, None]
    L = apply_operator(m, U)
    U2 = W.random_state(3, U.shape)
    scale = np.abs(apply_operator(m, U2)).max()
    assert np.abs(L).max() < 1e-12 * scale


def _energy_rate(m, U, L):
    d = m.dim
    Mv, Mp = op.mass_matrices(m, np.arange(m.nc))
    return (np.einsum("cai,cij,caj->", U[:, :d], Mv, L[:, :d])
            + np.einsum("ci,cij,cj->", U[:, d], Mp, L[:, d]))


def _jump_dissipation(m, U):
    """-sum over faces of (Z/2 [v_n]^2 + [p]^2 / (2 Z)), each face counted once."""
    d = m.dim
    tot = 0.0
    for f in range(1, 2 * d, 2):  # + faces only: every interior face once
        fd = m.face_data(np.arange(m.nc), f)
        phim = basis.tensor_basis(m.xgl, m.face_ref[f])
        phip = basis.tensor_basis(m.xgl, m.face_ref[f ^ 1])
        um = np.einsum("qi,cvi->cvq", phim, U)
        up = np.einsum("qi,cvi->cvq", phip, U[fd["nb"]])
        a = fd["a"]
        area = np.linalg.norm(a, axis=-1)
        nrm = a / area[..., None]
        jv = np.einsum("cqa,caq->cq", nrm, um[:, :d] - up[:, :d])
        jp = um[:, d] - up[:, d]
        Z = fd["Zm"]
        tot -= np.sum(area * (0.5 * Z * jv ** 2 + jp ** 2 / (2 * Z)))
    return tot


@pytest.mark.parametrize("dim,nc,k", [(2, 3, 3), (3, 2, 2)])
def test_energy_identity_affine_variable_material(dim, nc, k):
    m = make(dim, nc, k, 0.0, W.FourierMaterial(11, dim=dim))
    U = W.random_state(5, (m.nc, dim + 1, m.np_))
    scale = norms.energy_norm2(m, U) * np.abs(apply_operator(m, U)).max()
    e_c = _energy_rate(m, U, apply_operator(m, U, flux="central"))
    assert abs(e_c) < 1e-13 * scale
    e_u = _energy_rate(m, U, apply_operator(m, U, flux="upwind"))
    diss = _jump_dissipation(m, U)
    assert diss < 0 and abs(e_u - diss) < 1e-12 * abs(diss)


def _dense_operator(m, flux):
    N = m.nc * (m.dim + 1) * m.np_
    L = np.empty((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        L[:, j] = apply_operator(m, e.reshape(m.nc, m.dim + 1, m.np_), flux=flux).ravel()
    return L


def _mass_dense(m):
    d = m.dim
    Mv, Mp = op.mass_matrices(m, np.arange(m.nc))
    blocks = []
    for c in range(m.nc):
        blocks += [Mv[c]] * d + [Mp[c]]
    from scipy.linalg import block_diag
    return block_diag(*blocks)


@pytest.mark.parametrize("dim,k,amp", [(2, 3, 0.0), (2, 2, 0.05), (3, 2, 0.0)])
def test_single_cell_brute_force(dim, k, amp):
    """One periodic cell (its own neighbour on every face), L assembled column by
    column: M L is skew for the central flux on the affine cell and has a
    negative semidefinite symmetric part for the upwind flux."""
    m = make(dim, 1, k, amp, W.ConstantMaterial(1.3, 0.8))
    M = _mass_dense(m)
    Lu = _dense_operator(m, "upwind")
    A = M @ Lu
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.max() < 1e-12 * np.abs(ev).max()
    if amp == 0.0:
        Lc = _dense_operator(m, "central")
        B = M @ Lc
        assert np.abs(B + B.T).max() < 1e-12 * np.abs(B).max()


def test_inverse_mass_equals_basis_change():
    """M_GL^-1 r = S^-1 diag(1/(w det J rho)) S^-T r (Sec. 3.1): the oracle's
    dense Cholesky solve against the tensorized basis-change formula."""
    dim, k = 2, 4
    m = make(dim, 2, k, 0.05)
    n = k + 1
    xg, _ = basis.gauss(n)
    S1 = basis.lagrange(m.xgl, xg)                     # GL coefficients -> G values
    S = np.kron(S1, S1)                                 # y slow, x fast
    r = W.random_state(9, (m.nc, dim + 1, m.np_))
    got = op.apply_mass_inverse(m, r, np.arange(m.nc))
    cd = m.cell_data(np.arange(m.nc))
    Sinv = np.linalg.inv(S)
    for c in range(m.nc):
        mv = cd["wdet"][c] * cd["rho"][c]
        mp = cd["wdet"][c] / (cd["rho"][c] * cd["c"][c] ** 2)
        for v in range(dim + 1):
            mu = mv if v < dim else mp
            want = Sinv @ ((Sinv.T @ r[c, v]) / mu)
            assert np.allclose(got[c, v], want, rtol=1e-11, atol=1e-11 * np.abs(want).max())


@pytest.mark.parametrize("k", [2, 3])
def test_spatial_convergence_standing_wave(k):
    """Standing wave on the affine 2D box: LSRK(5,4) with Cr 0.2, rate k+1."""
    errs = []
    for nc in (4, 8):
        m = make(2, nc, k, 0.0, W.ConstantMaterial())
        U = m.interpolate(lambda x: W.standing_wave_2d(x, 0.0))
        dt, ns = ts.dt_from_courant(m, 0.2, 0.25)
        for s in range(ns):
            U = ts.lsrk_step(lambda u, t: apply_operator(m, u), U, s * dt, dt)
        errs.append(norms.l2_error(m, U, W.standing_wave_2d, 0.25)[0])
    rate = np.log2(errs[0] / errs[1])
    assert rate > k + 1 - 0.3


def test_curved_3d_plane_wave_convergence():
    """Periodic plane wave on the curved 3D box (rho=c=1): rate about k+1."""
    k = 3
    errs = []
    for nc in (4, 6):
        m = make(3, nc, k, 0.05, W.ConstantMaterial())
        U = m.interpolate(lambda x: W.plane_wave_3d(x, 0.0))
        dt, ns = ts.dt_from_courant(m, 0.2, 0.1)
        for s in range(ns):
            U = ts.lsrk_step(lambda u, t: apply_operator(m, u), U, s * dt, dt)
        errs.append(norms.l2_error(m, U, W.plane_wave_3d, 0.1)[0])
    assert np.log(errs[0] / errs[1]) / np.log(1.5) > k + 1 - 0.5


@pytest.mark.parametrize("k", [5, 7])
def test_mass_solve_matches_extended_precision(k):
    """The oracle's float64 Cholesky solve of the dense mass matrix (condition
    kappa_1D^3, about 3.5e3 for k = 7) against the same solve in extended
    precision: the oracle's own rounding is far below the 1e-12 parity bar.
    And the extended solve equals the basis-change formula of Sec. 3.1
    (M_GL^-1 = S^-1 diag(1/(w det J rho)) S^-T), evaluated in float64 one
    direction at a time, to the same level."""
    dim = 3
    m = make(dim, 1, k, 0.05, W.FourierMaterial(11, dim=dim, rho_amp=0.3))
    r = W.random_state(k, (m.nc, dim + 1, m.np_))
    cells = np.arange(m.nc)
    a = op.apply_mass_inverse(m, r, cells)
    b = op.apply_mass_inverse(m, r, cells, extended=True)
    assert norms.rel_l2(a, b) < 1e-14
    assert np.abs(a - b).max() < 1e-14 * np.abs(b).max()
    n = k + 1
    xg, _ = basis.gauss(n)
    Si = np.linalg.inv(basis.lagrange(m.xgl, xg))       # G values -> GL coefficients
    cd = m.cell_data(cells)
    mu = [1.0 / (cd["wdet"][0] * cd["rho"][0])] * dim + [cd["rho"][0] * cd["c"][0] ** 2 / cd["wdet"][0]]
    for v in range(dim + 1):
        t = r[0, v].reshape(n, n, n)                        # [z][y][x]
        for ax in range(3):                                 # S^-T
            t = np.moveaxis(np.tensordot(Si.T, t, axes=([1], [2 - ax])), 0, 2 - ax)
        t = t * mu[v].reshape(n, n, n)
        for ax in range(3):                                 # S^-1
            t = np.moveaxis(np.tensordot(Si, t, axes=([1], [2 - ax])), 0, 2 - ax)
        assert np.abs(t.ravel() - b[0, v]).max() < 1e-13 * np.abs(b[0, v]).max()


def _lagrange_ld(nodes, x):
    """Values and derivatives of the Lagrange polynomials on `nodes` at x, in
    extended precision from the product formula."""
    ld = np.longdouble
    nodes = np.asarray(nodes, dtype=ld)
    x = np.asarray(x, dtype=ld)
    q = len(nodes)
    L = np.ones((len(x), q), dtype=ld)
    dL = np.zeros((len(x), q), dtype=ld)
    for j in range(q):
        for i in range(q):
            if i != j:
                L[:, j] *= (x - nodes[i]) / (nodes[j] - nodes[i])
        for m in range(q):
            if m == j:
                continue
            t = np.full(len(x), 1, dtype=ld) / (nodes[j] - nodes[m])
            for i in range(q):
                if i != j and i != m:
                    t *= (x - nodes[i]) / (nodes[j] - nodes[i])
            dL[:, j] += t
    return L, dL


def test_jacobian_of_small_cells_matches_extended_precision():
    """Cells of the 48^3 box, degree-7 geometry: the oracle's Jacobian against
    the same map differentiated in extended precision with exact tables,
    to 2e-13 relative (in absolute coordinates the derivative sums of a cell
    of size 1/48 lose about 4e-12)."""
    k, n = 7, 48
    nodes = W.box_nodes(3, n, k, 0.05)
    cells = np.array([0, 1234, 50000, n ** 3 - 1])
    m = Mesh(3, k, nodes[cells], np.zeros((4, 6), dtype=np.int64), W.ConstantMaterial())
    _, J = m.map_points(np.arange(4), m.cell_ref)
    L1, D1 = _lagrange_ld(np.arange(k + 1) / k, basis.gauss(k + 1)[0])
    P = L1.shape[0]

    def tens(A, Bm, C):  # x fastest on both sides
        return np.einsum("ia,jb,kc->kjicba", A, Bm, C).reshape(P ** 3, (k + 1) ** 3)

    X = nodes[cells].astype(np.longdouble)
    Jx = np.stack([np.einsum("pg,cga->cpa", t, X) for t in (tens(D1, L1, L1), tens(L1, D1, L1), tens(L1, L1, D1))],
                  axis=-1)
    assert float(np.abs(J - Jx).max() / np.abs(Jx).max()) < 2e-13
