"""The semi-discrete DG operator L = -M^-1 K for first-order acoustics (oracle).

Paper, Sec. 2 (the PDE with S, eq. general-hyp-pde), Sec. 2.1 (weak form,
eq. weak-form; M dU/dt + K U = 0, eq. matrix-tc-sd) and Sec. 2.4 (the HDG
flux, which with tau = 1/(c rho) is the upwind flux).

Reading of the weak form with pointwise-varying rho and c (the paper places
1/rho and rho c^2 inside S and writes an unweighted mass; with coefficients
varying inside a cell that placement loses a gradient of 1/rho).  Here the
material is moved into a weighted mass, which is identical for cell-wise
constant coefficients.  For a GL test function phi and a = 1..d:

    (phi, rho d/dt v_a)_K       = (d phi/d x_a, p)_K - sum_F <phi a_a, p*>_F
    (phi, d/dt p / (rho c^2))_K = (grad phi, v)_K    - sum_F <phi |a|, v*_n>_F

with Gauss quadrature on n = k+1 points per direction (Sec. 3), and
a = w_F det J J^-T n_ref the area vector of a face point.  The numerical
fluxes at a face point (- own side, + neighbour, n the own outward normal,
Z = rho c sampled by each side):

    upwind:  p*   = (Z+ p- + Z- p+ + Z- Z+ (v-.n - v+.n)) / (Z- + Z+)
             v*_n = (Z- v-.n + Z+ v+.n + p- - p+)        / (Z- + Z+)
    central: p*   = (p- + p+)/2,   v*_n = (v-.n + v+.n)/2

For Z- = Z+ the upwind flux is p* = {p} + Z/2 [v_n], v*_n = {v_n} + [p]/(2Z),
the paper's HDG flux with tau = 1/(c rho) once its rows are divided by the
coefficients that the paper keeps inside S.

Boundary faces (the paper asks for boundary conditions without fixing any,
Sec. 2; reading): the exterior state is built from the own trace and goes
through the same flux with Z+ = Z-.  Rigid wall (v.n = 0): the mirror state
p+ = p-, v+ = v- - 2 (v-.n) n, so that v*_n = 0 for both fluxes.  First-order
absorbing boundary: p+ = 0, v+ = 0, so that the upwind flux keeps only the
outgoing characteristic (p- + Z v-.n)/2.  Prescribed exterior state: u+ is
given data u_ext(x) at the face points (the caller chooses its time: the
stage time for Runge-Kutta, the time integral over the step for ADER, whose
update L(I) is linear in the exterior state of I).

The operator is evaluated with the full d-dimensional GL basis tables at the
quadrature points (no sum factorization) and the dense per-cell mass matrices
M_v = sum_q w detJ rho phi_i phi_j, M_p = sum_q w detJ/(rho c^2) phi_i phi_j
are inverted through a Cholesky factorization.

Storage basis (Sec. 3.1 compares two for the Runge-Kutta operator): "gl",
the Lagrange polynomials in the k+1 Gauss-Lobatto points per direction
(nodes on the faces), or "gauss", the Lagrange polynomials in the k+1 Gauss
points (the collocated setup: phi is the identity at the quadrature points,
so the mass matrices are diagonal).  Both span the same space and use the
same quadrature, so the two operators are one linear map in two bases; the
"gauss" one is evaluated here directly from the weak form with its own
tables, not through that identity.
"""
from __future__ import annotations

import numpy as np

from . import basis
from .mesh import BC_WALL, BC_PRESCRIBED


def storage_nodes(mesh, storage):
    """1D nodes of the storage basis: GL points ("gl") or Gauss points ("gauss")."""
    if storage == "gl":
        return mesh.xgl
    if storage == "gauss":
        return mesh.xg
    raise ValueError(f"unknown storage basis {storage!r}")


class Tables:
    """Direct d-dimensional tables of the storage basis at the cell and face Gauss points."""

    def __init__(self, mesh, storage="gl"):
        x1 = storage_nodes(mesh, storage)
        self.nodes = x1
        self.phi = basis.tensor_basis(x1, mesh.cell_ref)            # [Q][np]
        self.dphi = basis.tensor_basis_grad(x1, mesh.cell_ref)      # [d][Q][np]
        self.phif = [basis.tensor_basis(x1, mesh.face_ref[f]) for f in range(mesh.nface)]


def tables(mesh, storage="gl"):
    key = "tables" if storage == "gl" else "tables_" + storage
    t = mesh._cache.get(key)
    if t is None:
        t = Tables(mesh, storage)
        mesh._cache[key] = t
    return t


def numerical_flux(pm, pp, vnm, vnp, Zm, Zp, flux):
    """(p*, v*_n) at face points; see the module docstring."""
    if flux == "upwind":
        s = Zm + Zp
        ps = (Zp * pm + Zm * pp + Zm * Zp * (vnm - vnp)) / s
        vs = (Zm * vnm + Zp * vnp + pm - pp) / s
    elif flux == "central":
        ps = 0.5 * (pm + pp)
        vs = 0.5 * (vnm + vnp)
    else:
        raise ValueError(flux)
    return ps, vs


def exterior_state(um, nrm, nb, d, x=None, exterior=None):
    """Neighbour trace float64[C][d+1][Qf] of boundary faces from the own
    trace um and the unit normals nrm[C][Qf][d] (rows with nb >= 0 are left
    zero for the caller to fill); prescribed faces take exterior(x) at their
    points x[C][Qf][d] (a state float64[...][Qf][d+1])."""
    up = np.zeros_like(um)
    wall = nb == BC_WALL
    if np.any(wall):
        vn = np.einsum("cqa,caq->cq", nrm[wall], um[wall, :d, :])
        up[wall, :d, :] = um[wall, :d, :] - 2.0 * vn[:, None, :] * np.moveaxis(nrm[wall], -1, 1)
        up[wall, d, :] = um[wall, d, :]
    pres = nb == BC_PRESCRIBED
    if np.any(pres):
        if exterior is None:
            raise ValueError("the mesh has prescribed boundary faces: give the exterior state")
        up[pres] = np.moveaxis(np.asarray(exterior(x[pres]), dtype=np.float64), -1, 1)
    # BC_ABSORBING: zero exterior state
    return up


def residual(mesh, U, cells, flux="upwind", storage="gl", exterior=None):
    """Right-hand side r = -K U restricted to `cells`, float64[C][d+1][np]
    (test functions and U in the storage basis)."""
    d = mesh.dim
    T = tables(mesh, storage)
    cells = np.atleast_1d(np.asarray(cells, dtype=np.int64))
    cd = mesh.cell_data(cells)
    Uc = U[cells]
    uq = np.einsum("qi,cvi->cvq", T.phi, Uc)          # values at the Gauss points
    r = np.zeros((len(cells), d + 1, mesh.np_))
    wJ = cd["wdet"][..., None, None] * cd["Jinv"]      # [C][Q][b][a] = w detJ dxi_b/dx_a
    for b in range(d):
        # (d phi/d x_a, p) part for the v_a tests, (grad phi, v) part for the p test
        Fv = wJ[:, :, b, :] * uq[:, d, :, None]        # [C][Q][a]
        Fp = np.einsum("cqa,caq->cq", wJ[:, :, b, :], uq[:, :d, :])
        r[:, :d, :] += np.einsum("qi,cqa->cai", T.dphi[b], Fv)
        r[:, d, :] += np.einsum("qi,cq->ci", T.dphi[b], Fp)
    for f in range(mesh.nface):
        fd = mesh.face_data(cells, f)
        um = np.einsum("qi,cvi->cvq", T.phif[f], Uc)
        a = fd["a"]                                     # [C][Qf][d]
        area = np.sqrt(np.sum(a * a, axis=-1))
        nrm = a / area[..., None]
        nb = fd["nb"]
        inner = nb >= 0
        up = exterior_state(um, nrm, nb, d, fd["x"], exterior)
        for cd in np.unique(fd["code"][inner]):
            sel = inner & (fd["code"] == cd)
            phin = basis.tensor_basis(T.nodes, mesh.neighbor_face_points(f, cd))
            up[sel] = np.einsum("qi,cvi->cvq", phin, U[nb[sel]])
        vnm = np.einsum("cqa,caq->cq", nrm, um[:, :d, :])
        vnp = np.einsum("cqa,caq->cq", nrm, up[:, :d, :])
        ps, vs = numerical_flux(um[:, d], up[:, d], vnm, vnp, fd["Zm"], fd["Zp"], flux)
        r[:, :d, :] -= np.einsum("qi,cqa->cai", T.phif[f], a * ps[..., None])
        r[:, d, :] -= np.einsum("qi,cq->ci", T.phif[f], area * vs)
    return r


def mass_matrices(mesh, cells, storage="gl"):
    """Dense per-cell mass matrices (M_v, M_p), each float64[C][np][np]."""
    T = tables(mesh, storage)
    cd = mesh.cell_data(cells)
    wv = cd["wdet"] * cd["rho"]
    wp = cd["wdet"] / (cd["rho"] * cd["c"] ** 2)
    Mv = np.einsum("qi,cq,qj->cij", T.phi, wv, T.phi)
    Mp = np.einsum("qi,cq,qj->cij", T.phi, wp, T.phi)
    return Mv, Mp


def cholesky_factors(mesh, cells, storage="gl"):
    """Lower Cholesky factors of (M_v, M_p); cached for meshes small enough."""
    cells = np.atleast_1d(np.asarray(cells, dtype=np.int64))
    if not mesh._allow_cache or mesh.nc * 2 * mesh.np_ ** 2 * 8 > 1.0e9:
        Mv, Mp = mass_matrices(mesh, cells, storage)
        return np.linalg.cholesky(Mv), np.linalg.cholesky(Mp)
    key = "chol" if storage == "gl" else "chol_" + storage
    full = mesh._cache.get(key)
    if full is None:
        Mv, Mp = mass_matrices(mesh, np.arange(mesh.nc), storage)
        full = (np.linalg.cholesky(Mv), np.linalg.cholesky(Mp))
        mesh._cache[key] = full
    return full[0][cells], full[1][cells]


def _chol_apply(L, r):
    y = np.linalg.solve(L, np.swapaxes(r, -1, -2))
    x = np.linalg.solve(np.swapaxes(L, -1, -2), y)
    return np.swapaxes(x, -1, -2)


def apply_mass_inverse(mesh, r, cells, storage="gl", extended=False):
    """M^-1 r with the dense per-cell mass matrices (Cholesky).

    extended: assemble M and solve in extended precision (numpy.longdouble,
    64-bit significand on x86) and round the result to float64.  The dense
    mass matrix has condition kappa_1D^d (about 3.5e3 for k = 7 in 3D), so the
    float64 solve carries a relative error up to about kappa eps; the extended
    solve removes that part of the oracle's own rounding."""
    d = mesh.dim
    if extended:
        return _mass_inverse_extended(mesh, r, cells, storage)
    Lv, Lp = cholesky_factors(mesh, cells, storage)
    out = np.empty_like(r)
    out[:, :d, :] = _chol_apply(Lv, r[:, :d, :])
    out[:, d:, :] = _chol_apply(Lp, r[:, d:, :])
    return out


def _cholesky_ld(M):
    """Lower Cholesky factors of a batch M[C][n][n] in the dtype of M
    (column by column: L_jj = sqrt(M_jj - sum_k L_jk^2), then the column below)."""
    C, n, _ = M.shape
    L = np.zeros_like(M)
    for j in range(n):
        col = M[:, j:, j] - np.einsum("cik,ck->ci", L[:, j:, :j], L[:, j, :j])
        piv = np.sqrt(col[:, 0])
        L[:, j, j] = piv
        L[:, j + 1:, j] = col[:, 1:] / piv[:, None]
    return L


def _tri_solve_ld(L, b, lower):
    """Solve L x = b (lower) or L^T x = b (upper) for b[C][n][m] by substitution."""
    C, n, _ = L.shape
    x = np.zeros_like(b)
    rng = range(n) if lower else range(n - 1, -1, -1)
    for i in rng:
        if lower:
            acc = b[:, i, :] - np.einsum("ck,ckm->cm", L[:, i, :i], x[:, :i, :])
        else:
            acc = b[:, i, :] - np.einsum("ck,ckm->cm", L[:, i + 1:, i], x[:, i + 1:, :])
        x[:, i, :] = acc / L[:, i, i][:, None]
    return x


def _mass_inverse_extended(mesh, r, cells, storage):
    ld = np.longdouble
    d = mesh.dim
    T = tables(mesh, storage)
    cd = mesh.cell_data(cells)
    phi = T.phi.astype(ld)
    wdet = cd["wdet"].astype(ld)
    rho = cd["rho"].astype(ld)
    c = cd["c"].astype(ld)
    out = np.empty_like(r)
    for wq, comps in ((wdet * rho, slice(0, d)), (wdet / (rho * c * c), slice(d, d + 1))):
        M = np.stack([(phi * wq[i][:, None]).T @ phi for i in range(len(cells))])
        L = _cholesky_ld(M)
        b = np.swapaxes(r[:, comps, :].astype(ld), 1, 2)          # [C][np][ncomp]
        y = _tri_solve_ld(L, b, lower=True)
        x = _tri_solve_ld(L, y, lower=False)
        out[:, comps, :] = np.swapaxes(x, 1, 2).astype(np.float64)
    return out


def _chunks(mesh, cells):
    budget = 64 * 2 ** 20  # bytes of dense mass matrices per chunk
    step = max(1, budget // (2 * mesh.np_ * mesh.np_ * 8))
    for s in range(0, len(cells), step):
        yield cells[s:s + step]


def apply_operator(mesh, U, cells=None, flux="upwind", storage="gl", exterior=None, extended=False):
    """L U = M^-1 (-K U) (Sec. 2.1, eq. matrix-tc-sd) on `cells` (default all).

    U: float64[Nc][d+1][np] coefficients of the full state in the storage
    basis (neighbours are read); exterior: the prescribed exterior state
    x[...][d] -> float64[...][d+1] for BC_PRESCRIBED faces; extended: the
    mass solve in extended precision (apply_mass_inverse).  Returns
    float64[C][d+1][np].
    """
    U = np.asarray(U, dtype=np.float64)
    cells = np.arange(mesh.nc) if cells is None else np.atleast_1d(np.asarray(cells, dtype=np.int64))
    out = np.empty((len(cells), mesh.dim + 1, mesh.np_))
    pos = 0
    for ch in _chunks(mesh, cells):
        r = residual(mesh, U, ch, flux, storage, exterior)
        out[pos:pos + len(ch)] = apply_mass_inverse(mesh, r, ch, storage, extended)
        pos += len(ch)
    return out


def gl_to_gauss(mesh, U):
    """Coefficients in the Gauss storage basis (the values at the cell Gauss
    points) of a state given in the GL basis: U_G = S U with S[q][i] the GL
    Lagrange polynomial i at Gauss point q (Sec. 3.2)."""
    return np.einsum("qi,cvi->cvq", tables(mesh).phi, np.asarray(U, dtype=np.float64))
