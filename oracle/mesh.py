"""Curved-cell geometry and material sampling (oracle).

The paper allows general curved quadrilaterals/hexahedra with variable
coefficients (abstract; Sec. 3 where the Gauss rule is chosen) and uses
pre-computed inverse Jacobians at the quadrature points (Sec. 3.4, degree
reduction; Sec. 4.4, roofline discussion).  It does not fix a representation
of the curved map; the reading taken here is an isoparametric-style map of
degree q given by the positions of (q+1)^d equispaced nodes per cell:

    x(xi) = sum_j X_j psi_j(xi),   J_ab = d x_a / d xi_b,

with psi_j the d-dimensional Lagrange polynomials on the equispaced nodes,
evaluated directly (no sum factorization).  Face quadrature uses the n^(d-1)
tensor Gauss points of the face (the paper only implies this), and the face
"area vector" folds in the face weight:  a = w_F det(J) J^-T n_ref, whose
length is the surface element and whose direction is the outward normal.
"""
from __future__ import annotations

import numpy as np

from . import basis


# Boundary codes of the neighbour table: rigid (sound-hard) wall, first-order
# absorbing boundary, prescribed exterior state.
BC_WALL, BC_ABSORBING, BC_PRESCRIBED = -1, -2, -3


class Mesh:
    """A mesh of curved quads (d=2) or hexes (d=3) with degree-k DG fields.

    geo_nodes: float64[Nc][(q+1)^d][d]; neighbors: int64[Nc][2d] in face order
    -x,+x,-y,+y,-z,+z; a negative entry marks a face on the domain boundary
    with its condition (BC_WALL, BC_ABSORBING, BC_PRESCRIBED; the paper
    leaves the boundary conditions open, Sec. 2); material: callable
    x[...,d] -> (rho, c).
    face_orient: None (every neighbour meets face f with its face f^1, the
    tangential coordinates aligned) or int[Nc][2d] with 8 f' + o: the
    neighbour's face f' and the orientation o that maps the own tangential
    coordinates (s, t) to the neighbour's: bit 2 swaps them first, bit 0
    reverses the first, bit 1 the second (2D: bit 0 reverses s).
    """

    def __init__(self, dim, k, geo_nodes, neighbors, material, cache=True, face_orient=None):
        self.dim = int(dim)
        self.k = int(k)
        self.n = self.k + 1
        self.geo_nodes = np.ascontiguousarray(geo_nodes, dtype=np.float64)
        self.neighbors = np.ascontiguousarray(neighbors, dtype=np.int64)
        if np.any((self.neighbors < 0) & (self.neighbors != BC_WALL) & (self.neighbors != BC_ABSORBING)
                  & (self.neighbors != BC_PRESCRIBED)):
            raise ValueError("negative neighbour entries must be BC_WALL, BC_ABSORBING or BC_PRESCRIBED")
        if face_orient is None:
            fo = np.array([8 * (f ^ 1) for f in range(2 * self.dim)], dtype=np.int64)
            self.face_orient = np.broadcast_to(fo, self.neighbors.shape).copy()
        else:
            self.face_orient = np.ascontiguousarray(face_orient, dtype=np.int64)
            no = 8 if self.dim == 3 else 2
            if np.any(self.face_orient // 8 >= 2 * self.dim) or np.any(self.face_orient % 8 >= no):
                raise ValueError("face_orient codes out of range")
        self.material = material
        self.nc = self.geo_nodes.shape[0]
        ng = self.geo_nodes.shape[1]
        q = int(round(ng ** (1.0 / self.dim))) - 1
        if (q + 1) ** self.dim != ng or q < 1:
            raise ValueError("geo_nodes must hold (q+1)^d nodes per cell")
        self.q = q
        self.np_ = self.n ** self.dim
        self.nface = 2 * self.dim
        self._geo_ref = basis.equispaced(q)
        # reference rules
        self.xg, self.wg = basis.gauss(self.n)
        self.xgl, self.wgl = basis.gauss_lobatto(self.n)
        self.cell_ref = basis.tensor_points(self.xg, self.dim)
        self.cell_w = basis.tensor_weights(self.wg, self.dim)
        self.face_ref = [self._face_points(f) for f in range(self.nface)]
        self.face_w = basis.tensor_weights(self.wg, self.dim - 1) if self.dim > 1 else np.ones(1)
        self._cache = {}
        self._allow_cache = bool(cache)

    # ---- reference geometry --------------------------------------------
    def _face_points(self, f):
        """Reference Gauss points of face f: xi_a = side, tangential coordinates
        in increasing direction order, the first remaining direction fastest."""
        a, s = divmod(f, 2)
        tang = basis.tensor_points(self.xg, self.dim - 1)
        pts = np.empty((tang.shape[0], self.dim))
        t = 0
        for b in range(self.dim):
            if b == a:
                pts[:, b] = float(s)
            else:
                pts[:, b] = tang[:, t]
                t += 1
        return pts

    def neighbor_face_points(self, f, code):
        """Reference points, on the neighbour's face code // 8, of the Gauss
        points of own face f (same order as face_ref[f]), for orientation code
        % 8 (class docstring)."""
        fn, o = divmod(int(code), 8)
        own = self.face_ref[f]
        tang = [a for a in range(self.dim) if a != f // 2]
        st = own[:, tang].copy()                       # own tangential coordinates
        if self.dim == 3 and o & 4:
            st = st[:, ::-1].copy()
        if o & 1:
            st[:, 0] = 1.0 - st[:, 0]
        if self.dim == 3 and o & 2:
            st[:, 1] = 1.0 - st[:, 1]
        pts = np.empty_like(own)
        t = 0
        for a in range(self.dim):
            if a == fn // 2:
                pts[:, a] = float(fn % 2)
            else:
                pts[:, a] = st[:, t]
                t += 1
        return pts

    def face_normal_ref(self, f):
        a, s = divmod(f, 2)
        nv = np.zeros(self.dim)
        nv[a] = 1.0 if s == 1 else -1.0
        return nv

    # ---- the map ---------------------------------------------------------
    def map_points(self, cells, ref_pts):
        """Physical points x[C][P][d] and Jacobians J[C][P][d][d] (J[..,a,b] = dx_a/dxi_b).

        J is the derivative of the map of the nodes taken relative to the
        cell's first node (a translation leaves it unchanged; in absolute
        coordinates of order 1 a cell of size 1/48 would lose about 1e-12 of
        its Jacobian to cancellation in the derivative sums)."""
        cells = np.atleast_1d(np.asarray(cells, dtype=np.int64))
        psi = basis.tensor_basis(self._geo_ref, ref_pts)          # [P][Ng]
        dpsi = basis.tensor_basis_grad(self._geo_ref, ref_pts)    # [d][P][Ng]
        X = self.geo_nodes[cells]                                  # [C][Ng][d]
        x = np.einsum("pg,cga->cpa", psi, X)
        Xr = X - X[:, :1, :]
        J = np.stack([np.einsum("pg,cga->cpa", dpsi[b], Xr) for b in range(self.dim)], axis=-1)
        return x, J

    # ---- cached per-point data ---------------------------------------------
    def _cacheable(self):
        return self._allow_cache and self.nc * self.np_ * 40 * 8 < 1.5e9

    def _sliced(self, key, fn, cells):
        cells = np.atleast_1d(np.asarray(cells, dtype=np.int64))
        if not self._cacheable():
            return fn(cells)
        full = self._cache.get(key)
        if full is None:
            parts = [fn(np.arange(s, min(s + 4096, self.nc))) for s in range(0, self.nc, 4096)]
            full = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
            self._cache[key] = full
        return {k: v[cells] for k, v in full.items()}

    def cell_data(self, cells):
        """Geometry and material at the n^d Gauss points of each cell."""
        return self._sliced("cell", self._cell_data, cells)

    def face_data(self, cells, f):
        return self._sliced(("face", f), lambda c: self._face_data(c, f), cells)

    def _cell_data(self, cells):
        x, J = self.map_points(cells, self.cell_ref)
        detJ = np.linalg.det(J)
        if np.any(detJ <= 0.0):
            raise ValueError("non-positive Jacobian determinant")
        Jinv = np.linalg.inv(J)                                    # Jinv[..,b,a] = dxi_b/dx_a
        rho, c = self.material(x)
        return dict(x=x, J=J, detJ=detJ, Jinv=Jinv, wdet=self.cell_w[None, :] * detJ,
                    rho=np.asarray(rho, dtype=np.float64), c=np.asarray(c, dtype=np.float64))

    def _face_data(self, cells, f):
        """Area vectors a[C][Qf][d] (face weight folded in), own and neighbour
        impedance Z = rho c at the face points (each side samples the material
        at its own mapped point; on a boundary face the exterior impedance is
        the own one)."""
        x, J = self.map_points(cells, self.face_ref[f])
        detJ = np.linalg.det(J)
        if np.any(detJ <= 0.0):
            raise ValueError("non-positive Jacobian determinant on a face")
        JinvT = np.swapaxes(np.linalg.inv(J), -1, -2)
        a = self.face_w[None, :, None] * detJ[..., None] * (JinvT @ self.face_normal_ref(f))
        rho, c = self.material(x)
        nbc = self.neighbors[cells, f]
        code = self.face_orient[cells, f]
        Zm = np.asarray(rho * c, dtype=np.float64)
        Zp = Zm.copy()
        for cd in np.unique(code[nbc >= 0]):
            sel = (nbc >= 0) & (code == cd)
            xn, _ = self.map_points(nbc[sel], self.neighbor_face_points(f, cd))
            rhon, cn = self.material(xn)
            Zp[sel] = rhon * cn
        return dict(a=a, x=x, Zm=Zm, Zp=Zp, nb=nbc, code=code)

    def node_points(self, cells=None):
        """Physical positions of the GL nodes, float64[C][n^d][d] (for interpolating
        initial data)."""
        cells = np.arange(self.nc) if cells is None else cells
        x, _ = self.map_points(cells, basis.tensor_points(self.xgl, self.dim))
        return x

    def interpolate(self, fn, cells=None):
        """GL nodal interpolant of fn(x) -> [..., d+1]: state float64[C][d+1][n^d]."""
        x = self.node_points(cells)
        return np.ascontiguousarray(np.moveaxis(fn(x), -1, 1))
