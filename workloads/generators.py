"""Input recipes for the acoustic DG solver (no method arithmetic here).

Conventions shared with the C ABI:

* reference cell [0,1]^d; a cell's geometry is given by (q+1)^d nodes at the
  *equispaced* points j/q of the reference cell, lexicographic with x fastest;
* cells of the n^d box are numbered lexicographically, x fastest;
* neighbour table columns are the faces -x,+x,-y,+y(,-z,+z); periodic wrap;
* the state has components (v_1..v_d, p).
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def _cell_index(idx, n):
    out = 0
    stride = 1
    for i in idx:
        out += (i % n) * stride
        stride *= n
    return out


# Boundary codes in a neighbour table (a face on the domain boundary): a rigid
# (sound-hard) wall, a first-order absorbing boundary and a prescribed
# exterior state.
BC_WALL, BC_ABSORBING, BC_PRESCRIBED = -1, -2, -3


def box_neighbors(dim: int, ncell: int, bc=None) -> np.ndarray:
    """Neighbour table int64[n^dim][2*dim] of the unit box (faces -x,+x,-y,+y,-z,+z).

    bc: None (periodic in every direction) or one entry per direction, each
    "periodic", "wall", "absorbing" or "prescribed": the faces of that
    direction on the box boundary get BC_WALL / BC_ABSORBING / BC_PRESCRIBED
    instead of the periodic neighbour.
    """
    bc = ["periodic"] * dim if bc is None else list(bc)
    if len(bc) != dim or any(b not in ("periodic", "wall", "absorbing", "prescribed") for b in bc):
        raise ValueError("bc: one of periodic / wall / absorbing / prescribed per direction")
    code = {"wall": BC_WALL, "absorbing": BC_ABSORBING, "prescribed": BC_PRESCRIBED}
    nc = ncell ** dim
    nb = np.empty((nc, 2 * dim), dtype=np.int64)
    grid = np.indices((ncell,) * dim).reshape(dim, -1)[::-1]  # grid[0] = x index (fastest)
    for e in range(nc):
        idx = [int(grid[a, e]) for a in range(dim)]
        for a in range(dim):
            for s, off in ((0, -1), (1, +1)):
                j = list(idx)
                j[a] += off
                if bc[a] != "periodic" and not 0 <= j[a] < ncell:
                    nb[e, 2 * a + s] = code[bc[a]]
                else:
                    nb[e, 2 * a + s] = _cell_index(j, ncell)
    return nb


def cube_rotations(dim: int):
    """Orientation-preserving symmetries of the reference cell [0,1]^dim as
    (perm, flip): new coordinate b is old coordinate perm[b], reversed when
    flip[b]; 4 in 2D, 24 in 3D, identity first."""
    import itertools
    out = []
    for perm in itertools.permutations(range(dim)):
        inv = sum(1 for i in range(dim) for j in range(i + 1, dim) if perm[i] > perm[j])
        for flip in itertools.product((0, 1), repeat=dim):
            if (inv + sum(flip)) % 2 == 0:
                out.append((tuple(perm), tuple(flip)))
    out.sort(key=lambda r: (r[0] != tuple(range(dim)), r[1] != (0,) * dim))
    return out


def _old_index(j, rot, m):
    """Old lattice multi-index of new multi-index j (m+1 points per direction)."""
    perm, flip = rot
    i = [0] * len(j)
    for b in range(len(j)):
        i[perm[b]] = m - j[b] if flip[b] else j[b]
    return i


def lattice_permutation(dim: int, m: int, rot) -> np.ndarray:
    """Index array P with new_values[j] = old_values[P[j]] for the (m+1)^dim
    lattice (x fastest) of a cell renumbered by the rotation rot."""
    n = m + 1
    P = np.empty(n ** dim, dtype=np.int64)
    for lin in range(n ** dim):
        j = [(lin // n ** a) % n for a in range(dim)]
        i = _old_index(j, rot, m)
        P[lin] = sum(i[a] * n ** a for a in range(dim))
    return P


def face_orientation(own, other):
    """Orientation code o with other = orient(own) for tangential coordinate
    tuples in [0, 1]: 3D (s, t): bit 2 swaps (s, t) first, bit 0 reverses the
    first and bit 1 the second coordinate; 2D (s,): bit 0 reverses s."""
    for o in range(8 if len(own) == 2 else 2):
        a = list(own)
        if len(a) == 2 and o & 4:
            a = [a[1], a[0]]
        if o & 1:
            a[0] = 1 - a[0]
        if len(a) == 2 and o & 2:
            a[1] = 1 - a[1]
        if all(abs(x - y) < 1e-12 for x, y in zip(a, other)):
            return o
    return None


def rotated_box(dim: int, ncell: int, q: int, amp: float, seed: int, frac: float = 0.6):
    """The periodic box with a random subset of its cells renumbered by random
    reference-cell rotations: the same mesh (same physical cells), but faces
    meet with other face indices and orientations.  Returns (geo_nodes,
    neighbors, face_orient, rotations) where face_orient[c][f] = 8 f' + o
    (the neighbour's face f' and the orientation o of face_orientation) and
    rotations[c] the (perm, flip) applied to cell c."""
    nodes = box_nodes(dim, ncell, q, amp)
    nb_old = box_neighbors(dim, ncell)
    rots_all = cube_rotations(dim)
    rng = np.random.default_rng(seed)
    nc = nodes.shape[0]
    rot = [rots_all[0] if rng.random() > frac else rots_all[rng.integers(1, len(rots_all))] for _ in range(nc)]
    new_nodes = np.stack([nodes[c][lattice_permutation(dim, q, rot[c])] for c in range(nc)])

    def old_face(c, f):  # old face index of new face f of cell c
        perm, flip = rot[c]
        b, side = divmod(f, 2)
        return 2 * perm[b] + (side ^ flip[b])

    def new_face(c, F):
        perm, flip = rot[c]
        b = perm.index(F // 2)
        return 2 * b + ((F % 2) ^ flip[b])

    def tangential(f, pt):  # tangential coordinates of a reference point on face f
        return tuple(pt[a] for a in range(dim) if a != f // 2)

    def to_old(c, xi):  # reference point of the new numbering -> old numbering
        perm, flip = rot[c]
        x = [0.0] * dim
        for b in range(dim):
            x[perm[b]] = 1 - xi[b] if flip[b] else xi[b]
        return x

    def to_new(c, x):
        perm, flip = rot[c]
        return [1 - x[perm[b]] if flip[b] else x[perm[b]] for b in range(dim)]

    nb = np.empty((nc, 2 * dim), dtype=np.int64)
    fo = np.empty((nc, 2 * dim), dtype=np.int32)
    probe = [(0.25, 0.6), (0.7, 0.15)] if dim == 3 else [(0.3,)]
    for c in range(nc):
        for f in range(2 * dim):
            F = old_face(c, f)
            c2 = nb_old[c, F]
            f2 = new_face(c2, F ^ 1)
            codes = set()
            for tp in probe:
                xi = []
                t = 0
                for a in range(dim):
                    if a == f // 2:
                        xi.append(float(f % 2))
                    else:
                        xi.append(tp[t])
                        t += 1
                x_old = to_old(c, xi)
                x_old[F // 2] = 1.0 - x_old[F // 2]          # the same point seen from the neighbour
                y = to_new(c2, x_old)
                codes.add(face_orientation(tangential(f, xi), tangential(f2, y)))
            assert len(codes) == 1 and None not in codes
            nb[c, f] = c2
            fo[c, f] = 8 * f2 + codes.pop()
    return new_nodes, nb, fo, rot


def box_nodes(dim: int, ncell: int, q: int, amp: float) -> np.ndarray:
    """Geometry nodes float64[n^dim][(q+1)^dim][dim] of the periodic unit box.

    Each undeformed node X is moved to X + amp * prod_j sin(2 pi X_j) in every
    coordinate (the same displacement for all coordinates).  amp = 0 gives the
    affine Cartesian mesh.
    """
    h = 1.0 / ncell
    ref = np.arange(q + 1, dtype=np.float64) / q
    # node offsets inside one cell, lexicographic x fastest
    loc = np.stack(np.meshgrid(*([ref] * dim), indexing="ij"), axis=-1)  # [..][dim] with axis order (x0,x1,..)
    loc = loc.transpose(*range(dim - 1, -1, -1), dim).reshape(-1, dim)   # x fastest
    grid = np.indices((ncell,) * dim).reshape(dim, -1)[::-1].T          # [nc][dim], x fastest
    X = (grid[:, None, :] + loc[None, :, :]) * h
    disp = amp * np.prod(np.sin(TWO_PI * X), axis=-1)
    return np.ascontiguousarray(X + disp[..., None])


class ConstantMaterial:
    """rho and c constant."""

    def __init__(self, rho: float = 1.0, c: float = 1.0):
        self.rho = float(rho)
        self.c = float(c)

    def __call__(self, x: np.ndarray):
        x = np.asarray(x)
        shp = x.shape[:-1]
        return np.full(shp, self.rho), np.full(shp, self.c)


def _fourier_modes(rng, dim, nmodes):
    """nmodes wave vectors uniform in {-2..2}^d without 0, amplitudes ~ U[-1,1],
    phases ~ U[0, 2 pi), drawn in this order from rng."""
    modes = []
    while len(modes) < nmodes:
        m = rng.integers(-2, 3, size=dim)
        if np.any(m != 0):
            modes.append(m)
    return (np.array(modes, dtype=np.int64), rng.uniform(-1.0, 1.0, size=nmodes),
            rng.uniform(0.0, TWO_PI, size=nmodes))


class FourierMaterial:
    """c(x) = clamp(c0 + amp * nmodes^-1/2 * sum_i a_i cos(2 pi m_i.x + phi_i), cmin, cmax).

    The mode data are drawn with numpy.random.default_rng(seed): wave vectors
    m_i uniform in {-2..2}^d without 0, a_i ~ U[-1,1], phi_i ~ U[0, 2 pi).
    The field is 1-periodic in every coordinate.

    Density: rho(x) = rho for rho_amp = 0 (the default); otherwise a second
    field of the same kind with its own modes, drawn from
    default_rng(seed + 7919) so that c is the same for either choice:
    rho(x) = clamp(rho (1 + rho_amp nmodes^-1/2 sum_i b_i cos(2 pi n_i.x + psi_i)),
    0.7 rho, 1.3 rho).
    """

    def __init__(self, seed: int, dim: int = 3, nmodes: int = 8, amp: float = 0.3,
                 c0: float = 1.0, cmin: float = 0.7, cmax: float = 1.3, rho: float = 1.0,
                 rho_amp: float = 0.0):
        self.m, self.a, self.phi = _fourier_modes(np.random.default_rng(seed), dim, nmodes)
        self.dim, self.nmodes, self.amp = dim, nmodes, amp
        self.c0, self.cmin, self.cmax, self.rho = c0, cmin, cmax, rho
        self.rho_amp = float(rho_amp)
        if self.rho_amp != 0.0:
            self.rm, self.rb, self.rpsi = _fourier_modes(np.random.default_rng(seed + 7919), dim, nmodes)

    def c(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        arg = TWO_PI * (x @ self.m.T.astype(np.float64)) + self.phi
        s = np.cos(arg) @ self.a
        return np.clip(self.c0 + self.amp / np.sqrt(self.nmodes) * s, self.cmin, self.cmax)

    def density(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        if self.rho_amp == 0.0:
            return np.full(x.shape[:-1], self.rho)
        arg = TWO_PI * (x @ self.rm.T.astype(np.float64)) + self.rpsi
        s = np.cos(arg) @ self.rb
        return np.clip(self.rho * (1.0 + self.rho_amp / np.sqrt(self.nmodes) * s), 0.7 * self.rho, 1.3 * self.rho)

    def __call__(self, x: np.ndarray):
        return self.density(x), self.c(x)


def standing_wave_2d(x: np.ndarray, t: float = 0.0) -> np.ndarray:
    """Exact standing wave on the periodic unit square, rho = c = 1.

    p = sin(2 pi x) sin(2 pi y) cos(2 pi sqrt2 t),
    v = -(1/sqrt2) (cos 2pi x sin 2pi y, sin 2pi x cos 2pi y) sin(2 pi sqrt2 t).
    Returns float64[..., 3] with components (v1, v2, p).
    """
    x = np.asarray(x, dtype=np.float64)
    w = TWO_PI * np.sqrt(2.0)
    sx, cx = np.sin(TWO_PI * x[..., 0]), np.cos(TWO_PI * x[..., 0])
    sy, cy = np.sin(TWO_PI * x[..., 1]), np.cos(TWO_PI * x[..., 1])
    out = np.empty(x.shape[:-1] + (3,))
    st = np.sin(w * t)
    out[..., 0] = -cx * sy * st / np.sqrt(2.0)
    out[..., 1] = -sx * cy * st / np.sqrt(2.0)
    out[..., 2] = sx * sy * np.cos(w * t)
    return out


def plane_wave_3d(x: np.ndarray, t: float = 0.0) -> np.ndarray:
    """Periodic plane wave on the unit cube, rho = c = 1.

    p = cos(2 pi (x+y+z) - 2 pi sqrt3 t), v = p (1,1,1)/sqrt3.
    Returns float64[..., 4] with components (v1, v2, v3, p).
    """
    x = np.asarray(x, dtype=np.float64)
    p = np.cos(TWO_PI * (x[..., 0] + x[..., 1] + x[..., 2]) - TWO_PI * np.sqrt(3.0) * t)
    out = np.empty(x.shape[:-1] + (4,))
    out[..., :3] = p[..., None] / np.sqrt(3.0)
    out[..., 3] = p
    return out


def membrane_mode(x: np.ndarray, t: float = 0.0, m=None) -> np.ndarray:
    """Standing mode of the unit box with rigid walls, rho = c = 1:
    p = cos(omega t) prod_j cos(pi m_j x_j), omega = pi |m|,
    v_a = sin(omega t) (pi m_a / omega) sin(pi m_a x_a) prod_{j != a} cos(pi m_j x_j)
    (v.n = 0 on every wall).  m: mode numbers per direction (default all 1)."""
    x = np.asarray(x, dtype=np.float64)
    dim = x.shape[-1]
    m = np.ones(dim) if m is None else np.asarray(m, dtype=np.float64)
    om = np.pi * np.sqrt(np.sum(m * m))
    cs = np.cos(np.pi * m * x)
    sn = np.sin(np.pi * m * x)
    out = np.empty(x.shape[:-1] + (dim + 1,))
    out[..., dim] = np.cos(om * t) * np.prod(cs, axis=-1)
    for a in range(dim):
        others = np.prod(np.delete(cs, a, axis=-1), axis=-1) if dim > 1 else 1.0
        out[..., a] = np.sin(om * t) * (np.pi * m[a] / om) * sn[..., a] * others
    return out


class PlaneWaves:
    """A superposition of acoustic plane waves in a homogeneous medium, the
    prescribed exterior state of boundary faces and a closed-form solution:
    wave j has p_j = A_j cos(k_j.x - omega_j t + phi_j) and
    v_j = p_j k_j / (|k_j| Z_j) (Z = rho c, omega = c |k| for a solution).
    waves: rows (A, k_1, k_2, k_3, omega, phi, Z), k_3 ignored in 2D."""

    def __init__(self, waves):
        self.w = np.atleast_2d(np.asarray(waves, dtype=np.float64))
        assert self.w.shape[1] == 7

    def _parts(self, x):
        x = np.asarray(x, dtype=np.float64)
        dim = x.shape[-1]
        for A, k1, k2, k3, om, ph, Z in self.w:
            k = np.array([k1, k2, k3])[:dim]
            yield dim, A, k, om, ph, Z, x @ k + ph

    def __call__(self, x, t=0.0):
        """State float64[..., d+1] at time t."""
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros(x.shape[:-1] + (x.shape[-1] + 1,))
        for dim, A, k, om, ph, Z, th in self._parts(x):
            p = A * np.cos(th - om * t)
            out[..., dim] += p
            out[..., :dim] += p[..., None] * (k / (np.linalg.norm(k) * Z))
        return out

    def integral(self, x, t0, dt):
        """Time integral of the state over [t0, t0 + dt], float64[..., d+1]:
        int cos(th - om s) ds = 2 cos(th - om (t0 + dt/2)) sin(om dt/2) / om."""
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros(x.shape[:-1] + (x.shape[-1] + 1,))
        for dim, A, k, om, ph, Z, th in self._parts(x):
            fac = dt if om == 0.0 else 2.0 * np.sin(0.5 * om * dt) / om
            p = A * fac * np.cos(th - om * (t0 + 0.5 * dt))
            out[..., dim] += p
            out[..., :dim] += p[..., None] * (k / (np.linalg.norm(k) * Z))
        return out


def c3_literal_plane_wave():
    """The plane wave of the 48^3 workload text, p = cos(2 pi (x+y+z)/sqrt 3 -
    2 pi t), rho = c = 1 (not periodic on the unit cube: needs its own exterior
    state on every boundary face)."""
    s = 2.0 * np.pi / np.sqrt(3.0)
    return PlaneWaves([[1.0, s, s, s, 2.0 * np.pi, 0.0, 1.0]])


def travelling_pulse_x(x: np.ndarray, t: float = 0.0, x0: float = 0.6, width: float = 0.05) -> np.ndarray:
    """Right-going plane pulse along x, rho = c = 1: p = v_x = g(x - x0 - t) with
    g a Gaussian of the given width, other velocity components 0.  Exact in the
    box with absorbing x faces while the pulse enters nowhere (g ~ 0 at x = 0)."""
    x = np.asarray(x, dtype=np.float64)
    dim = x.shape[-1]
    g = np.exp(-((x[..., 0] - x0 - t) ** 2) / (2.0 * width * width))
    out = np.zeros(x.shape[:-1] + (dim + 1,))
    out[..., 0] = g
    out[..., dim] = g
    return out


def gaussian_pulse(x: np.ndarray, x0, width: float = 0.05) -> np.ndarray:
    """p = exp(-|x - x0|^2 / (2 width^2)) with minimum-image periodic distance, v = 0."""
    x = np.asarray(x, dtype=np.float64)
    d = x - np.asarray(x0, dtype=np.float64)
    d -= np.round(d)
    r2 = np.sum(d * d, axis=-1)
    dim = x.shape[-1]
    out = np.zeros(x.shape[:-1] + (dim + 1,))
    out[..., dim] = np.exp(-r2 / (2.0 * width * width))
    return out


def random_state(seed: int, shape) -> np.ndarray:
    """Standard-normal float64 array of the given shape."""
    return np.random.default_rng(seed).standard_normal(shape)


def random_points(seed: int, count: int, dim: int) -> np.ndarray:
    """Uniform points in the unit box, float64[count][dim]."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(count, dim))


def c2_workload(ncell: int = 24, k: int = 5, seed: int = 1805):
    """The 3D curved-hex workload: unit cube, n^3 cells deformed with amplitude
    0.05, rho = 1, c a random Fourier field, Gaussian pulse (width 0.05) at a
    seeded point.  Returns a dict of inputs."""
    mat = FourierMaterial(seed, dim=3)
    x0 = random_points(seed + 1, 1, 3)[0]
    return dict(dim=3, ncell=ncell, k=k, q=k, amp=0.05, material=mat,
                ic=lambda x: gaussian_pulse(x, x0, 0.05), x0=x0)


class GradedMedium:
    """A medium graded along x with a constant impedance, and its exact wave.

    c(x) = c0 / (1 + eps sin(2 pi x)), rho(x) = (Z / c0)(1 + eps sin(2 pi x)),
    so Z = rho c is constant and both coefficients vary inside every cell along
    the direction of propagation.  With the travel time
    tau(x) = (x + eps (1 - cos(2 pi x)) / (2 pi)) / c0 (tau' = 1/c) the
    right-going wave p = cos(2 pi c0 (tau(x) - t)), v = (p / Z, 0, ..) solves
    rho v_t + grad p = 0, p_t + rho c^2 div v = 0 exactly (p + Z v_x is carried
    along x at the local speed c; the impedance is matched, so nothing is
    reflected).  The field is 1-periodic in x."""

    def __init__(self, eps: float = 0.3, c0: float = 1.0, Z: float = 1.2):
        self.eps, self.c0, self.Z = float(eps), float(c0), float(Z)

    def _g(self, x):
        return 1.0 + self.eps * np.sin(TWO_PI * np.asarray(x, dtype=np.float64)[..., 0])

    def __call__(self, x):
        g = self._g(x)
        return self.Z / self.c0 * g, self.c0 / g

    def wave(self, x, t=0.0):
        x = np.asarray(x, dtype=np.float64)
        s = x[..., 0] + self.eps * (1.0 - np.cos(TWO_PI * x[..., 0])) / TWO_PI
        p = np.cos(TWO_PI * (s - self.c0 * t))
        out = np.zeros(x.shape[:-1] + (x.shape[-1] + 1,))
        out[..., 0] = p / self.Z
        out[..., -1] = p
        return out
