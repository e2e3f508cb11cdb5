"""Thin ctypes binding of libdgw (the C ABI in include/dgw.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory (CUDA/HIP tensors) and streams.  Importing
this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

import torch  # noqa: F401  (loads the HIP runtime the library links against)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgw.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1805_03981_amd.build`")
lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EUNSTABLE, EBUSY = 0, -1, -2, -3, -4, -5, -6
FLUX_UPWIND, FLUX_CENTRAL = 0, 1
FP64, FP32_SPLIT = 0, 1
BASIS_GL, BASIS_GAUSS = 0, 1
LSRK54, ADER = 0, 1
LSRK54_MERGED_VU, LSRK54_STANDARD_VU = 2, 3   # unfused LSRK variants (ablation)
LSRK59 = 4                                     # nine-stage fifth-order two-register scheme
ADER_REDUCE, ADER_NOREDUCE, ADER_HDG = 0, 1, 2
ADER_REDUCE_EVERY_STEP, ADER_REDUCE_EVERY_THIRD = 4, 8
DEVICE_NONE = -1
GET_NODE_COORDS, GET_CELL_METRIC, GET_FACE, GET_LEVEL0 = 0, 1, 2, 16

MATERIAL_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.c_int64, C.c_int, C.POINTER(C.c_double),
                          C.POINTER(C.c_double), C.c_void_p)


BC_WALL, BC_ABSORBING, BC_PRESCRIBED = -1, -2, -3


class PlaneWave(C.Structure):
    """p = A cos(k.x - omega t + phi), v = p k / (|k| Z): exterior state of BC_PRESCRIBED faces."""
    _fields_ = [("amplitude", C.c_double), ("k", C.c_double * 3), ("omega", C.c_double), ("phase", C.c_double),
                ("impedance", C.c_double)]


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("degree", C.c_int), ("n_cells", C.c_int64), ("geo_degree", C.c_int),
                ("geo_nodes", C.POINTER(C.c_double)), ("neighbors", C.POINTER(C.c_int64)),
                ("face_orient", C.POINTER(C.c_int)), ("material", MATERIAL_FN), ("material_ctx", C.c_void_p),
                ("flux", C.c_int), ("precision", C.c_int), ("device", C.c_int), ("max_batch", C.c_int),
                ("storage_basis", C.c_int), ("plane_waves", C.POINTER(PlaneWave)), ("n_plane_waves", C.c_int)]


class MeshInfo(C.Structure):
    _fields_ = [("dim", C.c_int), ("degree", C.c_int), ("n1d", C.c_int), ("nodes_per_cell", C.c_int),
                ("n_comp", C.c_int), ("geo_degree", C.c_int), ("n_cells", C.c_int64), ("dofs", C.c_int64),
                ("state_bytes", C.c_int64), ("lsrk_work_bytes", C.c_int64), ("ader_work_bytes", C.c_int64),
                ("device_bytes", C.c_int64), ("n_levels", C.c_int), ("level_points", C.c_int * 8),
                ("h_min", C.c_double), ("c_max", C.c_double), ("dt_unit", C.c_double), ("precision", C.c_int),
                ("flux", C.c_int), ("max_batch", C.c_int), ("device", C.c_int)]


class FourierMaterial(C.Structure):
    _fields_ = [("nmodes", C.c_int), ("m", (C.c_int * 3) * 16), ("a", C.c_double * 16), ("phi", C.c_double * 16),
                ("c0", C.c_double), ("amp", C.c_double), ("cmin", C.c_double), ("cmax", C.c_double),
                ("rho0", C.c_double)]


class SourceDesc(C.Structure):
    _fields_ = [("n", C.c_int), ("position", C.POINTER(C.c_double)), ("frequency", C.POINTER(C.c_double)),
                ("t0", C.POINTER(C.c_double)), ("amplitude", C.POINTER(C.c_double))]


class Profile(C.Structure):
    _fields_ = [("n", C.c_int), ("ms", C.c_double * 4), ("launches", C.c_int64 * 4), ("names", (C.c_char * 32) * 4)]


class SolveDesc(C.Structure):
    _fields_ = [("scheme", C.c_int), ("ader_flags", C.c_int), ("courant", C.c_double), ("dt", C.c_double),
                ("t0", C.c_double), ("t_end", C.c_double), ("sources", C.c_void_p), ("use_graph", C.c_int),
                ("autotune", C.c_int), ("watchdog_every", C.c_int), ("watchdog_growth", C.c_double),
                ("stream", C.c_void_p)]


class SolveReport(C.Structure):
    _fields_ = [("steps", C.c_int64), ("dt", C.c_double), ("wall_s", C.c_double),
                ("dof_steps_per_s", C.c_double), ("energy0", C.c_double), ("energy_end", C.c_double)]


class Request(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("dim", C.c_int), ("ncell", C.c_int), ("degree", C.c_int),
                ("scheme", C.c_int), ("precision", C.c_int), ("t_end", C.c_double), ("courant", C.c_double),
                ("deform_amp", C.c_double), ("material", FourierMaterial), ("ic_center", C.c_double * 3),
                ("ic_width", C.c_double)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("t_arrive", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("steps", C.c_int64), ("dofs", C.c_int64), ("energy0", C.c_double), ("energy_end", C.c_double),
                ("state_host", C.POINTER(C.c_double))]


class ServerDesc(C.Structure):
    _fields_ = [("device", C.c_int), ("hbm_budget_bytes", C.c_double), ("max_live", C.c_int),
                ("realtime", C.c_int), ("progress", C.c_int)]


class ServeReport(C.Structure):
    _fields_ = [("n_done", C.c_int), ("n_failed", C.c_int), ("wall_s", C.c_double), ("p50_s", C.c_double),
                ("p99_s", C.c_double), ("dof_steps_per_s", C.c_double), ("max_wait_s", C.c_double)]


_vp, _dp, _i, _d, _i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int, C.c_double, C.c_int64
_SIGS = {
    "dgw_mesh_create": ([C.POINTER(MeshDesc), C.POINTER(_vp)], _i),
    "dgw_mesh_create_box": ([_i, _i, _i, _d, MATERIAL_FN, _vp, _i, _i, _i, _i, _i, C.POINTER(_vp)], _i),
    "dgw_mesh_destroy": ([_vp], None),
    "dgw_mesh_info_get": ([_vp, C.POINTER(MeshInfo)], _i),
    "dgw_mesh_get": ([_vp, _i, _dp, _i64], _i),
    "dgw_operator_apply": ([_vp, _vp, _vp, _i, _vp], _i),
    "dgw_sources_create": ([_vp, C.POINTER(SourceDesc), C.POINTER(_vp)], _i),
    "dgw_sources_destroy": ([_vp], None),
    "dgw_step_lsrk": ([_vp, _i, _d, _d, _i, _vp, _vp, _i, _vp, _vp], _i),
    "dgw_step_ader": ([_vp, _i, _d, _d, _i, _vp, _vp, _i, _vp, _vp], _i),
    "dgw_step_ader_noalloc": ([_vp, _i, _d, _d, _i, _vp, _i, _vp, _vp], _i),
    "dgw_energy": ([_vp, _vp, _i, _dp, _vp], _i),
    "dgw_step_profile": ([_vp, _i, _i, _d, _d, _i, _vp, _vp, _i, _vp, _vp, C.POINTER(Profile)], _i),
    "dgw_autotune": ([_vp, _i, _vp], _i),
    "dgw_launch_shape": ([_vp, _i, C.POINTER(_i), C.POINTER(_i)], _i),
    "dgw_solve_batch": ([_vp, C.POINTER(SolveDesc), _vp, _vp, _i, C.POINTER(SolveReport)], _i),
    "dgw_serve": ([C.POINTER(ServerDesc), C.POINTER(Request), _i, C.POINTER(Result), C.POINTER(ServeReport)], _i),
    "dgw_request_footprint": ([C.POINTER(Request)], _i64),
    "dgw_last_error": ([], C.c_char_p),
    "dgw_version": ([], C.c_char_p),
    "dgw_basis_1d": ([_i, _i, _dp], _i),
    "dgw_lsrk_coefficients": ([_i, _dp], _i),
    "dgw_material_fourier": ([_dp, _i64, _i, _dp, _dp, _vp], None),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = sorted(_SIGS)
FOURIER_MATERIAL_FN = MATERIAL_FN(("dgw_material_fourier", lib))


class DgwError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: status {status}: {lib.dgw_last_error().decode()}")


def check(status, where):
    if status != OK:
        raise DgwError(status, where)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _tptr(t):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 device tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def material_callback(fn):
    """Wrap fn(x[npts][dim]) -> (rho, c) as a dgw_material_fn."""
    def cb(x, npts, dim, rho, c, ctx):
        xa = np.ctypeslib.as_array(x, shape=(npts, dim))
        r, s = fn(xa)
        np.ctypeslib.as_array(rho, shape=(npts,))[:] = r
        np.ctypeslib.as_array(c, shape=(npts,))[:] = s
    return MATERIAL_FN(cb)


def fourier_material_struct(mat) -> FourierMaterial:
    """The C struct of a workloads.FourierMaterial (same modes, same formula;
    the C material has a constant density)."""
    if getattr(mat, "rho_amp", 0.0) != 0.0:
        raise ValueError("the C Fourier material has a constant density (rho_amp must be 0)")
    f = FourierMaterial()
    f.nmodes = mat.nmodes
    for i in range(mat.nmodes):
        for a in range(mat.dim):
            f.m[i][a] = int(mat.m[i, a])
        f.a[i] = float(mat.a[i])
        f.phi[i] = float(mat.phi[i])
    f.c0, f.amp, f.cmin, f.cmax, f.rho0 = mat.c0, mat.amp, mat.cmin, mat.cmax, mat.rho
    return f


class Mesh:
    """Owns a dgw_mesh.  Create with Mesh(...) from explicit nodes or Mesh.box(...)."""

    def __init__(self, dim, degree, geo_nodes, neighbors, material, flux=FLUX_UPWIND, precision=FP64,
                 device=0, max_batch=1, geo_degree=0, face_orient=None, storage_basis=BASIS_GL, plane_waves=None):
        """plane_waves: rows (A, k1, k2, k3, omega, phi, Z), the exterior state of BC_PRESCRIBED faces."""
        nodes = np.ascontiguousarray(geo_nodes, dtype=np.float64)
        nb = np.ascontiguousarray(neighbors, dtype=np.int64)
        fo = None if face_orient is None else np.ascontiguousarray(face_orient, dtype=np.int32)
        if fo is not None and fo.shape != nb.shape:
            raise ValueError("face_orient must have the shape of neighbors")
        ctx = None
        if isinstance(material, FourierMaterial):
            self._ctx = material
            self._cb = FOURIER_MATERIAL_FN
            ctx = C.cast(C.pointer(material), C.c_void_p)
        else:
            self._cb = material if isinstance(material, MATERIAL_FN) else material_callback(material)
        d = MeshDesc(dim=dim, degree=degree, n_cells=nodes.shape[0], geo_degree=geo_degree,
                     geo_nodes=_dptr(nodes), neighbors=nb.ctypes.data_as(C.POINTER(C.c_int64)),
                     face_orient=None if fo is None else fo.ctypes.data_as(C.POINTER(C.c_int)), material=self._cb, material_ctx=ctx, flux=flux, precision=precision,
                     device=device, max_batch=max_batch, storage_basis=storage_basis)
        if plane_waves is not None:
            rows = np.atleast_2d(np.asarray(plane_waves, dtype=np.float64))
            self._pw = (PlaneWave * len(rows))()
            for j, r in enumerate(rows):
                self._pw[j] = PlaneWave(r[0], (C.c_double * 3)(r[1], r[2], r[3]), r[4], r[5], r[6])
            d.plane_waves = C.cast(self._pw, C.POINTER(PlaneWave))
            d.n_plane_waves = len(rows)
        h = C.c_void_p()
        check(lib.dgw_mesh_create(C.byref(d), C.byref(h)), "dgw_mesh_create")
        self.h = h
        self._finish()

    @classmethod
    def box(cls, dim, ncell, degree, amp, material, flux=FLUX_UPWIND, precision=FP64, device=0, max_batch=1,
            storage_basis=BASIS_GL):
        self = cls.__new__(cls)
        if isinstance(material, FourierMaterial):
            self._ctx = material
            self._cb = FOURIER_MATERIAL_FN
            ctx = C.cast(C.pointer(material), C.c_void_p)
        else:
            self._cb = material_callback(material)
            ctx = None
        h = C.c_void_p()
        check(lib.dgw_mesh_create_box(dim, ncell, degree, amp, self._cb, ctx, flux, precision, device, max_batch,
                                      storage_basis, C.byref(h)), "dgw_mesh_create_box")
        self.h = h
        self._finish()
        return self

    def _finish(self):
        info = MeshInfo()
        check(lib.dgw_mesh_info_get(self.h, C.byref(info)), "dgw_mesh_info_get")
        self.info = info
        self.dim, self.degree, self.n_cells = info.dim, info.degree, info.n_cells
        self.np = info.nodes_per_cell
        self.shape = (info.n_cells, info.n_comp, info.nodes_per_cell)

    def close(self):
        if getattr(self, "h", None):
            lib.dgw_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self, what):
        d, nc, n = self.dim, self.n_cells, self.degree + 1
        if what == GET_NODE_COORDS:
            shape = (nc, self.np, d)
        elif what == GET_CELL_METRIC:
            shape = (nc, d * d + 2, self.np)
        elif what == GET_FACE:
            shape = (nc, 2 * d, d + 2, n ** (d - 1))
        else:
            m = self.info.level_points[what - GET_LEVEL0]
            shape = (nc, d * d + 2, m ** d)
        out = np.empty(shape)
        check(lib.dgw_mesh_get(self.h, what, _dptr(out), out.size), "dgw_mesh_get")
        return out

    def new_state(self, B=1):
        return torch.zeros((B,) + self.shape, dtype=torch.float64, device="cuda")

    def work(self, B=1):
        return torch.empty((2 * B,) + self.shape, dtype=torch.float64, device="cuda")

    def apply(self, u, out=None, B=None, stream=None):
        B = B or (u.shape[0] if u.dim() == 4 else 1)
        out = torch.empty_like(u) if out is None else out
        check(lib.dgw_operator_apply(self.h, _tptr(u), _tptr(out), B, _stream(stream)), "dgw_operator_apply")
        return out

    def step_lsrk(self, u, t0, dt, nsteps, work=None, sources=None, B=None, stream=None, scheme=LSRK54):
        B = B or (u.shape[0] if u.dim() == 4 else 1)
        work = self.work(B) if work is None else work
        check(lib.dgw_step_lsrk(self.h, scheme, t0, dt, nsteps, _tptr(u), _tptr(work), B,
                                sources.h if sources else None, _stream(stream)), "dgw_step_lsrk")
        return u

    def step_ader(self, u, t0, dt, nsteps, work=None, sources=None, B=None, flags=ADER_REDUCE, stream=None):
        B = B or (u.shape[0] if u.dim() == 4 else 1)
        work = self.work(B) if work is None else work
        check(lib.dgw_step_ader(self.h, flags, t0, dt, nsteps, _tptr(u), _tptr(work), B,
                                sources.h if sources else None, _stream(stream)), "dgw_step_ader")
        return u

    def step_ader_noalloc(self, u, t0, dt, nsteps, sources=None, B=None, flags=ADER_REDUCE, stream=None):
        """ADER steps with the work registers in the library's static device scratch."""
        B = B or (u.shape[0] if u.dim() == 4 else 1)
        check(lib.dgw_step_ader_noalloc(self.h, flags, t0, dt, nsteps, _tptr(u), B,
                                        sources.h if sources else None, _stream(stream)), "dgw_step_ader_noalloc")
        return u

    def profile(self, u, scheme, t0, dt, nsteps, work=None, sources=None, B=None, ader_flags=0, stream=None):
        """Mean duration (ms) of one launch of each kernel over nsteps steps."""
        B = B or (u.shape[0] if u.dim() == 4 else 1)
        work = self.work(B) if work is None else work
        pr = Profile()
        check(lib.dgw_step_profile(self.h, scheme, ader_flags, t0, dt, nsteps, _tptr(u), _tptr(work), B,
                                   sources.h if sources else None, _stream(stream), C.byref(pr)), "dgw_step_profile")
        return {pr.names[i].value.decode(): (pr.ms[i], pr.launches[i]) for i in range(pr.n)}

    def autotune(self, B=1, stream=None):
        check(lib.dgw_autotune(self.h, B, _stream(stream)), "dgw_autotune")
        return self.launch_shape(0), self.launch_shape(1)

    def launch_shape(self, which, cells=0, threads=0):
        c, t = C.c_int(cells), C.c_int(threads)
        check(lib.dgw_launch_shape(self.h, which, C.byref(c), C.byref(t)), "dgw_launch_shape")
        return c.value, t.value

    def energy(self, u, B=None, stream=None):
        B = B or (u.shape[0] if u.dim() == 4 else 1)
        out = np.empty(B)
        check(lib.dgw_energy(self.h, _tptr(u), B, _dptr(out), _stream(stream)), "dgw_energy")
        return out

    def solve(self, u, scheme, t_end, courant=0.0, dt=0.0, t0=0.0, sources=None, use_graph=False,
              autotune=False, watchdog_every=0, watchdog_growth=10.0, ader_flags=0, work=None, B=None,
              stream=None):
        B = B or (u.shape[0] if u.dim() == 4 else 1)
        work = self.work(B) if work is None else work
        d = SolveDesc(scheme=scheme, ader_flags=ader_flags, courant=courant, dt=dt, t0=t0, t_end=t_end,
                      sources=sources.h if sources else None, use_graph=int(use_graph), autotune=int(autotune),
                      watchdog_every=watchdog_every, watchdog_growth=watchdog_growth, stream=_stream(stream))
        rep = SolveReport()
        check(lib.dgw_solve_batch(self.h, C.byref(d), _tptr(u), _tptr(work), B, C.byref(rep)), "dgw_solve_batch")
        return rep


class Sources:
    def __init__(self, mesh: Mesh, positions, frequency, t0=None, amplitude=None):
        pos = np.ascontiguousarray(positions, dtype=np.float64)
        n = pos.shape[0]
        f = np.ascontiguousarray(np.broadcast_to(np.asarray(frequency, dtype=np.float64), (n,)))
        t = None if t0 is None else np.ascontiguousarray(np.broadcast_to(np.asarray(t0, float), (n,)))
        a = None if amplitude is None else np.ascontiguousarray(np.broadcast_to(np.asarray(amplitude, float), (n,)))
        d = SourceDesc(n=n, position=_dptr(pos), frequency=_dptr(f), t0=_dptr(t) if t is not None else None,
                       amplitude=_dptr(a) if a is not None else None)
        h = C.c_void_p()
        check(lib.dgw_sources_create(mesh.h, C.byref(d), C.byref(h)), "dgw_sources_create")
        self.h = h
        self.mesh = mesh

    def close(self):
        if getattr(self, "h", None):
            lib.dgw_sources_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def basis_1d(n, what):
    out = np.empty(n * n if what >= 4 else n)
    check(lib.dgw_basis_1d(n, what, _dptr(out)), "dgw_basis_1d")
    return out.reshape(n, n) if what >= 4 else out


def serve(requests, device=0, budget_bytes=None, max_live=8, realtime=True, keep_states=False, progress=False):
    n = len(requests)
    arr = (Request * n)(*requests)
    res = (Result * n)()
    states = []
    if keep_states:
        for i, r in enumerate(requests):
            sz = lib.dgw_request_footprint(C.byref(r))
            ncell, k, dim = r.ncell, r.degree, r.dim
            dofs = ncell ** dim * (dim + 1) * (k + 1) ** dim
            buf = np.empty(dofs)
            states.append(buf)
            res[i].state_host = _dptr(buf)
            del sz
    if budget_bytes is None:
        free, _ = torch.cuda.mem_get_info(device)
        budget_bytes = 0.9 * free
    sd = ServerDesc(device=device, hbm_budget_bytes=float(budget_bytes), max_live=max_live, realtime=int(realtime),
                    progress=int(progress))
    rep = ServeReport()
    check(lib.dgw_serve(C.byref(sd), arr, n, res, C.byref(rep)), "dgw_serve")
    return rep, list(res), states
