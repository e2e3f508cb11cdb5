"""CPU tests of the C ABI: the library loads and exports every function that
include/dgw.h declares; the host-side setup (built with DGW_DEVICE_NONE, no
GPU needed) agrees with the oracle's independent geometry; argument
validation returns the documented status codes.  No compute kernel runs."""
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import Mesh as OMesh
from oracle import basis, timestep as ts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_1805_03981_amd import binding
    return binding


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dgw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(dgw_[a-z0-9_]+)\s*\(", text))
    names.discard("dgw_material_fn")
    return sorted(n for n in names if not n.startswith("DGW_"))


def test_exports_every_declared_symbol(B):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(B.lib, n), n
    assert set(names) == set(B.EXPORTED)


def test_ceilings_library_exports_its_header():
    import ctypes
    text = open(os.path.join(ROOT, "include", "dgw_ceilings.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(dgw_[a-z0-9_]+)\s*\(", text)))
    assert names == ["dgw_ceiling_contract6", "dgw_ceiling_contract6_check", "dgw_ceiling_lds_read", "dgw_ceiling_mfma",
                     "dgw_ceiling_vector_fma"]
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1805_03981_amd", "libdgw_ceilings.so"))
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("n", [2, 4, 6, 9])
def test_basis_tables_match_oracle(B, n):
    xg, wg = basis.gauss(n)
    xgl, wgl = basis.gauss_lobatto(n)
    assert np.allclose(B.basis_1d(n, 0), xg, atol=1e-15) and np.allclose(B.basis_1d(n, 1), wg, atol=1e-15)
    assert np.allclose(B.basis_1d(n, 2), xgl, atol=1e-15) and np.allclose(B.basis_1d(n, 3), wgl, atol=1e-15)
    assert np.allclose(B.basis_1d(n, 4), basis.lagrange(xgl, xg), atol=1e-14)
    assert np.allclose(B.basis_1d(n, 5), basis.lagrange(xg, xgl), atol=1e-13)
    assert np.allclose(B.basis_1d(n, 6), basis.lagrange_deriv(xg, xg), atol=1e-12 * n * n)


@pytest.mark.parametrize("dim,nc,k,amp,bc", [(2, 3, 3, 0.05, None), (3, 2, 4, 0.05, None), (3, 2, 2, 0.0, None),
                                             (2, 3, 3, 0.05, ("wall", "absorbing")),
                                             (3, 3, 2, 0.05, ("absorbing", "periodic", "wall"))])
def test_host_setup_matches_oracle_geometry(B, dim, nc, k, amp, bc):
    mat = W.FourierMaterial(3, dim=dim, rho_amp=0.3)
    nodes, nb = W.box_nodes(dim, nc, k, amp), W.box_neighbors(dim, nc, bc)
    gm = B.Mesh(dim, k, nodes, nb, mat, device=B.DEVICE_NONE)
    om = OMesh(dim, k, nodes, nb, mat)
    cd = om.cell_data(np.arange(om.nc))
    G = gm.get(B.GET_CELL_METRIC)
    want = np.moveaxis((cd["wdet"][:, :, None, None] * cd["Jinv"]).reshape(om.nc, om.np_, dim * dim), 1, 2)
    assert np.abs(G[:, :dim * dim] - want).max() < 1e-13 * np.abs(want).max()
    muv = 1 / (cd["wdet"] * cd["rho"])
    mup = cd["rho"] * cd["c"] ** 2 / cd["wdet"]
    assert np.abs(G[:, dim * dim] - muv).max() < 1e-13 * muv.max()
    assert np.abs(G[:, dim * dim + 1] - mup).max() < 1e-13 * mup.max()
    F = gm.get(B.GET_FACE)
    for f in range(2 * dim):
        fd = om.face_data(np.arange(om.nc), f)
        assert np.abs(F[:, f, :dim] - np.moveaxis(fd["a"], 2, 1)).max() < 1e-14
        assert np.abs(F[:, f, dim] - fd["Zm"]).max() < 1e-14
        assert np.abs(F[:, f, dim + 1] - fd["Zp"]).max() < 1e-14
    h, c = ts.cell_h_and_c(om)
    assert abs(gm.info.dt_unit - (h / c).min() / k ** 1.5) < 1e-14 * gm.info.dt_unit
    x = gm.get(B.GET_NODE_COORDS)
    assert np.abs(x - om.node_points()).max() < 1e-14


def test_host_metric_of_small_cells(B):
    """Cells of the 48^3 box at degree 7 (each cell its own neighbour: only
    the cell metric is compared): the library's metric against the oracle's
    to 2e-13 relative, where the map's derivative sums would lose about
    4e-12 in absolute coordinates."""
    k, n = 7, 48
    nodes = W.box_nodes(3, n, k, 0.05)[[0, 1234, 50000, n ** 3 - 1]]
    nb = np.tile(np.arange(4)[:, None], (1, 6))
    mat = W.FourierMaterial(3, dim=3, rho_amp=0.3)
    gm = B.Mesh(3, k, nodes, nb, mat, device=B.DEVICE_NONE)
    om = OMesh(3, k, nodes, nb, mat)
    cd = om.cell_data(np.arange(om.nc))
    G = gm.get(B.GET_CELL_METRIC)
    want = np.moveaxis((cd["wdet"][:, :, None, None] * cd["Jinv"]).reshape(om.nc, om.np_, 9), 1, 2)
    assert np.abs(G[:, :9] - want).max() < 2e-13 * np.abs(want).max()
    muv = 1 / (cd["wdet"] * cd["rho"])
    assert np.abs(G[:, 9] - muv).max() < 2e-13 * muv.max()


@pytest.mark.parametrize("dim,nc,k", [(2, 3, 3), (3, 3, 2), (3, 2, 4)])
def test_host_setup_with_face_orientations(B, dim, nc, k):
    """Renumbered cells (faces meeting with other indices and orientations):
    the host face data, the neighbour impedance at the oriented point
    included, agrees with the oracle's."""
    mat = W.FourierMaterial(5, dim=dim, rho_amp=0.3)
    nodes, nb, fo, _ = W.rotated_box(dim, nc, k, 0.05, seed=17 + k)
    gm = B.Mesh(dim, k, nodes, nb, mat, device=B.DEVICE_NONE, face_orient=fo)
    om = OMesh(dim, k, nodes, nb, mat, face_orient=fo)
    F = gm.get(B.GET_FACE)
    for f in range(2 * dim):
        fd = om.face_data(np.arange(om.nc), f)
        assert np.abs(F[:, f, :dim] - np.moveaxis(fd["a"], 2, 1)).max() < 1e-14
        assert np.abs(F[:, f, dim] - fd["Zm"]).max() < 1e-14
        assert np.abs(F[:, f, dim + 1] - fd["Zp"]).max() < 1e-14
    # the impedance really varies along the faces, so a wrong point map shows
    assert np.abs(F[:, :, dim + 1] - F[:, :, dim + 1].mean(axis=-1, keepdims=True)).max() > 1e-3


def test_face_orientation_validation(B):
    mat = W.ConstantMaterial()
    nodes, nb, fo, _ = W.rotated_box(3, 2, 2, 0.0, seed=5)
    B.Mesh(3, 2, nodes, nb, mat, device=B.DEVICE_NONE, face_orient=fo)
    c, f = np.argwhere(fo % 8 != 0)[0]
    for bad_code in (fo[c, f] ^ 1, 6 * 8, -1, fo[c, f] // 8 * 8 + 8 if fo[c, f] // 8 < 5 else 0):
        bad = fo.copy()
        bad[c, f] = bad_code
        with pytest.raises(B.DgwError) as e:
            B.Mesh(3, 2, nodes, nb, mat, device=B.DEVICE_NONE, face_orient=bad)
        assert e.value.status == B.EINVAL, bad_code
    # 2D: only orientation 0 or 1
    nodes2, nb2, fo2, _ = W.rotated_box(2, 3, 2, 0.0, seed=6)
    bad = fo2.copy()
    bad[0, 0] = 8 * (bad[0, 0] // 8) + 2
    with pytest.raises(B.DgwError) as e:
        B.Mesh(2, 2, nodes2, nb2, mat, device=B.DEVICE_NONE, face_orient=bad)
    assert e.value.status == B.EINVAL
    with pytest.raises(ValueError):
        B.Mesh(2, 2, nodes2, nb2, mat, device=B.DEVICE_NONE, face_orient=fo2[:, :2])


def test_level_metric_matches_oracle(B):
    from oracle import ader
    dim, nc, k = 3, 2, 5
    mat = W.FourierMaterial(4, dim=dim, rho_amp=0.3)
    nodes, nb = W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc)
    gm = B.Mesh(dim, k, nodes, nb, mat, device=B.DEVICE_NONE)
    om = OMesh(dim, k, nodes, nb, mat)
    assert list(gm.info.level_points)[:gm.info.n_levels] == [6, 4, 2]
    for l, m in ((1, 4), (2, 2)):
        Gl = gm.get(B.GET_LEVEL0 + l)
        ld = ader.level_data(om, np.arange(om.nc), m)
        # stored: w detJ J^-1 and 1/(w detJ rho), rho c^2/(w detJ): their products are J^-1/rho, rho c^2 J^-1
        jr = Gl[:, :dim * dim] * Gl[:, dim * dim:dim * dim + 1]
        want = np.moveaxis(ld["Jinv"].reshape(om.nc, m ** dim, dim * dim), 1, 2) / ld["rho"][:, None, :]
        assert np.abs(jr - want).max() < 1e-13 * np.abs(want).max()
        jp = Gl[:, :dim * dim] * Gl[:, dim * dim + 1:dim * dim + 2]
        want = want * (ld["rho"] ** 2 * ld["c"] ** 2)[:, None, :]
        assert np.abs(jp - want).max() < 1e-13 * np.abs(want).max()
    # the density really varies inside the cells
    assert np.ptp(om.cell_data(np.arange(om.nc))["rho"], axis=1).min() > 1e-3


def test_footprint_and_validation(B):
    import ctypes as C
    r = B.Request(dim=3, ncell=8, degree=3, scheme=0, precision=0, t_end=0.1, courant=0.2, deform_amp=0.05)
    fp = B.lib.dgw_request_footprint(C.byref(r))
    state = 512 * 4 * 64 * 8
    assert fp > 3 * state
    r.scheme = B.LSRK59
    assert B.lib.dgw_request_footprint(C.byref(r)) == fp
    r.scheme = 7  # not a scheme
    assert B.lib.dgw_request_footprint(C.byref(r)) == -1
    r.scheme = 0
    r.degree = 9
    assert B.lib.dgw_request_footprint(C.byref(r)) == -1
    mat = W.ConstantMaterial()
    with pytest.raises(B.DgwError) as e:
        B.Mesh(3, 9, W.box_nodes(3, 2, 2, 0.0), W.box_neighbors(3, 2), mat, device=B.DEVICE_NONE)
    assert e.value.status == B.EUNSUPPORTED
    nb = W.box_neighbors(2, 3)
    nb[0, 1] = 5
    with pytest.raises(B.DgwError) as e:
        B.Mesh(2, 2, W.box_nodes(2, 3, 2, 0.0), nb, mat, device=B.DEVICE_NONE)
    assert e.value.status == B.EINVAL
    nb = W.box_neighbors(2, 3)
    nb[4, 2] = W.BC_WALL      # boundary on one side of an interior face: not conforming
    with pytest.raises(B.DgwError) as e:
        B.Mesh(2, 2, W.box_nodes(2, 3, 2, 0.0), nb, mat, device=B.DEVICE_NONE)
    assert e.value.status == B.EINVAL
    nb = W.box_neighbors(2, 3, ("wall", "periodic"))
    nb[nb == W.BC_WALL] = -4  # not a boundary code
    with pytest.raises(B.DgwError) as e:
        B.Mesh(2, 2, W.box_nodes(2, 3, 2, 0.0), nb, mat, device=B.DEVICE_NONE)
    assert e.value.status == B.EINVAL
    # a folded cell (negative Jacobian)
    nodes = W.box_nodes(2, 3, 2, 0.0)
    nodes[0] = nodes[0].reshape(3, 3, 2)[:, ::-1].reshape(9, 2)  # mirror x: det J < 0
    with pytest.raises(B.DgwError) as e:
        B.Mesh(2, 2, nodes, W.box_neighbors(2, 3), mat, device=B.DEVICE_NONE)
    assert e.value.status == B.EINVAL


def test_prescribed_faces_setup_and_validation(B):
    """Prescribed boundary faces: face data as the oracle's (exterior
    impedance = own), plane waves required and checked."""
    dim, nc, k = 3, 2, 3
    mat = W.FourierMaterial(8, dim=dim)
    nodes, nb = W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc, ("prescribed", "periodic", "wall"))
    pw = W.c3_literal_plane_wave().w
    gm = B.Mesh(dim, k, nodes, nb, mat, device=B.DEVICE_NONE, plane_waves=pw)
    om = OMesh(dim, k, nodes, nb, mat)
    F = gm.get(B.GET_FACE)
    for f in range(2 * dim):
        fd = om.face_data(np.arange(om.nc), f)
        assert np.abs(F[:, f, dim + 1] - fd["Zp"]).max() < 1e-14
        assert np.abs(F[:, f, :dim] - np.moveaxis(fd["a"], 2, 1)).max() < 1e-14
    for waves in (None, np.zeros((0, 7)), [[1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 1.0]], [[1.0, 1.0, 0.0, 0.0, 1.0, 0.0, 0.0]],
                  [[np.nan, 1.0, 0.0, 0.0, 1.0, 0.0, 1.0]], np.tile(pw, (9, 1))):
        with pytest.raises(B.DgwError) as e:
            B.Mesh(dim, k, nodes, nb, mat, device=B.DEVICE_NONE, plane_waves=waves)
        assert e.value.status == B.EINVAL, waves


def test_lsrk_coefficients_match_oracle(B):
    """The library refines the LSRK5(9) key with its own Newton solver; the
    result equals the oracle's tableau, and the LSRK4(5) table its rationals."""
    import ctypes as C
    out = np.empty(26)
    assert B.lib.dgw_lsrk_coefficients(B.LSRK59, out.ctypes.data_as(C.POINTER(C.c_double))) == 0
    a, b, c = ts.lsrk59_tableau()
    # the same root to a few units in the last place (it is conditioned ~1e3)
    assert np.abs(out[:8] - np.diag(a, -1)).max() < 5e-15
    assert np.abs(out[8:17] - b).max() < 5e-15
    assert np.abs(out[17:] - c).max() < 5e-15
    assert B.lib.dgw_lsrk_coefficients(B.LSRK54, out.ctypes.data_as(C.POINTER(C.c_double))) == 0
    want = [float(x) for x in ts.LSRK54_A + ts.LSRK54_B + ts.LSRK54_C]
    assert np.abs(out[:15] - want).max() < 1e-16
    assert B.lib.dgw_lsrk_coefficients(B.ADER, out.ctypes.data_as(C.POINTER(C.c_double))) == B.EINVAL


def test_storage_basis_validation(B):
    mat = W.ConstantMaterial()
    args = (2, 2, W.box_nodes(2, 3, 2, 0.0), W.box_neighbors(2, 3), mat)
    B.Mesh(*args, device=B.DEVICE_NONE, storage_basis=B.BASIS_GAUSS)
    B.Mesh(*args, device=B.DEVICE_NONE, storage_basis=B.BASIS_GAUSS, precision=B.FP32_SPLIT)
    with pytest.raises(B.DgwError) as e:
        B.Mesh(*args, device=B.DEVICE_NONE, storage_basis=2)
    assert e.value.status == B.EINVAL


def test_c_box_nodes_match_generator(B):
    """dgw_mesh_create_box and workloads.box_nodes describe the same mesh."""
    mat = W.FourierMaterial(9, dim=3)
    gm = B.Mesh.box(3, 3, 2, 0.05, B.fourier_material_struct(mat), device=B.DEVICE_NONE)
    om = OMesh(3, 2, W.box_nodes(3, 3, 2, 0.05), W.box_neighbors(3, 3), mat)
    assert np.abs(gm.get(B.GET_NODE_COORDS) - om.node_points()).max() < 1e-14
    G = gm.get(B.GET_CELL_METRIC)
    cd = om.cell_data(np.arange(om.nc))
    assert np.abs(G[:, 10] - cd["rho"] * cd["c"] ** 2 / cd["wdet"]).max() < 1e-12 * G[:, 10].max()
