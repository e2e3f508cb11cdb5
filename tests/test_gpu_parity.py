"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Bars (tests/tolerances.py): FP64 time steps from the same state and single
operator applications within 1e-12 relative, in the coefficient 2-norm and
element by element per component; FP32-split error stated against the
oracle.  Density and sound speed vary inside every cell.  Meshes span several workgroups with a ragged
last group; edge cases: a single periodic cell, k = 1 and k = 8, batches.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import Mesh as OMesh
from oracle import apply_operator, ader, norms, sources as osrc, timestep as ts
from oracle.operator import gl_to_gauss
from tolerances import STEP_TOL as TOL, op_tol

pytestmark = pytest.mark.gpu

# every mesh of these tests has a density varying inside the cells (a second
# seeded Fourier field, 0.7..1.3) besides the varying sound speed
RHO_AMP = 0.3


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def rel(a, b):
    return norms.rel_l2(a, b)


def close(got, want, tol, label=""):
    """Parity bar: the relative coefficient 2-norm difference, and element by
    element the largest |got - want| of each state component relative to the
    largest |want| of the state, are both below tol.  The components share
    one scale (the energy norm weighs them by rho and 1/(rho c^2), both
    near 1 here); a component much smaller than the others (the velocity of
    a pressure pulse) carries the rounding of its coupling to the larger
    one, so its own maximum is no scale for it.  The per-component ratios to
    their own maxima are logged beside.  The component axis is the
    second-to-last one ([cells][d+1][nodes] and [B][cells][d+1][nodes])."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    r = rel(got, want)
    nv = want.shape[-2]
    g = np.moveaxis(got, -2, 0).reshape(nv, -1)
    w = np.moveaxis(want, -2, 0).reshape(nv, -1)
    wmax = np.abs(w).max()
    diff = [np.abs(g[c] - w[c]).max() for c in range(nv)]
    e = max(diff) / wmax
    own = ", ".join(f"{diff[c] / max(np.abs(w[c]).max(), 1e-300):.1e}" for c in range(nv))
    say(f"parity {label}: rel_l2 {r:.2e} elementwise {e:.2e} (bar {tol:.1e}); per component / own max: {own}")
    assert r < tol and e < tol, (label, r, e, tol)


def build(B, dim, nc, k, amp, mat=None, flux=0, precision=0, max_batch=1, bc=None):
    mat = mat or W.FourierMaterial(11, dim=dim, rho_amp=RHO_AMP)
    nodes, nb = W.box_nodes(dim, nc, k, amp), W.box_neighbors(dim, nc, bc)
    gm = B.Mesh(dim, k, nodes, nb, mat, flux=flux, precision=precision, max_batch=max_batch)
    om = OMesh(dim, k, nodes, nb, mat)
    return gm, om


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


OP_CASES = [(2, 4, 3, 0.0, 0), (2, 5, 3, 0.05, 0), (2, 3, 1, 0.05, 0), (2, 3, 8, 0.05, 1), (3, 3, 2, 0.05, 0),
            (3, 3, 3, 0.05, 1), (3, 2, 5, 0.05, 0), (3, 1, 4, 0.05, 0), (3, 2, 7, 0.05, 0), (3, 2, 1, 0.0, 0)]


@pytest.mark.parametrize("dim,nc,k,amp,flux", OP_CASES)
def test_operator_fp64(gpu_lib, dim, nc, k, amp, flux):
    say("operator", dim, nc, k, amp, flux)
    gm, om = build(gpu_lib, dim, nc, k, amp, flux=flux)
    U = W.random_state(dim * 100 + k, om.nc * (dim + 1) * om.np_).reshape(om.nc, dim + 1, om.np_)
    got = gm.apply(to_dev(U)).cpu().numpy()
    want = apply_operator(om, U, flux="central" if flux else "upwind")
    close(got, want, op_tol(k, dim))


BC_CASES = [(2, 3, 3, 0.05, ("wall", "absorbing"), 0), (2, 3, 4, 0.05, ("wall", "wall"), 1),
            (3, 2, 3, 0.05, ("absorbing", "periodic", "wall"), 0), (3, 3, 2, 0.0, ("wall", "wall", "wall"), 1),
            (3, 2, 5, 0.05, ("absorbing", "absorbing", "absorbing"), 0)]


@pytest.mark.parametrize("dim,nc,k,amp,bc,flux", BC_CASES)
def test_operator_boundary_faces_fp64(gpu_lib, dim, nc, k, amp, bc, flux):
    """Wall and absorbing faces (exterior state from the own trace) against the oracle."""
    say("operator bc", dim, nc, k, amp, bc, flux)
    gm, om = build(gpu_lib, dim, nc, k, amp, flux=flux, bc=bc)
    U = W.random_state(dim * 10 + k + 1, (om.nc, dim + 1, om.np_))
    got = gm.apply(to_dev(U)).cpu().numpy()
    want = apply_operator(om, U, flux="central" if flux else "upwind")
    close(got, want, op_tol(k, dim))


@pytest.mark.parametrize("scheme", ["lsrk", "ader"])
def test_steps_with_boundary_faces(gpu_lib, scheme):
    say("steps bc", scheme)
    dim, nc, k = 3, 3, 3
    gm, om = build(gpu_lib, dim, nc, k, 0.05, bc=("wall", "absorbing", "periodic"))
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.1, 0.9, 0.5], 0.15))
    dt = 0.3 * gm.info.dt_unit
    u = to_dev(U)[None]
    want = U
    if scheme == "lsrk":
        gm.step_lsrk(u, 0.0, dt, 2)
        for s in range(2):
            want = ts.lsrk_step(lambda x, t: apply_operator(om, x), want, s * dt, dt)
    else:
        gm.step_ader(u, 0.0, dt, 2)
        for s in range(2):
            want = ader.ader_step(om, want, dt)
    close(u[0].cpu().numpy(), want, TOL)


@pytest.mark.parametrize("dim,nc,k,nsteps", [(2, 4, 3, 2), (3, 3, 3, 2), (3, 2, 5, 2), (3, 2, 6, 2), (3, 2, 7, 1),
                                              (3, 2, 8, 1)])
def test_lsrk_step_fp64(gpu_lib, dim, nc, k, nsteps):
    """LSRK(5,4) with the fused stage epilogue, up to k = 8 in 3D (the
    1024-thread operator at 9^3 points)."""
    say("lsrk", dim, nc, k)
    gm, om = build(gpu_lib, dim, nc, k, 0.05)
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.3] * dim, 0.15))
    U = U + 0.01 * W.random_state(7, U.shape)
    dt = 0.5 * gm.info.dt_unit
    u = to_dev(U)[None]
    gm.step_lsrk(u, 0.0, dt, nsteps)
    want = U
    for s in range(nsteps):
        want = ts.lsrk_step(lambda x, t: apply_operator(om, x), want, s * dt, dt)
    close(u[0].cpu().numpy(), want, TOL)


@pytest.mark.parametrize("scheme", [2, 3])
def test_lsrk_unfused_variants_match_fused(gpu_lib, scheme):
    """The ablation variants (operator sweep + separate merged or standard
    vector update) advance the same scheme: equal to the fused stages up to
    rounding, and to the oracle within the step bar."""
    say("lsrk unfused", scheme)
    gm, om = build(gpu_lib, 3, 3, 3, 0.05)
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.3] * 3, 0.15))
    U = U + 0.01 * W.random_state(9, U.shape)
    dt = 0.5 * gm.info.dt_unit
    a = to_dev(U)[None]
    b = to_dev(U)[None]
    gm.step_lsrk(a, 0.0, dt, 2)
    gm.step_lsrk(b, 0.0, dt, 2, scheme=scheme)
    close(b[0].cpu().numpy(), a[0].cpu().numpy(), 1e-13)
    want = U
    for s in range(2):
        want = ts.lsrk_step(lambda x, t: apply_operator(om, x), want, s * dt, dt)
    close(b[0].cpu().numpy(), want, TOL)
    src = gpu_lib.Sources(gm, W.random_points(3, 1, 3), frequency=4.0)
    with pytest.raises(gpu_lib.DgwError) as e:
        gm.step_lsrk(b, 0.0, dt, 1, scheme=scheme, sources=src)
    assert e.value.status == gpu_lib.EUNSUPPORTED
    prof = gm.profile(to_dev(U)[None], scheme, 0.0, dt, 2)
    assert set(prof) == {"operator_store", "vector_update"}
    assert prof["operator_store"][1] == 10 and prof["vector_update"][1] == 10


ORIENT_CASES = [(2, 3, 3, 0), (2, 4, 2, 1), (3, 3, 2, 0), (3, 2, 3, 1), (3, 2, 5, 0), (3, 3, 4, 0)]


@pytest.mark.parametrize("dim,nc,k,flux", ORIENT_CASES)
def test_operator_face_orientations_fp64(gpu_lib, dim, nc, k, flux):
    """Cells renumbered by reference-cell rotations (faces meet other face
    indices in all orientations): against the oracle on the same mesh, and
    against the standard mesh with the state renumbered the same way."""
    say("operator orient", dim, nc, k, flux)
    mat = W.FourierMaterial(13, dim=dim, rho_amp=RHO_AMP)
    nodes, nb, fo, rot = W.rotated_box(dim, nc, k, 0.05, seed=31 + k)
    gm = gpu_lib.Mesh(dim, k, nodes, nb, mat, flux=flux, face_orient=fo)
    om = OMesh(dim, k, nodes, nb, mat, face_orient=fo)
    U = W.random_state(dim * 7 + k, (om.nc, dim + 1, om.np_))
    got = gm.apply(to_dev(U)).cpu().numpy()
    close(got, apply_operator(om, U, flux="central" if flux else "upwind"), op_tol(k, dim))
    gs, _ = build(gpu_lib, dim, nc, k, 0.05, mat=mat, flux=flux)
    perms = [W.lattice_permutation(dim, k, r) for r in rot]
    inv = [np.argsort(pm) for pm in perms]
    U_std = np.stack([U[c][:, inv[c]] for c in range(om.nc)])
    R_std = gs.apply(to_dev(U_std)).cpu().numpy()
    close(got, np.stack([R_std[c][:, perms[c]] for c in range(om.nc)]), op_tol(k, dim))


@pytest.mark.parametrize("scheme", ["lsrk", "ader"])
def test_steps_with_face_orientations(gpu_lib, scheme):
    say("steps orient", scheme)
    dim, nc, k = 3, 3, 3
    mat = W.FourierMaterial(14, dim=dim, rho_amp=RHO_AMP)
    nodes, nb, fo, _ = W.rotated_box(dim, nc, k, 0.05, seed=41)
    gm = gpu_lib.Mesh(dim, k, nodes, nb, mat, face_orient=fo)
    om = OMesh(dim, k, nodes, nb, mat, face_orient=fo)
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.3, 0.6, 0.5], 0.15)) + 0.01 * W.random_state(9, (om.nc, dim + 1, om.np_))
    dt = 0.3 * gm.info.dt_unit
    u = to_dev(U)[None]
    want = U
    if scheme == "lsrk":
        gm.step_lsrk(u, 0.0, dt, 2)
        for s in range(2):
            want = ts.lsrk_step(lambda x, t: apply_operator(om, x), want, s * dt, dt)
    else:
        gm.step_ader(u, 0.0, dt, 2)
        for s in range(2):
            want = ader.ader_step(om, want, dt)
    close(u[0].cpu().numpy(), want, TOL)


GAUSS_CASES = [(2, 4, 3, None, False, 0), (2, 3, 8, ("wall", "absorbing"), False, 1), (2, 3, 1, None, False, 0),
               (3, 3, 2, None, False, 0), (3, 2, 5, None, False, 0), (3, 2, 7, ("absorbing", "periodic", "wall"), False, 0),
               (3, 1, 4, None, False, 1), (3, 3, 3, None, True, 0), (3, 2, 6, None, True, 1)]


def build_gauss(B, dim, nc, k, bc, orient, flux):
    mat = W.FourierMaterial(17, dim=dim, rho_amp=RHO_AMP)
    fo = None
    if orient:
        nodes, nb, fo, _ = W.rotated_box(dim, nc, k, 0.05, seed=37 + k)
    else:
        nodes, nb = W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc, bc)
    gm = B.Mesh(dim, k, nodes, nb, mat, flux=flux, face_orient=fo, storage_basis=B.BASIS_GAUSS)
    om = OMesh(dim, k, nodes, nb, mat, face_orient=fo)
    return gm, om


@pytest.mark.parametrize("dim,nc,k,bc,orient,flux", GAUSS_CASES)
def test_operator_gauss_basis_fp64(gpu_lib, dim, nc, k, bc, orient, flux):
    """Collocated Gauss storage basis (Sec. 3.1): against the oracle's direct
    Gauss-basis weak form, and against the GL kernel mapped by S."""
    say("operator gauss", dim, nc, k, bc, orient, flux)
    gm, om = build_gauss(gpu_lib, dim, nc, k, bc, orient, flux)
    fl = "central" if flux else "upwind"
    U = W.random_state(dim * 11 + k, (om.nc, dim + 1, om.np_))
    got = gm.apply(to_dev(U)).cpu().numpy()
    close(got, apply_operator(om, U, flux=fl, storage="gauss"), op_tol(k, dim))
    if not orient:
        gl, _ = build(gpu_lib, dim, nc, k, 0.05, mat=W.FourierMaterial(17, dim=dim, rho_amp=RHO_AMP), flux=flux, bc=bc)
        V = W.random_state(dim * 13 + k, (om.nc, dim + 1, om.np_))
        r_gl = gl.apply(to_dev(V)).cpu().numpy()
        r_g = gm.apply(to_dev(gl_to_gauss(om, V))).cpu().numpy()
        close(r_g, gl_to_gauss(om, r_gl), op_tol(k, dim))


@pytest.mark.parametrize("scheme", [0, 3])
def test_lsrk_gauss_basis_fp64(gpu_lib, scheme):
    say("lsrk gauss", scheme)
    dim, nc, k = 3, 3, 4
    gm, om = build_gauss(gpu_lib, dim, nc, k, ("wall", "periodic", "absorbing"), False, 0)
    U = gl_to_gauss(om, om.interpolate(lambda x: W.gaussian_pulse(x, [0.3, 0.6, 0.5], 0.15)))
    U = U + 0.01 * W.random_state(19, U.shape)
    dt = 0.3 * gm.info.dt_unit
    u = to_dev(U)[None]
    gm.step_lsrk(u, 0.0, dt, 2, scheme=scheme)
    want = U
    for s in range(2):
        want = ts.lsrk_step(lambda x, t: apply_operator(om, x, storage="gauss"), want, s * dt, dt)
    close(u[0].cpu().numpy(), want, TOL)


GAUSS_ADER_CASES = [(3, 3, 4, "reduce", None), (3, 2, 5, "reduce", ("wall", "periodic", "absorbing")),
                    (2, 3, 3, "reduce", None), (3, 2, 5, "noreduce", None), (3, 2, 5, "every_step", None),
                    (3, 2, 6, "every_third", None), (3, 2, 7, "reduce", None), (3, 2, 8, "reduce", None),
                    (2, 3, 1, "reduce", None), (3, 2, 3, "hdg", None), (2, 3, 5, "hdg", None)]


def _ader_variant(B, variant):
    """(step flags, oracle step) of an ADER variant"""
    if variant == "hdg":
        return B.ADER_HDG, lambda om, x, dt: ader.hdg_ader_step(om, x, dt)
    flags = {"reduce": 0, "noreduce": B.ADER_NOREDUCE, "every_step": B.ADER_REDUCE_EVERY_STEP,
             "every_third": B.ADER_REDUCE_EVERY_THIRD}[variant]
    kw = {"reduce": {}, "noreduce": {"reduce": False}, "every_step": {"period": 1},
          "every_third": {"period": 3}}[variant]
    return flags, lambda om, x, dt: ader.ader_step(om, x, dt, **kw)


@pytest.mark.parametrize("dim,nc,k,variant,bc", GAUSS_ADER_CASES)
def test_ader_gauss_basis_fp64(gpu_lib, dim, nc, k, variant, bc):
    """ADER with the state stored at the Gauss points (Sec. 3.1: the TCK needs
    no basis change in or out, the update sweep reads the neighbours' normal
    lines): two steps from the Gauss values of a state against the oracle's
    GL steps mapped to the Gauss points by its own S.  Every reduction period,
    HDG-ADER, the fused (k <= 5) and unfused (k = 7, 8) final phases."""
    say("ader gauss", dim, nc, k, variant, bc)
    B = gpu_lib
    gm, om = build_gauss(B, dim, nc, k, bc, False, 0)
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.6] * dim, 0.15))
    U = U + 0.01 * W.random_state(41 + k, U.shape)
    dt = 0.2 * gm.info.dt_unit
    flags, step = _ader_variant(B, variant)
    u = to_dev(gl_to_gauss(om, U))[None]
    gm.step_ader(u, 0.0, dt, 2, flags=flags)
    want = U
    for s in range(2):
        want = step(om, want, dt)
    close(u[0].cpu().numpy(), gl_to_gauss(om, want), TOL)


def test_gauss_basis_sources_energy_solver(gpu_lib):
    """The Gauss storage basis through every entry point: the energy of the
    same polynomial, point sources in LSRK and ADER steps against the oracle,
    the solver loop (hipGraph replay, energy watchdog) equal to the eager
    steps bitwise, and the per-kernel profile."""
    say("gauss sources energy solver")
    B = gpu_lib
    dim, nc, k, Bn = 3, 3, 3, 2
    mat = W.FourierMaterial(11, dim=dim, rho_amp=RHO_AMP)
    nodes, nb = W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc, None)
    gm = B.Mesh(dim, k, nodes, nb, mat, max_batch=Bn, storage_basis=B.BASIS_GAUSS)
    om = OMesh(dim, k, nodes, nb, mat)
    U = W.random_state(5, (om.nc, dim + 1, om.np_))
    e = gm.energy(to_dev(gl_to_gauss(om, U))[None])[0]
    assert abs(e - norms.energy_norm2(om, U)) < 1e-12 * abs(e)
    pos = W.random_points(31, Bn, dim)
    src = B.Sources(gm, pos, frequency=4.0, amplitude=[1.0, 2.5])
    dt, t0 = 0.2 * gm.info.dt_unit, 0.25
    for scheme in ("lsrk", "ader"):
        u = to_dev(np.zeros((Bn, om.nc, dim + 1, om.np_)))
        if scheme == "lsrk":
            gm.step_lsrk(u, t0, dt, 2, sources=src, B=Bn)
        else:
            gm.step_ader(u, t0, dt, 2, sources=src, B=Bn)
        for b in range(Bn):
            ps = osrc.PointSource(om, pos[b], osrc.Ricker(f=4.0, amp=[1.0, 2.5][b]))
            want = np.zeros((om.nc, dim + 1, om.np_))
            for s in range(2):
                t = t0 + s * dt
                if scheme == "lsrk":
                    want = ts.lsrk_step(lambda x, tt: apply_operator(om, x) + ps.rhs(om, tt), want, t, dt)
                else:
                    want = ader.ader_step(om, want, dt, source=ps, t=t)
            assert np.abs(want).max() > 0
            close(u[b].cpu().numpy(), gl_to_gauss(om, want), 1e-11, f"gauss sources {scheme} {b}")
    V = gl_to_gauss(om, om.interpolate(lambda x: W.gaussian_pulse(x, [0.4] * dim, 0.15)))
    a = to_dev(V)[None]
    c = to_dev(V)[None]
    gm.step_ader(a, 0.0, dt, 4)
    rep = gm.solve(c, B.ADER, t_end=4 * dt, dt=dt, use_graph=True, watchdog_every=2)
    assert rep.steps == 4
    assert torch.equal(a, c)
    prof = gm.profile(to_dev(V)[None], B.ADER, 0.0, dt, 1)
    assert set(prof) == {"tck", "operator_ader_update"}


def test_gauss_basis_fp32_split_error_stated(gpu_lib):
    """FP32-split arithmetic with the state at the Gauss points: parity
    unpinned, the error of three ADER and three LSRK(5,4) steps against the
    oracle's FP64 steps (mapped by S) stays at the single-precision level."""
    say("gauss fp32 split")
    B = gpu_lib
    dim, nc, k = 3, 3, 4
    mat = W.FourierMaterial(17, dim=dim, rho_amp=RHO_AMP)
    nodes, nb = W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc, None)
    gm = B.Mesh(dim, k, nodes, nb, mat, precision=B.FP32_SPLIT, storage_basis=B.BASIS_GAUSS)
    om = OMesh(dim, k, nodes, nb, mat)
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.5] * dim, 0.2))
    dt = 0.2 * gm.info.dt_unit
    for scheme in ("ader", "lsrk"):
        u = to_dev(gl_to_gauss(om, U))[None]
        w = U
        if scheme == "ader":
            gm.step_ader(u, 0.0, dt, 3)
            for s in range(3):
                w = ader.ader_step(om, w, dt)
        else:
            gm.step_lsrk(u, 0.0, dt, 3)
            for s in range(3):
                w = ts.lsrk_step(lambda x, t: apply_operator(om, x), w, s * dt, dt)
        err = rel(u[0].cpu().numpy(), gl_to_gauss(om, w))
        say(f"gauss fp32 split {scheme} 3 steps rel err", err)
        assert 0 < err < 1e-6


def _pw(dim):
    k = 2 * np.pi * np.array([1.0, 0.6, 0.3])[:dim]
    return W.PlaneWaves([[1.0, *np.pad(k, (0, 3 - dim)), 1.1 * np.linalg.norm(k), 0.4, 1.1],
                         [0.3, *np.pad(-0.5 * k[::-1], (0, 3 - dim)), 0.5 * np.linalg.norm(k), -1.0, 0.9]])


def build_prescribed(B, dim, nc, k, bc, flux=0, storage_basis=0):
    mat = W.FourierMaterial(23, dim=dim, rho_amp=RHO_AMP)
    nodes, nb = W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc, bc)
    pw = _pw(dim)
    gm = B.Mesh(dim, k, nodes, nb, mat, flux=flux, plane_waves=pw.w, storage_basis=storage_basis)
    return gm, OMesh(dim, k, nodes, nb, mat), pw


PRESCRIBED_CASES = [(2, 3, 3, ("prescribed", "prescribed"), 0), (2, 4, 5, ("prescribed", "wall"), 1),
                    (3, 2, 3, ("prescribed", "periodic", "absorbing"), 0), (3, 3, 2, ("prescribed",) * 3, 1),
                    (3, 2, 5, ("prescribed",) * 3, 0)]


@pytest.mark.parametrize("dim,nc,k,bc,flux", PRESCRIBED_CASES)
def test_operator_prescribed_faces_fp64(gpu_lib, dim, nc, k, bc, flux):
    """Prescribed exterior state (plane waves, evaluated at t = 0 by the operator)."""
    say("operator prescribed", dim, nc, k, bc, flux)
    gm, om, pw = build_prescribed(gpu_lib, dim, nc, k, bc, flux)
    U = W.random_state(dim * 17 + k, (om.nc, dim + 1, om.np_))
    got = gm.apply(to_dev(U)).cpu().numpy()
    want = apply_operator(om, U, flux="central" if flux else "upwind", exterior=lambda x: pw(x, 0.0))
    close(got, want, op_tol(k, dim))
    if dim == 3 and k == 3:  # and in the Gauss storage basis
        gg, _, _ = build_prescribed(gpu_lib, dim, nc, k, bc, flux, storage_basis=gpu_lib.BASIS_GAUSS)
        got = gg.apply(to_dev(U)).cpu().numpy()
        want = apply_operator(om, U, flux="central" if flux else "upwind", exterior=lambda x: pw(x, 0.0),
                              storage="gauss")
        close(got, want, op_tol(k, dim))


@pytest.mark.parametrize("scheme", ["lsrk", "lsrk_standard_vu", "ader"])
def test_steps_with_prescribed_faces(gpu_lib, scheme):
    """Exterior data at the LSRK stage times, integrated over the step for
    ADER; steps start at t0 != 0."""
    say("steps prescribed", scheme)
    B = gpu_lib
    dim, nc, k = 3, 3, 3
    gm, om, pw = build_prescribed(B, dim, nc, k, ("prescribed", "periodic", "prescribed"))
    U = om.interpolate(lambda x: pw(x, 0.0)) + 0.01 * W.random_state(29, (om.nc, dim + 1, om.np_))
    dt, t0 = 0.3 * gm.info.dt_unit, 0.37
    u = to_dev(U)[None]
    want = U
    if scheme == "ader":
        gm.step_ader(u, t0, dt, 3)
        for s in range(3):
            want = ader.ader_step(om, want, dt, exterior_integral=lambda x: pw.integral(x, t0 + s * dt, dt))
    else:
        gm.step_lsrk(u, t0, dt, 3, scheme=B.LSRK54 if scheme == "lsrk" else B.LSRK54_STANDARD_VU)
        for s in range(3):
            want = ts.lsrk_step(lambda x, t: apply_operator(om, x, exterior=lambda y: pw(y, t)), want,
                                t0 + s * dt, dt)
    close(u[0].cpu().numpy(), want, TOL)


@pytest.mark.parametrize("scheme", ["lsrk", "ader"])
def test_steps_with_prescribed_faces_gauss_basis(gpu_lib, scheme):
    """The same with the state at the Gauss points: exterior data at the LSRK
    stage times, integrated over the step for ADER (whose TCK sum stays in
    the GL basis)."""
    say("steps prescribed gauss", scheme)
    B = gpu_lib
    dim, nc, k = 3, 3, 3
    gm, om, pw = build_prescribed(B, dim, nc, k, ("prescribed", "periodic", "prescribed"),
                                  storage_basis=B.BASIS_GAUSS)
    U = om.interpolate(lambda x: pw(x, 0.0)) + 0.01 * W.random_state(31, (om.nc, dim + 1, om.np_))
    dt, t0 = 0.3 * gm.info.dt_unit, 0.37
    u = to_dev(gl_to_gauss(om, U))[None]
    want = U
    if scheme == "ader":
        gm.step_ader(u, t0, dt, 3)
        for s in range(3):
            want = ader.ader_step(om, want, dt, exterior_integral=lambda x: pw.integral(x, t0 + s * dt, dt))
    else:
        gm.step_lsrk(u, t0, dt, 3)
        for s in range(3):
            want = ts.lsrk_step(lambda x, t: apply_operator(om, x, exterior=lambda y: pw(y, t)), want,
                                t0 + s * dt, dt)
    close(u[0].cpu().numpy(), gl_to_gauss(om, want), TOL)


@pytest.mark.parametrize("scheme", [0, 1])
def test_prescribed_graph_replay_equals_eager(gpu_lib, scheme):
    """Captured steps take the step time from the device counter: the same
    bits as eager steps."""
    say("prescribed graph", scheme)
    B = gpu_lib
    gm, om, pw = build_prescribed(B, 3, 2, 4, ("prescribed", "prescribed", "periodic"))
    U = om.interpolate(lambda x: pw(x, 0.0))
    dt, t0, n = 0.25 * gm.info.dt_unit, 0.11, 6
    a = to_dev(U)[None]
    b = to_dev(U)[None]
    t_end = t0 + n * dt
    gm.solve(a, B.ADER if scheme else B.LSRK54, t_end=t_end, dt=dt, t0=t0, use_graph=True)
    dts = (t_end - t0) / n  # the step the solver takes
    if scheme:
        gm.step_ader(b, t0, dts, n)
    else:
        gm.step_lsrk(b, t0, dts, n)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(B.DgwError) as e:
        gm.step_ader(b, 0.0, dt, 1, flags=B.ADER_HDG)
    assert e.value.status == B.EUNSUPPORTED


@pytest.mark.parametrize("dim,nc,k,bc,nsteps", [(2, 4, 3, None, 2), (3, 3, 3, ("wall", "periodic", "absorbing"), 2),
                                               (3, 2, 5, None, 2), (2, 3, 8, None, 2), (3, 2, 1, None, 2),
                                               (3, 2, 6, None, 1), (3, 2, 7, None, 1), (3, 2, 8, None, 1)])
def test_lsrk59_step_fp64(gpu_lib, dim, nc, k, bc, nsteps):
    """LSRK5(9) in two-register form (nine fused stages) against the oracle's
    Butcher-form step of the same tableau."""
    say("lsrk59", dim, nc, k, bc)
    gm, om = build(gpu_lib, dim, nc, k, 0.05, bc=bc)
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.4] * dim, 0.15)) + 0.01 * W.random_state(27, (om.nc, dim + 1, om.np_))
    dt = 0.4 * gm.info.dt_unit
    u = to_dev(U)[None]
    gm.step_lsrk(u, 0.0, dt, nsteps, scheme=gpu_lib.LSRK59)
    want = U
    for s in range(nsteps):
        want = ts.lsrk59_step(lambda x, t: apply_operator(om, x), want, s * dt, dt)
    close(u[0].cpu().numpy(), want, TOL)
    # and it differs from the LSRK4(5) step
    v = to_dev(U)[None]
    gm.step_lsrk(v, 0.0, dt, nsteps)
    assert rel(v[0].cpu().numpy(), want) > 1e-12


def test_lsrk59_sources_prescribed_and_graph(gpu_lib):
    """LSRK5(9) with point sources (stage times c_i) and prescribed faces, and
    the solver's captured steps equal to eager steps."""
    say("lsrk59 sources")
    B = gpu_lib
    dim, nc, k, Bn = 3, 3, 3, 2
    mat = W.FourierMaterial(23, dim=dim, rho_amp=RHO_AMP)
    nodes, nb = W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc, ("prescribed", "periodic", "periodic"))
    pw = _pw(dim)
    gm = B.Mesh(dim, k, nodes, nb, mat, plane_waves=pw.w, max_batch=Bn)
    om = OMesh(dim, k, nodes, nb, mat)
    pos = W.random_points(33, Bn, dim)
    src = B.Sources(gm, pos, frequency=4.0, amplitude=[1.0, 2.5])
    dt, t0 = 0.3 * gm.info.dt_unit, 0.2
    U = np.zeros((Bn, om.nc, dim + 1, om.np_))
    u = to_dev(U)
    gm.step_lsrk(u, t0, dt, 2, sources=src, B=Bn, scheme=B.LSRK59)
    for b in range(Bn):
        ps = osrc.PointSource(om, pos[b], osrc.Ricker(f=4.0, amp=[1.0, 2.5][b]))
        want = U[b]
        for s in range(2):
            want = ts.lsrk59_step(lambda x, tt: apply_operator(om, x, exterior=lambda y: pw(y, tt)) + ps.rhs(om, tt),
                                  want, t0 + s * dt, dt)
        close(u[b].cpu().numpy(), want, 1e-11)
    a = to_dev(U)
    c = to_dev(U)
    t_end = t0 + 4 * dt
    rep = gm.solve(a, B.LSRK59, t_end=t_end, dt=dt, t0=t0, sources=src, use_graph=True, B=Bn)
    gm.step_lsrk(c, t0, rep.dt, rep.steps, sources=src, B=Bn, scheme=B.LSRK59)
    torch.cuda.synchronize()
    assert torch.equal(a, c)
    prof = gm.profile(to_dev(U), B.LSRK59, t0, dt, 1, sources=src, B=Bn)
    assert prof["operator_lsrk"][1] == 9


def test_feature_combinations(gpu_lib):
    """LSRK5(9) on a Gauss-basis mesh with prescribed faces; LSRK5(9) in
    FP32-split (error stated against FP64); the standard-VU LSRK variant on a
    Gauss-basis mesh with prescribed faces."""
    say("combinations")
    B = gpu_lib
    dim, nc, k = 3, 3, 3
    gm, om, pw = build_prescribed(B, dim, nc, k, ("prescribed", "periodic", "wall"),
                                  storage_basis=B.BASIS_GAUSS)
    U = gl_to_gauss(om, om.interpolate(lambda x: pw(x, 0.0))) + 0.01 * W.random_state(37, (om.nc, dim + 1, om.np_))
    dt, t0 = 0.3 * gm.info.dt_unit, 0.05
    for scheme, step in ((B.LSRK59, ts.lsrk59_step), (B.LSRK54_STANDARD_VU, ts.lsrk_step)):
        u = to_dev(U)[None]
        gm.step_lsrk(u, t0, dt, 2, scheme=scheme)
        want = U
        for s in range(2):
            want = step(lambda x, t: apply_operator(om, x, exterior=lambda y: pw(y, t), storage="gauss"), want,
                        t0 + s * dt, dt)
        close(u[0].cpu().numpy(), want, TOL, scheme)
    # FP32-split LSRK5(9): parity unpinned, error at the single-precision level
    g64, _ = build(B, dim, nc, k, 0.05)
    g32, _ = build(B, dim, nc, k, 0.05, precision=B.FP32_SPLIT)
    V = om.interpolate(lambda x: W.gaussian_pulse(x, [0.5] * dim, 0.15))
    a, b = to_dev(V)[None], to_dev(V)[None]
    dt = 0.3 * g64.info.dt_unit
    g64.step_lsrk(a, 0.0, dt, 3, scheme=B.LSRK59)
    g32.step_lsrk(b, 0.0, dt, 3, scheme=B.LSRK59)
    err = rel(b[0].cpu().numpy(), a[0].cpu().numpy())
    say("lsrk59 fp32 vs fp64 after 3 steps", err)
    assert 0 < err < 1e-5
    # FP32-split operator with prescribed faces: error at the single-precision level
    mat = W.FourierMaterial(23, dim=dim, rho_amp=RHO_AMP)
    nodes, nb = W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc, ("prescribed", "wall", "periodic"))
    gf = B.Mesh(dim, k, nodes, nb, mat, precision=B.FP32_SPLIT, plane_waves=pw.w)
    of = OMesh(dim, k, nodes, nb, mat)
    Y = W.random_state(41, (of.nc, dim + 1, of.np_))
    e32 = rel(gf.apply(to_dev(Y)).cpu().numpy(), apply_operator(of, Y, exterior=lambda y: pw(y, 0.0)))
    say("prescribed fp32 operator error", e32)
    assert e32 < 1e-5
    # batch of two on a Gauss-basis mesh: each member as its own run
    gb, ob, _ = build_prescribed(B, dim, nc, k, ("periodic", "periodic", "wall"), storage_basis=B.BASIS_GAUSS)
    gb2 = B.Mesh(dim, k, W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc, ("periodic", "periodic", "wall")),
                 W.FourierMaterial(23, dim=dim, rho_amp=RHO_AMP), plane_waves=pw.w, storage_basis=B.BASIS_GAUSS, max_batch=2)
    Z = np.stack([W.random_state(43, (ob.nc, dim + 1, ob.np_)), W.random_state(44, (ob.nc, dim + 1, ob.np_))])
    zz = to_dev(Z)
    gb2.step_lsrk(zz, 0.0, 0.2 * gb2.info.dt_unit, 2, B=2)
    for m in range(2):
        z1 = to_dev(Z[m])[None]
        gb.step_lsrk(z1, 0.0, 0.2 * gb.info.dt_unit, 2)
        assert torch.equal(zz[m], z1[0])


@pytest.mark.parametrize("dim,nc,k,reduce", [(2, 4, 3, True), (2, 3, 4, True), (3, 3, 3, True), (3, 2, 5, True),
                                             (3, 2, 4, False), (3, 2, 8, True), (2, 3, 1, True)])
def test_ader_step_fp64(gpu_lib, dim, nc, k, reduce):
    say("ader", dim, nc, k, reduce)
    gm, om = build(gpu_lib, dim, nc, k, 0.05)
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.6] * dim, 0.15))
    U = U + 0.01 * W.random_state(8, U.shape)
    dt = 0.2 * gm.info.dt_unit
    u = to_dev(U)[None]
    gm.step_ader(u, 0.0, dt, 1, flags=0 if reduce else 1)
    want = ader.ader_step(om, U, dt, reduce=reduce)
    close(u[0].cpu().numpy(), want, TOL)
    # the TCK sum alone is the difference of two steps' inputs: check the
    # whole step also over two steps
    gm.step_ader(u, dt, dt, 1, flags=0 if reduce else 1)
    want = ader.ader_step(om, want, dt, reduce=reduce)
    close(u[0].cpu().numpy(), want, TOL)


@pytest.mark.parametrize("dim,nc,k,bc", [(2, 4, 3, None), (3, 3, 3, None), (3, 2, 5, ("wall", "periodic", "absorbing")),
                                       (2, 3, 8, None)])
def test_hdg_ader_step_fp64(gpu_lib, dim, nc, k, bc):
    """HDG-ADER (Sec. 2.4): operator sweep, TCK from the DG derivative, update."""
    say("hdg ader", dim, nc, k, bc)
    gm, om = build(gpu_lib, dim, nc, k, 0.05, bc=bc)
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.6] * dim, 0.15))
    U = U + 0.01 * W.random_state(18, U.shape)
    dt = 0.2 * gm.info.dt_unit
    u = to_dev(U)[None]
    gm.step_ader(u, 0.0, dt, 2, flags=gpu_lib.ADER_HDG)
    want = U
    for s in range(2):
        want = ader.hdg_ader_step(om, want, dt)
    close(u[0].cpu().numpy(), want, TOL)
    # and it is not the plain ADER step
    v = to_dev(U)[None]
    gm.step_ader(v, 0.0, dt, 2)
    assert rel(v[0].cpu().numpy(), u[0].cpu().numpy()) > 1e-9


@pytest.mark.parametrize("dim,nc,k,period", [(2, 4, 3, 1), (3, 3, 5, 1), (3, 2, 8, 1), (3, 2, 7, 1),
                                           (2, 3, 5, 3), (3, 3, 5, 3), (3, 2, 8, 3)])
def test_ader_reduction_period_fp64(gpu_lib, dim, nc, k, period):
    """TCK with the reduction every derivative / every third (ablation of Sec. 3.3)."""
    say("ader period", dim, nc, k, period)
    B = gpu_lib
    gm, om = build(B, dim, nc, k, 0.05)
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.6] * dim, 0.15))
    U = U + 0.01 * W.random_state(19, U.shape)
    dt = 0.2 * gm.info.dt_unit
    flag = B.ADER_REDUCE_EVERY_STEP if period == 1 else B.ADER_REDUCE_EVERY_THIRD
    u = to_dev(U)[None]
    gm.step_ader(u, 0.0, dt, 2, flags=flag)
    want = U
    for s in range(2):
        want = ader.ader_step(om, want, dt, period=period)
    close(u[0].cpu().numpy(), want, TOL)
    v = to_dev(U)[None]
    gm.step_ader(v, 0.0, dt, 2)
    assert rel(v[0].cpu().numpy(), u[0].cpu().numpy()) > 1e-10


def test_ader_reduction_flags_rejected(gpu_lib):
    say("ader period flags")
    B = gpu_lib
    gm, om = build(B, 3, 2, 3, 0.05)
    u = to_dev(np.zeros((1,) + gm.shape))
    for flags, code in ((B.ADER_REDUCE_EVERY_STEP | B.ADER_NOREDUCE, B.EINVAL),
                        (B.ADER_REDUCE_EVERY_STEP | B.ADER_REDUCE_EVERY_THIRD, B.EINVAL),
                        (B.ADER_REDUCE_EVERY_THIRD | B.ADER_HDG, B.EUNSUPPORTED), (16, B.EINVAL)):
        with pytest.raises(B.DgwError) as e:
            gm.step_ader(u, 0.0, 1e-3, 1, flags=flags)
        assert e.value.status == code, flags
    src = B.Sources(gm, W.random_points(3, 1, 3), frequency=4.0)
    with pytest.raises(B.DgwError) as e:
        gm.step_ader(u, 0.0, 1e-3, 1, flags=B.ADER_REDUCE_EVERY_STEP, sources=src)
    assert e.value.status == B.EUNSUPPORTED


def test_hdg_ader_rejects_unsupported(gpu_lib):
    say("hdg ader unsupported")
    gm, om = build(gpu_lib, 3, 2, 3, 0.05)
    u = to_dev(np.zeros((1,) + gm.shape))
    with pytest.raises(gpu_lib.DgwError) as e:
        gm.step_ader(u, 0.0, 1e-3, 1, flags=gpu_lib.ADER_HDG | gpu_lib.ADER_NOREDUCE)
    assert e.value.status == gpu_lib.EUNSUPPORTED
    src = gpu_lib.Sources(gm, W.random_points(3, 1, 3), frequency=4.0)
    with pytest.raises(gpu_lib.DgwError) as e:
        gm.step_ader(u, 0.0, 1e-3, 1, flags=gpu_lib.ADER_HDG, sources=src)
    assert e.value.status == gpu_lib.EUNSUPPORTED
    prof = gm.profile(u, gpu_lib.ADER, 0.0, 1e-3, 2, ader_flags=gpu_lib.ADER_HDG)
    assert set(prof) == {"tck", "operator_ader_update", "operator_store"}


def test_batch_members_equal_solo_runs(gpu_lib):
    say("batch")
    dim, nc, k, Bn = 3, 3, 3, 3
    gm, om = build(gpu_lib, dim, nc, k, 0.05, max_batch=Bn)
    U = np.stack([W.random_state(20 + b, (om.nc, dim + 1, om.np_)) for b in range(Bn)])
    dt = 0.3 * gm.info.dt_unit
    ub = to_dev(U)
    gm.step_ader(ub, 0.0, dt, 2, B=Bn)
    ul = to_dev(U)
    gm.step_lsrk(ul, 0.0, dt, 1, B=Bn)
    for b in range(Bn):
        solo = to_dev(U[b])[None]
        gm.step_ader(solo, 0.0, dt, 2)
        assert torch.equal(solo[0], ub[b])
        solo = to_dev(U[b])[None]
        gm.step_lsrk(solo, 0.0, dt, 1)
        assert torch.equal(solo[0], ul[b])
    want = ader.ader_step(om, ader.ader_step(om, U[1], dt), dt)
    close(ub[1].cpu().numpy(), want, TOL)


def test_energy_matches_oracle(gpu_lib):
    say("energy")
    gm, om = build(gpu_lib, 3, 3, 3, 0.05)
    U = W.random_state(5, (om.nc, 4, om.np_))
    e = gm.energy(to_dev(U)[None])[0]
    assert abs(e - norms.energy_norm2(om, U)) < 1e-12 * abs(e)


@pytest.mark.parametrize("scheme", ["lsrk", "ader"])
def test_point_sources(gpu_lib, scheme):
    """Sources (not in the paper; parity against the oracle's reading of the injection)."""
    say("sources", scheme)
    dim, nc, k, Bn = 3, 3, 3, 2
    gm, om = build(gpu_lib, dim, nc, k, 0.05, max_batch=Bn)
    pos = W.random_points(31, Bn, dim)
    src = gpu_lib.Sources(gm, pos, frequency=4.0, amplitude=[1.0, 2.5])
    dt = 0.2 * gm.info.dt_unit
    t0 = 0.25
    U = np.zeros((Bn, om.nc, dim + 1, om.np_))
    u = to_dev(U)
    if scheme == "lsrk":
        gm.step_lsrk(u, t0, dt, 2, sources=src, B=Bn)
    else:
        gm.step_ader(u, t0, dt, 2, sources=src, B=Bn)
    for b in range(Bn):
        ps = osrc.PointSource(om, pos[b], osrc.Ricker(f=4.0, amp=[1.0, 2.5][b]))
        want = U[b]
        for s in range(2):
            t = t0 + s * dt
            if scheme == "lsrk":
                want = ts.lsrk_step(lambda x, tt: apply_operator(om, x) + ps.rhs(om, tt), want, t, dt)
            else:
                want = ader.ader_step(om, want, dt, source=ps, t=t)
        assert np.abs(want).max() > 0
        close(u[b].cpu().numpy(), want, 1e-11)


def test_fp32_split_error_stated(gpu_lib):
    """FP32-split: parity unpinned; the error against the FP64 oracle must stay
    at the single-precision level (stated bound 1e-5 relative per application)."""
    say("fp32 split")
    dim, nc, k = 3, 3, 4
    gm, om = build(gpu_lib, dim, nc, k, 0.05, precision=1)
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.5] * dim, 0.2))
    got = gm.apply(to_dev(U)[None]).cpu().numpy()[0]
    want = apply_operator(om, U)
    err = rel(got, want)
    say("fp32 split operator rel err", err)
    assert err < 1e-5
    u = to_dev(U)[None]
    dt = 0.2 * gm.info.dt_unit
    gm.step_ader(u, 0.0, dt, 3)
    w = U
    for s in range(3):
        w = ader.ader_step(om, w, dt)
    err = rel(u[0].cpu().numpy(), w)
    say("fp32 split ader 3 steps rel err", err)
    assert err < 1e-6
    # LSRK(5,4) in FP32-split against the oracle's FP64 steps
    u = to_dev(U)[None]
    gm.step_lsrk(u, 0.0, dt, 3)
    w = U
    for s in range(3):
        w = ts.lsrk_step(lambda x, t: apply_operator(om, x), w, s * dt, dt)
    err = rel(u[0].cpu().numpy(), w)
    say("fp32 split lsrk 3 steps rel err", err)
    assert 0 < err < 1e-6


@pytest.mark.parametrize("k", [7, 8])
def test_fp32_split_large_matrix_phases(gpu_lib, k):
    """FP32-split at k = 7 and 8, where each phase of the operator sweep loads
    its own matrix entries and visits its lines in unrolled rounds (another
    code path than at lower degrees): the operator, one LSRK(5,4) step and
    one ADER step against the FP64 oracle within the stated single-precision
    bound, 1e-5 relative."""
    say("fp32 split large matrices", k)
    dim, nc = 3, 2
    gm, om = build(gpu_lib, dim, nc, k, 0.05, precision=1)
    U = om.interpolate(lambda x: W.gaussian_pulse(x, [0.5] * dim, 0.2))
    U = U + 0.01 * W.random_state(11 + k, U.shape)
    got = gm.apply(to_dev(U)[None]).cpu().numpy()[0]
    err = rel(got, apply_operator(om, U))
    say("operator rel err", err)
    assert 0 < err < 1e-5
    dt = 0.5 * gm.info.dt_unit
    u = to_dev(U)[None]
    gm.step_lsrk(u, 0.0, dt, 1)
    err = rel(u[0].cpu().numpy(), ts.lsrk_step(lambda x, t: apply_operator(om, x), U, 0.0, dt))
    say("lsrk step rel err", err)
    assert 0 < err < 1e-5
    dt = 0.15 * gm.info.dt_unit
    u = to_dev(U)[None]
    gm.step_ader(u, 0.0, dt, 1)
    err = rel(u[0].cpu().numpy(), ader.ader_step(om, U, dt))
    say("ader step rel err", err)
    assert 0 < err < 1e-5


def test_invalid_arguments(gpu_lib):
    say("invalid")
    gm, om = build(gpu_lib, 2, 3, 2, 0.0)
    u = to_dev(np.zeros((1,) + gm.shape))
    with pytest.raises(gpu_lib.DgwError) as e:
        gm.apply(u, out=u)
    assert e.value.status == gpu_lib.EINVAL
    with pytest.raises(gpu_lib.DgwError) as e:
        gm.step_lsrk(u, 0.0, -1.0, 1)
    assert e.value.status == gpu_lib.EINVAL
    with pytest.raises(gpu_lib.DgwError) as e:
        gm.step_ader(to_dev(np.zeros((2,) + gm.shape)), 0.0, 0.1, 1, B=2)
    assert e.value.status == gpu_lib.EINVAL
