"""GPU system tests: the batch solver with and without hipGraph replay, the
energy watchdog, the first workload end to end against its closed form, the
full-size 3D workloads on sampled cells against the oracle, and the request
server (each result identical alone and in the mix)."""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import Mesh as OMesh
from oracle import apply_operator, ader, norms, timestep as ts
from oracle.operator import gl_to_gauss
from tolerances import op_tol

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def test_standing_wave_2d_against_closed_form(gpu_lib):
    """2D periodic 8x8 affine quads, k=3, rho=c=1, upwind, LSRK(5,4), Cr 0.2, 200 steps."""
    say("c1 standing wave")
    B = gpu_lib
    k, nc = 3, 8
    gm = B.Mesh(2, k, W.box_nodes(2, nc, k, 0.0), W.box_neighbors(2, nc), W.ConstantMaterial())
    om = OMesh(2, k, W.box_nodes(2, nc, k, 0.0), W.box_neighbors(2, nc), W.ConstantMaterial())
    U0 = om.interpolate(lambda x: W.standing_wave_2d(x, 0.0))
    dt = 0.2 * gm.info.dt_unit
    assert abs(dt - 0.2 / 8 / 3 ** 1.5) < 1e-15
    u = to_dev(U0)[None]
    rep = gm.solve(u, B.LSRK54, t_end=200 * dt, dt=dt)
    assert rep.steps == 200
    T = 200 * dt
    got = u[0].cpu().numpy()
    ep, ev = norms.l2_error(om, got, W.standing_wave_2d, T)
    say(f"c1: T={T:.4f} L2(p)={ep:.3e} L2(v)={ev:.3e}")
    assert ep < 2e-4 and ev < 3e-4
    # and the same 200 steps on the oracle
    want = U0
    for s in range(200):
        want = ts.lsrk_step(lambda x, t: apply_operator(om, x), want, s * dt, dt)
    assert norms.rel_l2(got, want) < 1e-11


@pytest.mark.parametrize("scheme", [0, 1])
def test_membrane_mode_in_wall_box(gpu_lib, scheme):
    """2D unit box with rigid walls, 8x8 curved quads, k = 3, rho = c = 1: the
    (1, 1) membrane mode to T = 0.3 against its closed form, and against the
    oracle's run of the same steps."""
    say("membrane", scheme)
    B = gpu_lib
    k, nc = 3, 8
    nodes, nb = W.box_nodes(2, nc, k, 0.05), W.box_neighbors(2, nc, ("wall", "wall"))
    gm = B.Mesh(2, k, nodes, nb, W.ConstantMaterial())
    om = OMesh(2, k, nodes, nb, W.ConstantMaterial())
    U0 = om.interpolate(lambda x: W.membrane_mode(x, 0.0))
    u = to_dev(U0)[None]
    rep = gm.solve(u, scheme, t_end=0.3, courant=0.2 if scheme == 0 else 0.1)
    got = u[0].cpu().numpy()
    ep, ev = norms.l2_error(om, got, W.membrane_mode, rep.steps * rep.dt)
    say(f"membrane scheme {scheme}: {rep.steps} steps, L2(p) {ep:.3e} L2(v) {ev:.3e}")
    assert ep < 3e-5 and ev < 4e-5
    want = U0
    for s in range(rep.steps):
        want = (ts.lsrk_step(lambda x, t: apply_operator(om, x), want, s * rep.dt, rep.dt) if scheme == 0
                else ader.ader_step(om, want, rep.dt))
    assert norms.rel_l2(got, want) < 1e-11


@pytest.mark.parametrize("scheme", [0, 1])
def test_graph_replay_equals_eager(gpu_lib, scheme):
    """dgw_solve_batch with a captured two-step hipGraph replayed many times
    gives bitwise the eager result (sources included: the step counter lives
    on the device)."""
    say("graph", scheme)
    B = gpu_lib
    dim, nc, k, Bn = 3, 4, 3, 2
    mat = W.FourierMaterial(2, dim=dim)
    gm = B.Mesh(dim, k, W.box_nodes(dim, nc, k, 0.05), W.box_neighbors(dim, nc), mat, max_batch=Bn)
    src = B.Sources(gm, W.random_points(5, Bn, dim), frequency=6.0)
    U = W.random_state(3, (Bn,) + gm.shape) * 0.1
    dt = 0.2 * gm.info.dt_unit
    nsteps = 9
    a = to_dev(U)
    b = to_dev(U)
    ra = gm.solve(a, scheme, t_end=0.1 + nsteps * dt, dt=dt, t0=0.1, sources=src, use_graph=False)
    rb = gm.solve(b, scheme, t_end=0.1 + nsteps * dt, dt=dt, t0=0.1, sources=src, use_graph=True)
    assert ra.steps == rb.steps == nsteps and ra.dt == rb.dt
    assert torch.equal(a, b)
    # explicit stepping from the same state agrees too
    c = to_dev(U)
    (gm.step_ader if scheme else gm.step_lsrk)(c, 0.1, ra.dt, nsteps, sources=src, B=Bn)
    assert torch.equal(a, c)


@pytest.mark.parametrize("k", [3, 5])
def test_launch_shapes_give_identical_bits(gpu_lib, k):
    """Every compiled launch shape (cells per workgroup) of the operator and of
    the TCK gives the same operator, LSRK and ADER results up to the rounding
    of a different instruction schedule (each cell's arithmetic does not
    depend on its neighbours in the workgroup, but each shape is its own
    compiled kernel, whose multiply-adds the compiler may contract
    differently); the autotuner only picks among them."""
    say("launch shapes", k)
    B = gpu_lib
    gm = B.Mesh(3, k, W.box_nodes(3, 3, k, 0.05), W.box_neighbors(3, 3), W.FourierMaterial(1, dim=3, rho_amp=0.3))
    U = W.random_state(1, (1,) + gm.shape)
    dt = 0.3 * gm.info.dt_unit
    cpw = sorted({gm.launch_shape(0)[0]} | {2 * gm.launch_shape(0)[0]} | {max(1, gm.launch_shape(0)[0] // 2)})
    shapes = []
    for c in cpw:
        try:
            gm.launch_shape(0, cells=c)
            gm.launch_shape(1, cells=c)
        except B.DgwError:
            continue
        shapes.append(c)
    assert len(shapes) >= 2, shapes
    res = []
    for c in shapes:
        gm.launch_shape(0, cells=c)
        gm.launch_shape(1, cells=c)
        assert gm.launch_shape(0)[0] == c and gm.launch_shape(1)[0] == c
        a = gm.apply(to_dev(U))
        ul = to_dev(U)
        gm.step_lsrk(ul, 0.0, dt, 2)
        ua = to_dev(U)
        gm.step_ader(ua, 0.0, dt, 2)
        res.append((a, ul, ua))
    for c, r in zip(shapes[1:], res[1:]):
        for name, x, y in zip(("operator", "lsrk", "ader"), res[0], r):
            d = ((x - y).abs().max() / x.abs().max()).item()
            say(f"shape {shapes[0]} vs {c}: {name} max difference {d:.1e}, bitwise {torch.equal(x, y)}")
            assert d < 1e-14
    gm.autotune(1)
    c = gm.launch_shape(0)[0]
    assert c in shapes
    assert torch.equal(gm.apply(to_dev(U)), res[shapes.index(c)][0])


def test_autotune_cache_file(gpu_lib, tmp_path, monkeypatch):
    """The autotuner appends its choice per (architecture, d, k, precision,
    basis, B, cells) to the JSON-lines file named by DGW_AUTOTUNE_CACHE and
    takes a matching line from there instead of timing."""
    import json
    say("autotune cache file")
    B = gpu_lib
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("DGW_AUTOTUNE_CACHE", str(path))
    mat = W.FourierMaterial(1, dim=3)
    gm = B.Mesh(3, 3, W.box_nodes(3, 5, 3, 0.05), W.box_neighbors(3, 5), mat)
    gm.autotune(1)
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert len(lines) == 1 and lines[0]["key"].endswith("|d3|k3|fp64|gl|B1|nc125")
    rec = lines[0]
    cpw = {0: 4, 1: 8}  # the two compiled shapes of 4^3-point cells
    assert gm.launch_shape(0)[0] == cpw[rec["op_store"]] and gm.launch_shape(1)[0] == cpw[rec["tck"]]
    assert gm.launch_shape(2)[0] == cpw[rec["op_lsrk"]] and gm.launch_shape(3)[0] == cpw[rec["op_ader_update"]]
    # a line for another mesh size, written by hand, is taken as it is
    key = rec["key"].replace("nc125", "nc216")
    with open(path, "a") as f:
        f.write(json.dumps({"key": key, "op_store": 1, "op_lsrk": 0, "op_ader_update": 1, "tck": 0}) + "\n")
    g6 = B.Mesh(3, 3, W.box_nodes(3, 6, 3, 0.05), W.box_neighbors(3, 6), mat)
    g6.autotune(1)
    assert [g6.launch_shape(w)[0] for w in range(4)] == [8, 4, 4, 8]
    assert len(path.read_text().splitlines()) == 2  # nothing timed, nothing appended


@pytest.mark.parametrize("Bn", [3, 10])
def test_member_block_operator_equals_grid_batch(gpu_lib, tmp_path, monkeypatch, Bn):
    """The member-block operator (8 batch members per workgroup, geometry
    loaded once) against the plain batch (one member per workgroup), selected
    through an autotune cache line: operator, LSRK and ADER steps agree to
    rounding; B = 10 leaves a ragged last block."""
    import json
    say("member block", Bn)
    B = gpu_lib
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("DGW_AUTOTUNE_CACHE", str(path))
    gm = B.Mesh(3, 3, W.box_nodes(3, 3, 3, 0.05), W.box_neighbors(3, 3), W.FourierMaterial(3, dim=3, rho_amp=0.3),
                max_batch=Bn)
    U = W.random_state(40 + Bn, (Bn,) + gm.shape)
    src = B.Sources(gm, W.random_points(41, Bn, 3), frequency=5.0)
    dt = 0.25 * gm.info.dt_unit

    def run():
        a = gm.apply(to_dev(U), B=Bn)
        ul = to_dev(U)
        gm.step_lsrk(ul, 0.1, dt, 2, sources=src, B=Bn)
        ua = to_dev(U)
        gm.step_ader(ua, 0.1, dt, 2, sources=src, B=Bn)
        torch.cuda.synchronize()
        return a, ul, ua

    plain = run()
    key = f"gfx950|d3|k3|fp64|gl|B{Bn}|nc27"
    path.write_text(json.dumps({"key": key, "op_store": 2, "op_lsrk": 3, "op_ader_update": 2, "tck": 0}) + "\n")
    gm.autotune(Bn)
    assert [gm.launch_shape(w)[0] for w in (4, 5, 6)] == [8, 8, 8]
    block = run()
    for name, x, y in zip(("operator", "lsrk", "ader"), plain, block):
        d = ((x - y).abs().max() / x.abs().max()).item()
        say(f"member block B={Bn}: {name} max difference {d:.1e}")
        assert d < 1e-14


def test_watchdog_checks_every_member(gpu_lib):
    """Member 0 at rest and member 1 unstable: the watchdog trips (it checks
    every member); a source-driven solve from rest at a stable step runs
    through (a zero initial energy is no reference for growth)."""
    say("watchdog members")
    B = gpu_lib
    gm = B.Mesh(2, 3, W.box_nodes(2, 4, 3, 0.0), W.box_neighbors(2, 4), W.ConstantMaterial(), max_batch=2)
    U = np.zeros((2,) + gm.shape)
    U[1] = W.random_state(2, gm.shape)
    with pytest.raises(B.DgwError) as e:
        gm.solve(to_dev(U), B.ADER, t_end=200 * 3.0 * gm.info.dt_unit, courant=3.0, watchdog_every=10, B=2)
    assert e.value.status == B.EUNSTABLE
    src = B.Sources(gm, W.random_points(4, 2, 2), frequency=6.0)
    u = to_dev(np.zeros((2,) + gm.shape))
    rep = gm.solve(u, B.ADER, t_end=0.3, courant=0.1, sources=src, watchdog_every=5, B=2)
    assert rep.steps > 20 and rep.energy_end > 0


def test_watchdog_trips_on_unstable_step(gpu_lib):
    """A time step far above the stability limit is reported as DGW_EUNSTABLE."""
    say("watchdog")
    B = gpu_lib
    gm = B.Mesh(2, 3, W.box_nodes(2, 4, 3, 0.0), W.box_neighbors(2, 4), W.ConstantMaterial())
    u = to_dev(W.random_state(2, (1,) + gm.shape))
    with pytest.raises(B.DgwError) as e:
        gm.solve(u, B.ADER, t_end=200 * 3.0 * gm.info.dt_unit, courant=3.0, watchdog_every=10)
    assert e.value.status == B.EUNSTABLE


def _sampled_parity(B, ncell, k, precision, tol, nsample=24, storage_basis=0):
    """Operator and one ADER step against the oracle on sampled cells; with
    storage_basis = Gauss the states go in and come out at the Gauss points
    and are compared with the oracle's GL results mapped there by its own S."""
    wl = W.c2_workload(ncell, k, 1805)
    nodes, nb = W.box_nodes(3, ncell, k, 0.05), W.box_neighbors(3, ncell)
    gm = B.Mesh(3, k, nodes, nb, B.fourier_material_struct(wl["material"]), precision=precision,
                storage_basis=storage_basis)
    om = OMesh(3, k, nodes, nb, wl["material"], cache=False)
    rng = np.random.default_rng(ncell * 10 + k)
    cells = np.unique(np.concatenate([rng.choice(om.nc, nsample, replace=False), [0, om.nc - 1]]))
    # smooth state: the pulse plus noise; each side interpolates the pulse at
    # its own GL node positions (the oracle only on the cells it needs)
    x = gm.get(B.GET_NODE_COORDS)
    noise = 0.01 * rng.standard_normal((om.nc, 4, om.np_))
    U = np.ascontiguousarray(np.moveaxis(wl["ic"](x), -1, 1)) + noise
    gm.autotune(1)
    # operator on a random state (no cancellation between volume and face
    # terms, so the relative difference measures rounding, not conditioning)
    Ur = rng.standard_normal((om.nc, 4, om.np_))
    gauss = storage_basis == B.BASIS_GAUSS
    to_storage = (lambda V: gl_to_gauss(om, V)) if gauss else (lambda V: V)
    L = gm.apply(to_dev(to_storage(Ur))[None])[0].cpu().numpy()
    want = to_storage(apply_operator(om, Ur, cells=cells))
    e_op = norms.rel_l2(L[cells], want)
    # one ADER step: TCK on the sampled cells and their face neighbours, then
    # the update on the sampled cells
    dt = 0.16 * gm.info.dt_unit
    u = to_dev(to_storage(U))[None]
    gm.step_ader(u, 0.0, dt, 1)
    nbrs = np.unique(np.concatenate([cells, om.neighbors[cells].ravel()]))
    Uo = np.zeros_like(U)
    Uo[nbrs] = om.interpolate(wl["ic"], cells=nbrs) + noise[nbrs]
    I = np.zeros_like(U)
    I[nbrs] = ader.tck(om, Uo, dt, cells=nbrs)
    want = to_storage(Uo[cells] + apply_operator(om, I, cells=cells))
    e_ad = norms.rel_l2(u[0].cpu().numpy()[cells], want)
    say(f"sampled {ncell}^3 k={k} prec={precision} basis={storage_basis}: operator {e_op:.2e}, "
        f"ADER step {e_ad:.2e}")
    assert e_op < max(tol, op_tol(k, 3)) and e_ad < tol


def test_full_size_c2_sampled(gpu_lib):
    """24^3 curved hexes, k=5 (1.19e7 DoF), in the launch shape the benchmark
    uses, on sampled cells."""
    say("c2 full size")
    _sampled_parity(gpu_lib, 24, 5, 0, 1e-12)


def test_full_size_c2_sampled_gauss_basis(gpu_lib):
    """The same with the state at the Gauss points, the storage the benchmark
    times ADER in."""
    say("c2 full size gauss")
    _sampled_parity(gpu_lib, 24, 5, 0, 1e-12, storage_basis=gpu_lib.BASIS_GAUSS)


def test_full_size_c3_sampled(gpu_lib):
    """48^3 curved hexes, k=7 (2.26e8 DoF), FP64 and FP32-split, sampled cells;
    FP64 also with the state at the Gauss points."""
    say("c3 full size")
    _sampled_parity(gpu_lib, 48, 7, 0, 1e-12, nsample=8)
    _sampled_parity(gpu_lib, 48, 7, 1, 1e-5, nsample=8)
    _sampled_parity(gpu_lib, 48, 7, 0, 1e-12, nsample=8, storage_basis=gpu_lib.BASIS_GAUSS)


def _request(B, seed, ncell, k, scheme, t_end, arrival):
    mat = W.FourierMaterial(seed, dim=3)
    r = B.Request(arrival_s=arrival, dim=3, ncell=ncell, degree=k, scheme=scheme, precision=1,
                  t_end=t_end, courant=0.8 * {0: 0.44, 1: 0.18, 4: 0.57}[scheme], deform_amp=0.05)
    r.material = B.fourier_material_struct(mat)
    c = W.random_points(seed + 1000, 1, 3)[0]
    for a in range(3):
        r.ic_center[a] = c[a]
    r.ic_width = 0.1
    return r


def test_serving_alone_equals_mix(gpu_lib):
    """Requests served concurrently give bitwise the states they give alone; a
    request larger than the budget fails with DGW_ENOMEM and the rest go on."""
    say("serve")
    B = gpu_lib
    reqs = [_request(B, 10 + i, n, k, (B.LSRK54, B.ADER, B.LSRK59)[i % 3], t, 0.002 * i)
            for i, (n, k, t) in enumerate([(4, 2, 0.05), (6, 3, 0.04), (5, 4, 0.03), (8, 2, 0.05), (4, 5, 0.02)])]
    big = _request(B, 99, 40, 8, 0, 0.1, 0.0)
    budget = 3 * max(B.lib.dgw_request_footprint(C.byref(r)) for r in reqs)
    assert B.lib.dgw_request_footprint(C.byref(big)) > budget
    rep, res, states = B.serve(reqs + [big], budget_bytes=budget, max_live=4, realtime=True, keep_states=True)
    say(f"serve: done {rep.n_done} failed {rep.n_failed} p50 {rep.p50_s:.4f}s p99 {rep.p99_s:.4f}s "
        f"{rep.dof_steps_per_s:.3e} DoF-steps/s")
    assert res[-1].status == B.ENOMEM
    assert rep.n_done == len(reqs) and rep.n_failed == 1
    for i, r in enumerate(reqs):
        assert res[i].status == 0 and res[i].steps > 0
        rep1, res1, st1 = B.serve([r], budget_bytes=budget, max_live=1, realtime=False, keep_states=True)
        assert res1[0].status == 0
        assert np.array_equal(states[i], st1[0])
        assert res[i].t_admit >= res[i].t_arrive - 1e-9 and res[i].t_done >= res[i].t_admit
    assert rep.p99_s >= rep.p50_s > 0


@pytest.mark.parametrize("scheme", [0, 1])
def test_served_request_matches_oracle(gpu_lib, scheme):
    """An FP64 request through dgw_serve (C box generator, C-built Gaussian
    initial state, the server's step count) against the oracle's steps on the
    same box from the same pulse, and against dgw_step_* on a mesh made by
    dgw_mesh_create_box."""
    say("served vs oracle", scheme)
    B = gpu_lib
    n, k, T = 3, 3, 0.03
    mat = W.FourierMaterial(61, dim=3)
    r = B.Request(arrival_s=0.0, dim=3, ncell=n, degree=k, scheme=scheme, precision=0, t_end=T,
                  courant=0.2, deform_amp=0.05)
    r.material = B.fourier_material_struct(mat)
    c = [0.3, 0.55, 0.7]
    for a in range(3):
        r.ic_center[a] = c[a]
    r.ic_width = 0.15
    rep, res, states = B.serve([r], budget_bytes=1 << 30, max_live=1, realtime=False, keep_states=True)
    assert res[0].status == 0
    steps = res[0].steps
    dt = T / steps
    got = states[0].reshape(n ** 3, 4, (k + 1) ** 3)
    om = OMesh(3, k, W.box_nodes(3, n, k, 0.05), W.box_neighbors(3, n), mat)
    U0 = om.interpolate(lambda x: W.gaussian_pulse(x, c, 0.15))
    want = U0
    for s in range(steps):
        want = (ts.lsrk_step(lambda x, t: apply_operator(om, x), want, s * dt, dt) if scheme == 0
                else ader.ader_step(om, want, dt))
    e = norms.rel_l2(got, want)
    say(f"served request scheme {scheme}: {steps} steps, rel err vs oracle {e:.2e}")
    assert steps >= 3 and e < 1e-12 * steps
    gm = B.Mesh.box(3, n, k, 0.05, B.fourier_material_struct(mat))
    u = to_dev(U0)[None]
    (gm.step_ader if scheme else gm.step_lsrk)(u, 0.0, dt, steps)
    assert norms.rel_l2(got, u[0].cpu().numpy()) < 1e-13


@pytest.mark.parametrize("scheme", [0, 1])
def test_graded_medium_against_closed_form(gpu_lib, scheme):
    """Density and sound speed graded along x inside every cell, impedance
    matched: the right-going wave on the curved 2D box (k = 3, 8x8 cells) to
    T = 0.15 against its closed form, and the same steps on the oracle."""
    say("graded medium", scheme)
    B = gpu_lib
    g = W.GradedMedium()
    k, nc = 3, 8
    nodes, nb = W.box_nodes(2, nc, k, 0.05), W.box_neighbors(2, nc)
    gm = B.Mesh(2, k, nodes, nb, g)
    om = OMesh(2, k, nodes, nb, g)
    U0 = om.interpolate(lambda x: g.wave(x, 0.0))
    u = to_dev(U0)[None]
    rep = gm.solve(u, scheme, t_end=0.15, courant=0.15)
    got = u[0].cpu().numpy()
    ep, ev = norms.l2_error(om, got, g.wave, 0.15)
    say(f"graded medium scheme {scheme}: {rep.steps} steps, L2(p) {ep:.3e} L2(v) {ev:.3e}")
    assert ep < 4e-4 and ev < 4e-4
    want = U0
    for s in range(rep.steps):
        want = (ts.lsrk_step(lambda x, t: apply_operator(om, x), want, s * rep.dt, rep.dt) if scheme == 0
                else ader.ader_step(om, want, rep.dt))
    assert norms.rel_l2(got, want) < 1e-11
