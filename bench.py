#!/usr/bin/env python
"""Throughput benchmark of the DG acoustic solver on one MI355X.

Workload (default, "c2"): periodic unit cube, 24^3 hexahedra curved by
x += 0.05 sin(2 pi x) sin(2 pi y) sin(2 pi z) (all coordinates), degree k = 5,
rho = 1, c = 1 + 0.3 * 8 seeded Fourier modes (clamped to [0.7, 1.3]),
upwind flux, Gaussian pressure pulse (width 0.05) at a seeded point:
1.19e7 DoF.  A step is one full time step of the hot path: the ADER step
(Taylor-Cauchy-Kowalevski sweep + fused operator/update sweep) or five fused
LSRK(5,4) stages.  `value` is the FP64 ADER throughput in DoF-steps/s with
the state resident in HBM, timed over exactly K steps launched back to back
(the solver's hipGraph time loop over the same K steps, capture included, is
reported beside it); the other scheme/precision variants are reported
beside it.  Also reported by default: per-kernel roofline (HIP events on the
launch stream), FP32-split error against FP64, the batch of 64 point
sources on 32^3 cells (k = 5, 500 ADER steps, FP32-split, hipGraph), a
bounded leg of the 48^3 k = 7 workload (throughput of both schemes and
precisions, one step against the oracle on sampled cells, plane-wave error
against the closed form), a serving trace of 24 requests drawn like the
serving workload (n^3 cells, n in [8, 48], k in 2..8, T in [0.1, 1], Poisson
arrivals at 0.8 x capacity, p50/p99), the time to solution at a fixed
pressure error (1e-6 relative at T = 0.5) against FP64 ADER and FP64 LSRK
references, the measured device ceilings (copy, triad, DGEMM, LDS, vector
FMA, MFMA) and the CPU FP64 oracle timed on a bounded sample of the same
workload.  Optional: the 200-request serving trace, the degree sweep
k = 1..8 on the paper's cube sizes, ablations.

    python bench.py [--steps K] [--warmup W] [--variants ader-fp64,...]
                    [--no-fixed-error] [--ablations] [--c3] [--sweep] [--no-ceilings] [--no-batched] [--no-c3]
                    [--no-serving] [--serving-full]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ["paper_1805_03981_amd/csrc/kernels.hpp", "paper_1805_03981_amd/csrc/dgw_params.hpp"]
# Critical Courant numbers of the paper's Table 2 (3D, k = 4 and k = 7) bracket
# k = 5; the runs use 0.9 of the smaller value.
CR = {"lsrk": 0.9 * 0.44, "lsrk59": 0.9 * 0.57, "ader": 0.9 * 0.18}
# storage basis of the state per scheme (0 = GL nodes, 1 = Gauss points,
# Sec. 3.1): the faster one on MI355X, measured both ways in the ablations.
# ADER: the TCK reads u at the Gauss points without a basis change and the
# update writes it there; LSRK: GL nodes (the Gauss-basis stage reads the
# neighbours' whole normal lines for its face traces).
BASIS = {"ader": 1, "lsrk": 0, "lsrk59": 0}


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


T_START = time.perf_counter()


def log(*a):
    print(f"[{time.perf_counter() - T_START:7.1f}s]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(dim, k, kernel):
    """Algorithmic HBM bytes per cell of one launch (FP64 state, FP64 metric),
    by the byte model of the measurement plan: a state register
    (d+1) n^d 8 B per pass, the metric w det J J^-1 (d^2 n^d doubles) and the
    two mass factors (2 n^d), the face geometry of the faces a cell owns
    (d faces, d+1 values per face point: d(d+1) n^(d-1) doubles) and the
    metric of the reduced Gauss sets of the TCK ((d^2+2) m^d per set)."""
    n = k + 1
    np_, nf, nc = n ** dim, n ** (dim - 1), dim + 1
    state = nc * np_ * 8
    cell_geo = (dim * dim + 2) * np_ * 8
    face_geo = 8 * dim * (dim + 1) * nf
    levels = sum((dim * dim + 2) * m ** dim * 8 for m in range(n - 2, 0, -2))
    if kernel == "operator_lsrk":     # read u, du; write du, u_next
        return 4 * state + cell_geo + face_geo
    if kernel == "operator_ader_update":  # read I, u_n; write u_next
        return 3 * state + cell_geo + face_geo
    if kernel == "tck":                  # read u; write I; metric of every Gauss set
        return 2 * state + cell_geo + levels
    raise ValueError(kernel)


def read_traffic(kernel, workload, precision):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_pmc.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_sources_sha256_16:\s*(\w+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def basis_map(u, n, what):
    """Apply the library's 1D matrix `what` (4: S, GL -> Gauss points; 5:
    S^-1) along the three directions of a device state [..., n^3] (x
    fastest)."""
    import torch
    from paper_1805_03981_amd import binding as dg
    M = torch.from_numpy(dg.basis_1d(n, what)).to(u.device)
    a = u.reshape(u.shape[:-1] + (n, n, n))
    for ax in (-1, -2, -3):
        a = torch.movedim(torch.matmul(torch.movedim(a, ax, -1).contiguous(), M.T.contiguous()), -1, ax)
    return a.reshape(u.shape).contiguous()


def to_gl_nodes(u, n):
    """Values at the Gauss points -> GL coefficients of the same polynomial."""
    return basis_map(u, n, 5)


def make_c2(B, precision, ncell=24, k=5, seed=1805, storage_basis=0):
    import numpy as np
    import torch
    import workloads as W
    from paper_1805_03981_amd import binding as dg
    wl = W.c2_workload(ncell, k, seed)
    mat = dg.fourier_material_struct(wl["material"])
    mesh = dg.Mesh(3, k, W.box_nodes(3, ncell, k, 0.05), W.box_neighbors(3, ncell), mat,
                   precision=dg.FP32_SPLIT if precision == "fp32" else dg.FP64, max_batch=B,
                   storage_basis=storage_basis)
    x = mesh.get(dg.GET_NODE_COORDS)
    u0 = np.ascontiguousarray(np.moveaxis(wl["ic"](x), -1, 1))
    if storage_basis == dg.BASIS_GAUSS:
        # the GL interpolant of the initial state, evaluated at the Gauss
        # points with the library's own 1D GL -> Gauss matrix
        n = k + 1
        S = dg.basis_1d(n, 4)
        a = u0.reshape(u0.shape[:2] + (n, n, n))
        for ax in (2, 3, 4):
            a = np.moveaxis(np.tensordot(a, S, axes=([ax], [1])), -1, ax)
        u0 = np.ascontiguousarray(a.reshape(u0.shape))
    return mesh, torch.from_numpy(u0).to("cuda")[None].contiguous(), wl


def run_variant(scheme, precision, steps, warmup):
    """Time exactly `steps` steps (dgw_step_*: the kernels of each step
    launched back to back on one stream) after `warmup` steps.  The same
    number of steps through the solver's time loop (dgw_solve_batch, the steps
    captured as a hipGraph once per call and replayed; the capture is inside
    that timing) is reported beside it."""
    import torch
    from paper_1805_03981_amd import binding as dg
    mesh, u0, wl = make_c2(1, precision, storage_basis=BASIS[scheme])
    mesh.autotune(1)
    dt = CR[scheme] * mesh.info.dt_unit
    sid = {"ader": dg.ADER, "lsrk": dg.LSRK54, "lsrk59": dg.LSRK59}[scheme]
    u = u0.clone()
    work = mesh.work(1)
    step = (lambda n: mesh.step_ader(u, 0.0, dt, n, work=work)) if scheme == "ader" else \
        (lambda n: mesh.step_lsrk(u, 0.0, dt, n, work=work, scheme=sid))
    step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the solver's time loop with hipGraph replay, same step count
    v = u0.clone()
    if warmup:
        mesh.solve(v, sid, t_end=warmup * dt, dt=dt, use_graph=True, work=work)
    torch.cuda.synchronize()
    tg = time.perf_counter()
    rep = mesh.solve(v, sid, t_end=steps * dt, dt=dt, use_graph=True, work=work)
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - tg
    if rep.steps != steps:
        raise RuntimeError(f"solve ran {rep.steps} steps, not {steps}")
    dofs = mesh.info.dofs
    prof = mesh.profile(u0.clone(), sid, 0.0, dt, min(steps, 20), work=work)
    res = dict(scheme=scheme, precision=precision, dofs=dofs, dt=dt, steps=steps, wall_s=wall,
               ms_per_step=1e3 * wall / steps, dof_steps_per_s=dofs * steps / wall,
               graph_solve_ms_per_step=1e3 * wall_graph / steps,
               kernels_ms={kname: ms for kname, (ms, _) in prof.items()},
               launch_shape={"operator": mesh.launch_shape(0), "operator_lsrk": mesh.launch_shape(2),
                             "operator_ader_update": mesh.launch_shape(3), "tck": mesh.launch_shape(1)})
    # steps to T = 0.5 at this Courant number: time to solution
    nsteps_T = int(-(-0.5 // dt))
    res["steps_to_T"] = nsteps_T
    res["time_to_T_s"] = nsteps_T * wall / steps
    return res, mesh, u


def rel_l2(a, b):
    """Relative difference of two device arrays in the plain coefficient 2-norm."""
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def fp32_error(steps=5):
    """FP32-split vs FP64 after `steps` steps of each scheme from the same state."""
    import torch
    out = {}
    for scheme in ("ader", "lsrk"):
        m64, u64, _ = make_c2(1, "fp64", storage_basis=BASIS[scheme])
        m32, u32, _ = make_c2(1, "fp32", storage_basis=BASIS[scheme])
        dt = CR[scheme] * m64.info.dt_unit
        for m, u in ((m64, u64), (m32, u32)):
            (m.step_ader if scheme == "ader" else m.step_lsrk)(u, 0.0, dt, steps)
        torch.cuda.synchronize()
        out[scheme] = rel_l2(u32, u64)
    return out


def cpu_baseline(target_s=15.0):
    """The oracle (test infrastructure) timed on a sample of the c2 workload:
    one ADER step (TCK + operator with its dense per-cell mass solve) on a
    contiguous block of cells, scaled to DoF-steps/s."""
    import numpy as np
    import workloads as W
    from oracle import Mesh, ader, apply_operator
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    wl = W.c2_workload(24, 5, 1805)
    m = Mesh(3, 5, W.box_nodes(3, 24, 5, 0.05), W.box_neighbors(3, 24), wl["material"], cache=False)
    U = np.zeros((m.nc, 4, m.np_))
    U[:] = 1e-3
    dt = CR["ader"] * 0.01

    def one(cells):
        ader.level_data(m, cells, 6)  # geometry of the sample (setup, untimed below)
        t = time.perf_counter()
        I = np.zeros_like(U)
        I[cells] = ader.tck(m, U, dt, cells=cells)
        apply_operator(m, I, cells=cells)
        return time.perf_counter() - t

    probe = np.arange(16)
    tp = one(probe)
    ncell = int(min(m.nc, max(16, target_s / tp * len(probe))))
    cells = np.arange(ncell)
    t = one(cells)
    dof = ncell * 4 * m.np_
    return {"value": dof / t, "unit": "DoF-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"one ADER step (TCK + operator, dense per-cell Cholesky mass solve) on {ncell} of "
                      f"{m.nc} cells of the 24^3 k=5 workload, {t:.1f} s; geometry of the sample cells "
                      f"recomputed inside the timed region (the oracle caches nothing at this size)"}


def batched_sources(B=64, steps=500, precision="fp32", ncell=32, k=5, seed=64, use_graph=True):
    """Many Ricker point sources (peak frequency 8, t0 = 1.2/8, seeded uniform
    positions) on one 32^3 curved mesh as a batch of B right-hand sides, zero
    initial state, ADER order k+1, autotuned launch shape, hipGraph-captured
    steps.  Returns aggregate DoF-steps/s."""
    import torch
    import workloads as W
    from paper_1805_03981_amd import binding as dg
    wl = W.c2_workload(ncell, k, 1805)
    mesh = dg.Mesh(3, k, W.box_nodes(3, ncell, k, 0.05), W.box_neighbors(3, ncell),
                   dg.fourier_material_struct(wl["material"]),
                   precision=dg.FP32_SPLIT if precision == "fp32" else dg.FP64, max_batch=B,
                   storage_basis=BASIS["ader"])
    src = dg.Sources(mesh, W.random_points(seed, B, 3), frequency=8.0)
    u = torch.zeros((B,) + mesh.shape, dtype=torch.float64, device="cuda")
    work = mesh.work(B)
    dt = CR["ader"] * mesh.info.dt_unit
    rep = mesh.solve(u, dg.ADER, t_end=steps * dt, dt=dt, sources=src, use_graph=use_graph, autotune=True,
                     work=work, B=B)
    e = mesh.energy(u, B=B)
    out = {"workload": f"{ncell}^3 curved hexes, k={k}, {B} Ricker sources (f=8) as batch members, ADER, "
                       f"{precision}, state at the {'Gauss points' if BASIS['ader'] else 'GL nodes'}, "
                       f"hipGraph={bool(use_graph)}, autotuned",
           "B": B, "steps": int(rep.steps), "wall_s": rep.wall_s, "dof_steps_per_s": rep.dof_steps_per_s,
           "dofs_total": mesh.info.dofs * B, "energy_member0_end": float(e[0]),
           "launch_shape": {"operator": mesh.launch_shape(0), "operator_lsrk": mesh.launch_shape(2),
                            "operator_ader_update": mesh.launch_shape(3), "tck": mesh.launch_shape(1)},
           "members_per_workgroup": {"operator": mesh.launch_shape(4)[0], "operator_lsrk": mesh.launch_shape(5)[0],
                                     "operator_ader_update": mesh.launch_shape(6)[0]}}
    del u, work, src, mesh
    torch.cuda.empty_cache()
    return out


def serving(nreq=24, seed=5, load=0.8, nmin=6, nmax=20, tmin=0.05, tmax=0.2, progress=False):
    """A Poisson stream of solve requests: seeded periodic curved boxes with
    n^3 cells (n log-uniform in [nmin, nmax]), k uniform in 2..8, LSRK or
    ADER, FP32-split, final time U[tmin, tmax], Cr = 0.8 Cr_crit; arrival
    rate = `load` x the measured capacity.  Reports p50/p99 latency."""
    import ctypes as C
    import numpy as np
    import workloads as W
    from paper_1805_03981_amd import binding as dg
    rng = np.random.default_rng(seed)
    reqs = []
    work = []
    for i in range(nreq):
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        k = int(rng.integers(2, 9))
        scheme = int(rng.integers(0, 2))
        t_end = float(rng.uniform(tmin, tmax))
        r = dg.Request(arrival_s=0.0, dim=3, ncell=n, degree=k, scheme=scheme, precision=1, t_end=t_end,
                       courant=0.8 * (0.44 if scheme == 0 else 0.18), deform_amp=0.05)
        r.material = dg.fourier_material_struct(W.FourierMaterial(seed * 1000 + i, dim=3))
        c = W.random_points(seed * 1000 + i, 1, 3)[0]
        for a in range(3):
            r.ic_center[a] = c[a]
        r.ic_width = 0.1
        reqs.append(r)
    # capacity: all requests at once, no arrival process
    if progress:
        log(f"[bench] serving: capacity pass over {nreq} requests")
    cap, _, _ = dg.serve(reqs, realtime=False, max_live=8, progress=progress)
    mean_s = cap.wall_s / nreq
    gaps = rng.exponential(mean_s / load, size=nreq)
    t = np.cumsum(gaps) - gaps[0]
    for r, a in zip(reqs, t):
        r.arrival_s = float(a)
    if progress:
        log(f"[bench] serving: Poisson arrivals at {load} x capacity")
    rep, res, _ = dg.serve(reqs, realtime=True, max_live=8, progress=progress)
    return {"workload": f"{nreq} requests, 3D curved periodic boxes n^3, n log-uniform [{nmin},{nmax}], k in 2..8, "
                        f"LSRK/ADER, FP32-split, T in [{tmin},{tmax}], Poisson arrivals at {load} x capacity",
            "p50_s": rep.p50_s, "p99_s": rep.p99_s, "dof_steps_per_s": rep.dof_steps_per_s,
            "max_wait_s": rep.max_wait_s, "n_done": rep.n_done, "n_failed": rep.n_failed,
            "capacity_dof_steps_per_s": cap.dof_steps_per_s, "wall_s": rep.wall_s}


def fixed_error(target=1e-5, T=0.5, iters=3, max_run_s=12.0):
    """Time to solution at a fixed error, against two FP64 references on the
    same mesh at 1/8 of their steps (0.9 of the critical Courant number):
    ADER, and LSRK(5,4) (which converges at fourth order to the semi-discrete
    solution).  For each scheme and precision and each reference, the largest
    step (at most that Courant number, rounded down to T/n) whose pressure at
    T differs from the reference by at most `target` (relative, plain
    coefficient 2-norm over the GL nodes, states kept at the Gauss points
    mapped there first): the step is halved until the
    target is met, then bisected in log(dt).  Runs are shared between the two
    searches where the steps coincide; runs longer than `max_run_s` are not
    started; a search that stops converging reports the smallest error.  The
    target (1e-5) sits above the distance between the two references
    (about 1e-6: the ADER solution approaches the semi-discrete one at first
    order in dt, its predictor being cell-local), which is reported beside
    it, so that neither reference favours its own scheme."""
    from paper_1805_03981_amd import binding as dg
    refs, out = {}, {"target_rel_l2_p": target, "T": T, "references": {}}
    for rs in ("ader", "lsrk"):
        mesh, u0, _ = make_c2(1, "fp64", storage_basis=BASIS[rs])
        mesh.autotune(1)
        u = u0.clone()
        rep = mesh.solve(u, dg.ADER if rs == "ader" else dg.LSRK54, t_end=T,
                         dt=CR[rs] * mesh.info.dt_unit / 8, use_graph=True)
        refs[rs] = (to_gl_nodes(u, 6) if BASIS[rs] else u)[0, :, 3, :].clone()
        out["references"][rs] = {"precision": "fp64", "dt": rep.dt, "steps": rep.steps}
        log(f"[bench] fixed error: {rs} reference, {rep.steps} steps in {rep.wall_s:.2f} s")
        del mesh, u, u0
    out["references"]["ader_vs_lsrk_rel_l2_p"] = rel_l2(refs["ader"], refs["lsrk"])
    for scheme, prec in (("ader", "fp64"), ("lsrk", "fp64"), ("lsrk59", "fp64"), ("ader", "fp32"), ("lsrk", "fp32")):
        key = f"{scheme}-{prec}"
        m, v0, _ = make_c2(1, prec, storage_basis=BASIS[scheme])
        m.autotune(1)
        sid = {"ader": dg.ADER, "lsrk": dg.LSRK54, "lsrk59": dg.LSRK59}[scheme]
        dt_max = CR[scheme] * m.info.dt_unit
        runs = {}

        def run(dt):
            if dt not in runs:
                v = v0.clone()
                r = m.solve(v, sid, t_end=T, dt=dt, use_graph=True)
                p = (to_gl_nodes(v, 6) if BASIS[scheme] else v)[0, :, 3, :]
                errs = {rs: rel_l2(p, ref) for rs, ref in refs.items()}
                runs[dt] = (r.dt, r.steps, r.wall_s, r.dof_steps_per_s, errs)
                log(f"[bench] fixed error {key}: dt {r.dt:.3e} ({r.steps} steps, {r.wall_s:.2f} s): rel L2(p) "
                    + ", ".join(f"vs {rs} {e:.3e}" for rs, e in errs.items()))
            return runs[dt]

        sec_per_step = run(dt_max)[2] / run(dt_max)[1]
        res = {}
        for rs in refs:
            err = lambda dt: run(dt)[4][rs]
            best = dt_max if err(dt_max) <= target else None
            lo = dt_max
            while best is None:
                nxt = lo / 2
                if T / nxt * sec_per_step > max_run_s:
                    break
                if err(nxt) <= target:
                    best = nxt
                elif err(nxt) > 0.7 * err(lo):   # no longer converging: an error floor
                    break
                lo = nxt
            if best is not None and best < dt_max:
                good, bad = best, min(dt_max, 2 * best)
                for _ in range(iters):
                    mid = (good * bad) ** 0.5
                    if err(mid) <= target:
                        good = best = mid
                    else:
                        bad = mid
            if best is None:
                res[f"vs_{rs}"] = {"reached": False, "smallest_error": min(r[4][rs] for r in runs.values())}
            else:
                rdt, steps, wall, rate, errs = run(best)
                res[f"vs_{rs}"] = {"reached": True, "dt": rdt, "courant": rdt / m.info.dt_unit, "steps": steps,
                                   "rel_l2_p": errs[rs], "time_to_solution_s": wall, "dof_steps_per_s": rate,
                                   "limited_by": "stability" if best == dt_max else "accuracy"}
        out[key] = res
        log(f"[bench] fixed error {key}: {res}")
        del m
    return out


def fixed_summary(fe):
    """Time to solution of each variant at the fixed error, against the FP64
    LSRK(5,4) reference, for the top of the line (None if not measured)."""
    if not fe:
        return None
    out = {"target_rel_l2_p": fe["target_rel_l2_p"], "T": fe["T"],
           "reference_distance_ader_vs_lsrk": fe["references"].get("ader_vs_lsrk_rel_l2_p")}
    for key, res in fe.items():
        if not isinstance(res, dict) or "vs_lsrk" not in res:
            continue
        r = res["vs_lsrk"]
        out[key] = ({"time_to_solution_s": r["time_to_solution_s"], "dof_steps_per_s": r["dof_steps_per_s"],
                     "courant": r["courant"], "rel_l2_p": r["rel_l2_p"], "limited_by": r["limited_by"]}
                    if r.get("reached") else {"reached": False, "error_floor": r.get("smallest_error")})
    return out


def c3_plane_wave(T=0.5, ncell=48, k=7):
    """48^3 curved hexes (amplitude 0.05), k = 7 (2.27e8 DoF), rho = c = 1,
    periodic plane wave p = cos(2 pi (x+y+z) - 2 pi sqrt3 t): both schemes
    and precisions to T at 0.9 of the critical Courant number; error against
    the closed form at the GL nodes (relative, plain 2-norm over all
    components) and throughput.  Then the non-periodic wave of the workload
    text with prescribed exterior data on the box faces, FP64."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1805_03981_amd import binding as dg
    out = {"ncell": ncell, "k": k, "T": T}
    for prec in ("fp64", "fp32"):
        mesh = dg.Mesh(3, k, W.box_nodes(3, ncell, k, 0.05), W.box_neighbors(3, ncell), W.ConstantMaterial(),
                       precision=dg.FP32_SPLIT if prec == "fp32" else dg.FP64)
        mesh.autotune(1)
        x = mesh.get(dg.GET_NODE_COORDS)
        u0 = torch.from_numpy(np.ascontiguousarray(np.moveaxis(W.plane_wave_3d(x, 0.0), -1, 1))).to("cuda")[None]
        exact = None
        for scheme in ("ader", "lsrk"):
            u = u0.clone()
            rep = mesh.solve(u, dg.ADER if scheme == "ader" else dg.LSRK54, t_end=T,
                             dt=CR[scheme] * mesh.info.dt_unit, use_graph=True)
            if exact is None or exact[0] != rep.steps * rep.dt:
                ex = np.ascontiguousarray(np.moveaxis(W.plane_wave_3d(x, rep.steps * rep.dt), -1, 1))
                exact = (rep.steps * rep.dt, torch.from_numpy(ex).to("cuda")[None])
            err = rel_l2(u, exact[1])
            out[f"{scheme}-{prec}"] = {"dofs": mesh.info.dofs, "steps": rep.steps, "dt": rep.dt,
                                       "wall_s": rep.wall_s, "dof_steps_per_s": rep.dof_steps_per_s,
                                       "rel_l2_error_vs_closed_form": err}
            log(f"[bench] c3 {scheme}-{prec}: {out[f'{scheme}-{prec}']}")
        del mesh, u0, u, exact
        torch.cuda.empty_cache()
    # the wave as the workload text states it, cos(2 pi (x+y+z)/sqrt3 - 2 pi t):
    # not periodic on the unit cube, so every boundary face takes the wave as
    # its prescribed exterior state (integrated over each step for ADER)
    pw = W.c3_literal_plane_wave()
    mesh = dg.Mesh(3, k, W.box_nodes(3, ncell, k, 0.05), W.box_neighbors(3, ncell, ("prescribed",) * 3),
                   W.ConstantMaterial(), plane_waves=pw.w)
    mesh.autotune(1)
    x = mesh.get(dg.GET_NODE_COORDS)
    u0 = torch.from_numpy(np.ascontiguousarray(np.moveaxis(pw(x, 0.0), -1, 1))).to("cuda")[None]
    for scheme in ("ader", "lsrk"):
        u = u0.clone()
        rep = mesh.solve(u, dg.ADER if scheme == "ader" else dg.LSRK54, t_end=T,
                         dt=CR[scheme] * mesh.info.dt_unit, use_graph=True)
        ex = torch.from_numpy(np.ascontiguousarray(np.moveaxis(pw(x, rep.steps * rep.dt), -1, 1))).to("cuda")[None]
        key = f"literal_prescribed_{scheme}-fp64"
        out[key] = {"dofs": mesh.info.dofs, "steps": rep.steps, "dt": rep.dt, "wall_s": rep.wall_s,
                    "dof_steps_per_s": rep.dof_steps_per_s, "rel_l2_error_vs_closed_form": rel_l2(u, ex)}
        log(f"[bench] c3 {key}: {out[key]}")
        del u, ex
    del mesh, u0
    torch.cuda.empty_cache()
    return out


def c3_bounded(steps=8, ncell=48, k=7, nsample=6):
    """48^3 curved hexes, k = 7 (2.27e8 DoF) within a bounded time.  (i) The
    2.4e4-cell workload's material (c = 8-mode Fourier field) and pulse:
    ADER and LSRK(5,4) in FP64 and FP32-split over `steps` steps at 0.9 of
    the critical Courant number (graph-replayed solve): DoF-steps/s, and the
    FP32-split state against the FP64 one after those steps; one ADER step
    from the pulse against the oracle on `nsample` sampled cells (the oracle
    evaluates the Taylor sum on them and their face neighbours), both
    precisions.  (ii) rho = c = 1, periodic plane wave: the error against the
    closed form after `steps` steps, both schemes and precisions."""
    import numpy as np
    import torch
    import workloads as W
    from oracle import Mesh as OMesh
    from oracle import ader, apply_operator
    from paper_1805_03981_amd import binding as dg
    wl = W.c2_workload(ncell, k, 1805)
    out = {"ncell": ncell, "k": k, "steps": steps, "courant": {s: CR[s] for s in ("ader", "lsrk")}}
    unit = dg.FourierMaterial()
    unit.nmodes, unit.c0, unit.amp, unit.cmin, unit.cmax, unit.rho0 = 1, 1.0, 0.0, 1.0, 1.0, 1.0
    rng = np.random.default_rng(48)
    om = None
    cells = None
    final = {}
    n = k + 1
    for prec in ("fp64", "fp32"):
        pid = dg.FP32_SPLIT if prec == "fp32" else dg.FP64
        for scheme in ("ader", "lsrk"):
            log(f"[bench] c3: {ncell}^3 k={k} {prec} mesh (Fourier material), {scheme}, "
                f"state at the {'Gauss points' if BASIS[scheme] else 'GL nodes'}")
            mesh = dg.Mesh.box(3, ncell, k, 0.05, dg.fourier_material_struct(wl["material"]), precision=pid,
                               storage_basis=BASIS[scheme])
            mesh.autotune(1)
            x = mesh.get(dg.GET_NODE_COORDS)
            U = np.ascontiguousarray(np.moveaxis(wl["ic"](x), -1, 1))
            u0 = torch.from_numpy(U).to("cuda")[None]
            if BASIS[scheme]:
                u0 = basis_map(u0, n, 4)
            u = u0.clone()
            rep = mesh.solve(u, dg.ADER if scheme == "ader" else dg.LSRK54, t_end=steps * CR[scheme] * mesh.info.dt_unit,
                             dt=CR[scheme] * mesh.info.dt_unit, use_graph=True)
            out[f"{scheme}-{prec}"] = {"dofs": mesh.info.dofs, "steps": rep.steps, "dt": rep.dt, "wall_s": rep.wall_s,
                                       "dof_steps_per_s": rep.dof_steps_per_s}
            final[(scheme, prec)] = u
            log(f"[bench] c3 {scheme}-{prec}: {out[f'{scheme}-{prec}']}")
            if scheme != "ader":
                del mesh, u0, u
                torch.cuda.empty_cache()
                continue
            # one ADER step from the pulse, sampled cells against the oracle
            if om is None:
                om = OMesh(3, k, W.box_nodes(3, ncell, k, 0.05), W.box_neighbors(3, ncell), wl["material"], cache=False)
                cells = np.unique(np.concatenate([rng.choice(om.nc, nsample, replace=False), [0, om.nc - 1]]))
                nbrs = np.unique(np.concatenate([cells, om.neighbors[cells].ravel()]))
                dt1 = CR["ader"] * mesh.info.dt_unit
                t0 = time.perf_counter()
                # the oracle's own interpolant of the pulse on the cells it needs
                Uo = np.zeros_like(U)
                Uo[nbrs] = om.interpolate(wl["ic"], cells=nbrs)
                I = np.zeros_like(U)
                I[nbrs] = ader.tck(om, Uo, dt1, cells=nbrs)
                want = Uo[cells] + apply_operator(om, I, cells=cells)
                out["oracle_sampled_step_s"] = time.perf_counter() - t0
            u = u0.clone()
            mesh.step_ader(u, 0.0, dt1, 1)
            got = (to_gl_nodes(u, n) if BASIS["ader"] else u)[0].cpu().numpy()[cells]
            out[f"ader_step_vs_oracle_{prec}"] = {
                "cells": len(cells), "rel_l2": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
                "max_abs_over_max": float(np.abs(got - want).max() / np.abs(want).max())}
            log(f"[bench] c3 ader step vs oracle {prec}: {out[f'ader_step_vs_oracle_{prec}']}")
            del mesh, u0, u
            torch.cuda.empty_cache()
    for scheme in ("ader", "lsrk"):
        out[f"fp32_vs_fp64_after_steps_{scheme}"] = rel_l2(final[(scheme, "fp32")], final[(scheme, "fp64")])
    del final
    torch.cuda.empty_cache()
    for prec in ("fp64", "fp32"):
        pid = dg.FP32_SPLIT if prec == "fp32" else dg.FP64
        for scheme in ("ader", "lsrk"):
            log(f"[bench] c3: {ncell}^3 k={k} {prec} mesh (rho = c = 1, plane wave), {scheme}")
            mesh = dg.Mesh.box(3, ncell, k, 0.05, unit, precision=pid, storage_basis=BASIS[scheme])
            x = mesh.get(dg.GET_NODE_COORDS)
            u = torch.from_numpy(np.ascontiguousarray(np.moveaxis(W.plane_wave_3d(x, 0.0), -1, 1))).to("cuda")[None]
            if BASIS[scheme]:
                u = basis_map(u, n, 4)
            rep = mesh.solve(u, dg.ADER if scheme == "ader" else dg.LSRK54, t_end=steps * CR[scheme] * mesh.info.dt_unit,
                             dt=CR[scheme] * mesh.info.dt_unit, use_graph=True)
            T = rep.steps * rep.dt
            ex = torch.from_numpy(np.ascontiguousarray(np.moveaxis(W.plane_wave_3d(x, T), -1, 1))).to("cuda")[None]
            got = to_gl_nodes(u, n) if BASIS[scheme] else u
            out[f"plane_wave_{scheme}-{prec}"] = {"T": T, "steps": rep.steps,
                                                  "rel_l2_error_vs_closed_form": rel_l2(got, ex)}
            log(f"[bench] c3 plane wave {scheme}-{prec}: {out[f'plane_wave_{scheme}-{prec}']}")
            del u, ex, got, mesh
            torch.cuda.empty_cache()
    return out


def ablations(steps=10, warmup=2):
    """The paper's ablations on the c2 workload, FP64: LSRK(5,4) with the
    vector update fused into the operator sweep, merged into one separate pass
    (the paper's optimized updater) or as three BLAS-1 passes (its standard
    one); ADER with the degree reduction every second derivative (Alg. 3),
    every derivative, every third and without, and the HDG-ADER variant (one
    more operator sweep per step); the storage basis of the Runge-Kutta
    operator (Sec. 3.1): GL nodes with the basis change inside the kernel
    against Lagrange polynomials in the Gauss points (no basis change,
    diagonal mass, whole neighbour lines read for the face traces), for the
    operator alone, the LSRK step and the ADER step.  Per variant: ms per step
    and the mean duration of each component."""
    import torch
    from paper_1805_03981_amd import binding as dg
    mesh, u0, _ = make_c2(1, "fp64")
    mesh.autotune(1)
    work = mesh.work(1)
    out = {}
    variants = [("lsrk_fused", dg.LSRK54, None), ("lsrk_merged_vu", dg.LSRK54_MERGED_VU, None),
                ("lsrk_standard_vu", dg.LSRK54_STANDARD_VU, None), ("ader_reduce", dg.ADER, dg.ADER_REDUCE),
                ("ader_noreduce", dg.ADER, dg.ADER_NOREDUCE),
                ("ader_reduce_every_step", dg.ADER, dg.ADER_REDUCE_EVERY_STEP),
                ("ader_reduce_every_third", dg.ADER, dg.ADER_REDUCE_EVERY_THIRD), ("ader_hdg", dg.ADER, dg.ADER_HDG)]
    for name, scheme, flags in variants:
        dt = CR["ader" if scheme == dg.ADER else "lsrk"] * mesh.info.dt_unit
        u = u0.clone()
        if scheme == dg.ADER:
            step = lambda n: mesh.step_ader(u, 0.0, dt, n, work=work, flags=flags)
        else:
            step = lambda n: mesh.step_lsrk(u, 0.0, dt, n, work=work, scheme=scheme)
        step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(steps)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        prof = mesh.profile(u0.clone(), scheme, 0.0, dt, 3, work=work, ader_flags=flags or 0)
        out[name] = {"ms_per_step": ms, "dof_steps_per_s": mesh.info.dofs / (ms * 1e-3),
                     "components_ms": {k: v[0] for k, v in prof.items()},
                     "launches_per_step": {k: v[1] / 3 for k, v in prof.items()}}
        log(f"[bench] ablation {name}: {out[name]}")
    # storage basis: the operator alone (dgw_operator_apply) and the fused LSRK step
    del work
    for basis_name, sb in (("gl", dg.BASIS_GL), ("gauss", dg.BASIS_GAUSS)):
        m2, v0, _ = (mesh, u0, None) if sb == dg.BASIS_GL else make_c2(1, "fp64", storage_basis=sb)
        m2.autotune(1)
        r = torch.empty_like(v0)
        for _ in range(warmup):
            m2.apply(v0, out=r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5 * steps):
            m2.apply(v0, out=r)
        torch.cuda.synchronize()
        ms_op = 1e3 * (time.perf_counter() - t0) / (5 * steps)
        out[f"operator_{basis_name}_basis"] = {"ms_per_apply": ms_op,
                                               "dof_per_s": m2.info.dofs / (ms_op * 1e-3)}
        log(f"[bench] ablation operator_{basis_name}_basis: {out[f'operator_{basis_name}_basis']}")
        if sb == dg.BASIS_GAUSS:
            w2 = m2.work(1)
            # the fused LSRK step and the ADER step with the state at the Gauss points
            for name, scheme in (("lsrk_fused_gauss_basis", dg.LSRK54), ("ader_gauss_basis", dg.ADER)):
                dt = CR["ader" if scheme == dg.ADER else "lsrk"] * m2.info.dt_unit
                u = v0.clone()
                step = (lambda n: m2.step_ader(u, 0.0, dt, n, work=w2)) if scheme == dg.ADER else \
                    (lambda n: m2.step_lsrk(u, 0.0, dt, n, work=w2))
                step(warmup)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                step(steps)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0) / steps
                prof = m2.profile(v0.clone(), scheme, 0.0, dt, 3, work=w2)
                out[name] = {"ms_per_step": ms, "dof_steps_per_s": m2.info.dofs / (ms * 1e-3),
                             "components_ms": {k: v[0] for k, v in prof.items()},
                             "launches_per_step": {k: v[1] / 3 for k, v in prof.items()}}
                log(f"[bench] ablation {name}: {out[name]}")
            del m2, v0, u, w2, r
            torch.cuda.empty_cache()
    return out


def degree_sweep(steps=5, warmup=1):
    """FP64 DoF-steps/s of both schemes against the degree on the paper's
    cube sizes: 40^3 slightly curved hexes (80^3 for k <= 3), the c2 material
    and pulse, 0.9 of the critical Courant number, each scheme in its
    storage basis."""
    import torch
    out = {}
    for k in range(1, 9):
        ncell = 80 if k <= 3 else 40
        row = {"ncell": ncell}
        for scheme in ("lsrk", "ader"):
            mesh, u0, _ = make_c2(1, "fp64", ncell=ncell, k=k, storage_basis=BASIS[scheme])
            mesh.autotune(1)
            row["dofs"] = mesh.info.dofs
            work = mesh.work(1)
            dt = CR[scheme] * mesh.info.dt_unit
            u = u0.clone()
            step = mesh.step_ader if scheme == "ader" else mesh.step_lsrk
            step(u, 0.0, dt, warmup, work=work)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step(u, 0.0, dt, steps, work=work)
            torch.cuda.synchronize()
            row[scheme] = mesh.info.dofs * steps / (time.perf_counter() - t0)
            del mesh, u0, work, u
            torch.cuda.empty_cache()
        log(f"[bench] sweep k={k}: {row}")
        out[k] = row
    return out


def ceilings():
    """Measured ceilings: device copy and triad bandwidth, FP64 GEMM rate, LDS
    read bandwidth (8- and 16-byte lanes, contiguous and at the 48-byte stride
    of 6-point FP64 lines), vector FMA and matrix-core rates, and the k = 5
    FP32 line contraction on the vector units and on the matrix cores."""
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    c = torch.ones_like(a)

    def timeit(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps
    tc = timeit(lambda: b.copy_(a))
    tt = timeit(lambda: torch.add(a, c, alpha=2.0, out=b))
    m = 8192
    A = torch.randn(m, m, dtype=torch.float64, device="cuda")
    tg = timeit(lambda: A @ A, reps=5)
    out = {"copy_GBps": 2 * n * 8 / tc / 1e9, "triad_GBps": 3 * n * 8 / tt / 1e9,
           "fp64_gemm_TFLOPs": 2 * m ** 3 / tg / 1e12}
    del a, b, c, A
    torch.cuda.empty_cache()
    # LDS, vector FMA and matrix-core rates from the microbenchmark library
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_1805_03981_amd", "libdgw_ceilings.so"))
    torch.cuda.synchronize()

    def rate(fn, *args):
        v = C.c_double(0.0)
        if fn(*args, C.byref(v)) != 0:
            raise RuntimeError(f"{fn.__name__} failed")
        return v.value

    for acc, stride, name in ((8, 8, "lds_read_b64_TBps"), (16, 16, "lds_read_b128_TBps"),
                              (8, 48, "lds_read_b64_stride48B_TBps"), (16, 48, "lds_read_b128_stride48B_TBps"),
                              (8, 56, "lds_read_b64_stride56B_TBps")):
        out[name] = rate(lib.dgw_ceiling_lds_read, acc, stride) / 1e12
    out["fp64_vector_fma_TFLOPs"] = rate(lib.dgw_ceiling_vector_fma, 1) / 1e12
    out["fp32_vector_fma_TFLOPs"] = rate(lib.dgw_ceiling_vector_fma, 0) / 1e12
    out["fp64_mfma_TFLOPs"] = rate(lib.dgw_ceiling_mfma, 1) / 1e12
    out["fp32_mfma_TFLOPs"] = rate(lib.dgw_ceiling_mfma, 0) / 1e12
    # the k = 5 FP32 line contraction itself, vector FMAs against matrix cores
    out["contract6_fp32_valu_Glines_per_s"] = rate(lib.dgw_ceiling_contract6, 0) / 1e9
    out["contract6_fp32_mfma_Glines_per_s"] = rate(lib.dgw_ceiling_contract6, 1) / 1e9
    out["contract6_mfma_vs_valu_max_rel_diff"] = rate(lib.dgw_ceiling_contract6_check)
    return out


def copy_calibration(mib):
    """A plain device copy of known size, for calibrating the HBM counters."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {mib} MiB three times")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variants", default="ader-fp64,lsrk-fp64,lsrk59-fp64,ader-fp32,lsrk-fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32 error measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving trace (24 requests)")
    ap.add_argument("--serving-full", action="store_true",
                    help="also serve 200 requests, n in [8, 48], k in 2..8, T in [0.1, 1] "
                         "(about half an hour; one line per finished request)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 32^3 k=5 batch of 64 point sources (500 ADER steps)")
    ap.add_argument("--no-c3", action="store_true", help="skip the bounded 48^3 k=7 leg")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the copy/triad/DGEMM, LDS, vector FMA and MFMA ceilings")
    ap.add_argument("--ablations", action="store_true",
                    help="also run the fused / merged / standard LSRK vector updates and ADER without reduction")
    ap.add_argument("--c3", action="store_true",
                    help="also run 48^3 k=7 curved hexes, c = 1 plane wave to T = 0.5: error and throughput")
    ap.add_argument("--sweep", action="store_true",
                    help="also run the degree sweep k = 1..8 on 40^3 (80^3 for k <= 3) curved hexes, FP64")
    ap.add_argument("--no-fixed-error", action="store_true",
                    help="skip the time-to-solution at a fixed error (relative L2(p) 1e-6 at T = 0.5)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the cells would shard "
              "by slabs with a face-trace exchange per operator sweep); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    variants = [v.split("-") for v in args.variants.split(",") if v]
    results = {}
    for scheme, prec in variants:
        log(f"[bench] {scheme}-{prec}: warmup {args.warmup}, timing {args.steps} steps")
        res, mesh, _ = run_variant(scheme, prec, args.steps, args.warmup)
        log(f"[bench] {scheme}-{prec}: {res['dof_steps_per_s']:.3e} DoF-steps/s, {res['ms_per_step']:.3f} ms/step "
            f"(graph-replayed solve {res['graph_solve_ms_per_step']:.3f}), kernels {res['kernels_ms']}")
        results[f"{scheme}-{prec}"] = res
        del mesh
        torch.cuda.empty_cache()
    head_key = "ader-fp64" if "ader-fp64" in results else next(iter(results))
    head = results[head_key]
    # dominant kernel of the headline variant
    per_step = {k: ms * (5 if k == "operator_lsrk" else 1) for k, ms in head["kernels_ms"].items()}
    dom = max(per_step, key=per_step.get)
    ncells = 24 ** 3
    bytes_launch = algorithmic_bytes(3, 5, dom) * ncells
    achieved = bytes_launch / (head["kernels_ms"][dom] * 1e-3) / 1e9
    traffic = read_traffic(dom, "hex24k5", head["precision"])
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                "traffic_over_algorithmic": None if traffic is None else traffic / bytes_launch,
                "algorithmic_bytes_per_launch": bytes_launch, "launch_ms": head["kernels_ms"][dom],
                "launch_ms_source": "HIP events around every launch of the kernel on its stream "
                                    "(dgw_step_profile), mean over the launches of min(steps, 20) steps"}
    kernels = {}
    for key, r in results.items():
        for kname, ms in r["kernels_ms"].items():
            b = algorithmic_bytes(3, 5, kname) * ncells
            kernels[f"{key}:{kname}"] = {"ms": ms, "GB/s": b / (ms * 1e-3) / 1e9,
                                         "frac_hbm": b / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    extras = {}
    if not args.no_extras and "ader-fp32" in results:
        log("[bench] FP32-split error vs FP64")
        extras["fp32_split_rel_err_5_steps"] = fp32_error()
    if not args.no_batched:
        log("[bench] batched sources")
        extras["batched_sources"] = batched_sources()
        log(f"[bench] batched: {extras['batched_sources']}")
    if not args.no_c3:
        log("[bench] 48^3 k=7 bounded leg")
        extras["c3"] = c3_bounded()
    if not args.no_serving:
        log("[bench] serving trace")
        extras["serving"] = serving(nreq=24, seed=5, nmin=8, nmax=48, tmin=0.1, tmax=1.0, progress=True)
        log(f"[bench] serving: {extras['serving']}")
    if args.serving_full:
        log("[bench] full serving trace")
        extras["serving_full"] = serving(nreq=200, seed=7, nmin=8, nmax=48, tmin=0.1, tmax=1.0, progress=True)
        log(f"[bench] serving full: {extras['serving_full']}")
    if not args.no_fixed_error:
        log("[bench] time to solution at a fixed error")
        extras["fixed_error"] = fixed_error()
    if args.ablations:
        log("[bench] ablations")
        extras["ablations"] = ablations()
    if args.c3:
        log("[bench] 48^3 k=7 plane wave")
        extras["c3_plane_wave"] = c3_plane_wave()
    if args.sweep:
        log("[bench] degree sweep")
        extras["degree_sweep"] = degree_sweep()
    if not args.no_ceilings:
        log("[bench] ceilings")
        extras["ceilings"] = ceilings()
        # beside the published peak: the fraction of this box's measured device copy
        roofline["measured_copy_GBps"] = extras["ceilings"]["copy_GBps"]
        roofline["frac_of_measured_copy"] = achieved / extras["ceilings"]["copy_GBps"]
        log(f"[bench] ceilings: {extras['ceilings']}")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline (bounded sample)")
        cpu = cpu_baseline()
        log(f"[bench] oracle: {cpu['value']:.3e} DoF-steps/s on {cpu['cores']} threads")
    line = {
        "metric": "DoF-steps/s, FP64 vs FP32-split, LSRK vs ADER, at fixed error; p99 latency",
        "value": head["dof_steps_per_s"], "unit": "DoF-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if head["precision"] == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": "3D periodic unit cube, 24^3 hexes curved with amplitude 0.05, k=5 "
                               "(1.19e7 DoF), rho=1, c = 8-mode Fourier field (seed 1805), upwind, "
                               "Gaussian pressure pulse width 0.05",
                   "scheme": head["scheme"], "precision": head["precision"], "dt": head["dt"],
                   "courant": CR[head["scheme"]],
                   "storage_basis": "gauss points" if BASIS[head["scheme"]] else "gl nodes"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": {k: {"dof_steps_per_s": r["dof_steps_per_s"], "ms_per_step": r["ms_per_step"],
                         "steps_to_T_0.5": r["steps_to_T"], "time_to_T_0.5_s": r["time_to_T_s"],
                         "graph_solve_ms_per_step": r["graph_solve_ms_per_step"],
                         "kernels_ms": r["kernels_ms"], "launch_shape": r["launch_shape"],
                         "storage_basis": "gauss points" if BASIS[r["scheme"]] else "gl nodes"}
                     for k, r in results.items()},
        "kernels": kernels,
        "fixed_error_summary": fixed_summary(extras.get("fixed_error")),
        "fp32_split_error_vs_fp64": extras.get("fp32_split_rel_err_5_steps"),
        "extras": extras,
        "kernel_sources_sha256_16": kernel_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
