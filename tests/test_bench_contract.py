"""CPU checks of bench.py's contract: every leg main() can call exists, and
more than one GPU is refused with a message (the benchmark measures one GPU)."""
import ast
import builtins
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_called_function_is_defined():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    defined = {n.name for n in tree.body if isinstance(n, ast.FunctionDef)}
    main = next(n for n in tree.body if isinstance(n, ast.FunctionDef) and n.name == "main")
    called = {c.func.id for c in ast.walk(main) if isinstance(c, ast.Call) and isinstance(c.func, ast.Name)}
    missing = {f for f in called if f not in defined and not hasattr(builtins, f)}
    assert not missing, missing
    for leg in ("run_variant", "fp32_error", "cpu_baseline", "serving", "fixed_error", "batched_sources",
                "c3_plane_wave", "ablations", "degree_sweep", "ceilings", "copy_calibration"):
        assert leg in defined, leg


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_basis_map_matches_the_oracle():
    """bench.basis_map (the device map the benchmark uses to compare states
    kept at the Gauss points over the GL nodes) against the oracle's own
    GL -> Gauss map on a random state, and its round trip."""
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    from oracle import Mesh as OMesh
    from oracle.operator import gl_to_gauss
    k = 3
    om = OMesh(3, k, W.box_nodes(3, 2, k, 0.05), W.box_neighbors(3, 2), W.ConstantMaterial())
    U = W.random_state(3, (om.nc, 4, om.np_))
    g = bench.basis_map(torch.from_numpy(U), k + 1, 4).numpy()
    assert np.abs(g - gl_to_gauss(om, U)).max() < 1e-13 * np.abs(U).max()
    back = bench.to_gl_nodes(torch.from_numpy(g), k + 1).numpy()
    assert np.abs(back - U).max() < 1e-13 * np.abs(U).max()
