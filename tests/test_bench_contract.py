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
