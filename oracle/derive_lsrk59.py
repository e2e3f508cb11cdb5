"""How the LSRK5(9) key in oracle/timestep.py was chosen (test
infrastructure, like the rest of oracle/; run by hand, not by the tests).

Sec. 2.2 uses a nine-stage, fifth-order, two-register scheme of its
reference without printing the coefficients.  In the two-register (2R) form
(Butcher a_ij = b_j for j < i-1, free subdiagonal alpha) nine stages have 17
free coefficients for the 17 order-5 conditions, which have many isolated
real roots.  This script
  1. finds roots by Levenberg-Marquardt from seeded random starts
     (oracle.timestep.order5_conditions, tableau_2r),
  2. keeps those with all c_i in [0, 1] and |coefficients| <= 1,
  3. ranks them by the critical Courant number on the dense upwind DG
     operator of a periodic 4x4 box at k = 4 (the criterion of the paper's
     Table 2, with stability judged as in tests/test_oracle_stability.py),
and prints the 10-digit key of the best, with its critical Courant numbers
at the other Table 2 entries next to the printed ones.

    python -m oracle.derive_lsrk59 [--trials N] [--procs P]
"""
from __future__ import annotations

import argparse
from concurrent.futures import ProcessPoolExecutor

import numpy as np
from scipy.optimize import least_squares

from . import timestep as ts
from .mesh import Mesh
from .operator import apply_operator

# seeded start boxes: (seed, alpha range, b range)
STARTS = [(s, (0.0, 0.6), (0.0, 0.3)) for s in (1, 2, 3, 4)] + \
         [(s, (-0.5, 1.5), (-0.3, 0.6)) for s in (11, 12, 13, 14, 15, 16)]


def _residual(x):
    a, b, _ = ts.tableau_2r(x[:8], x[8:])
    return ts.order5_conditions(a, b)


def _roots(job):
    seed, (alo, ahi), (blo, bhi), trials = job
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(trials):
        x0 = np.concatenate([rng.uniform(alo, ahi, 8), rng.uniform(blo, bhi, 9)])
        r = least_squares(_residual, x0, xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=3000, method="lm")
        if np.max(np.abs(r.fun)) < 1e-13:
            out.append(r.x)
    return out


def _box_spectrum(dim, nc, k):
    class Unit:
        def __call__(self, x):
            x = np.asarray(x)
            return np.ones(x.shape[:-1]), np.ones(x.shape[:-1])
    from workloads import box_nodes, box_neighbors  # seeded mesh recipe, no method arithmetic
    m = Mesh(dim, k, box_nodes(dim, nc, k, 0.0), box_neighbors(dim, nc), Unit())
    n = m.nc * (dim + 1) * m.np_
    L = np.column_stack([apply_operator(m, e.reshape(m.nc, dim + 1, m.np_)).ravel() for e in np.eye(n)])
    return np.linalg.eigvals(L), 1.0 / nc, k


def critical_courant(x, spectrum):
    lam, h, k = spectrum
    a, b, _ = ts.tableau_2r(x[:8], x[8:])
    g, v = [1.0], np.ones(9)
    for _ in range(9):
        g.append(b @ v)
        v = a @ v
    lo, hi = 0.01, 3.0
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        dt = mid * h / k ** 1.5
        if np.max(np.abs(np.polyval(np.array(g)[::-1], dt * lam))) ** (1.0 / dt) <= 2.0:
            lo = mid
        else:
            hi = mid
    return lo


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trials", type=int, default=1600, help="starts per seed")
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    with ProcessPoolExecutor(args.procs) as ex:
        found = [x for xs in ex.map(_roots, [(s, a, b, args.trials) for s, a, b in STARTS]) for x in xs]
    roots = []
    for x in found:
        if not any(np.abs(x - r).max() < 1e-8 for r in roots):
            roots.append(x)
    keep = [x for x in roots if np.abs(x).max() <= 1.0 and
            np.all((ts.tableau_2r(x[:8], x[8:])[2] >= -1e-12) & (ts.tableau_2r(x[:8], x[8:])[2] <= 1 + 1e-12))]
    print(f"{len(roots)} distinct roots, {len(keep)} with c in [0, 1] and |coefficients| <= 1")
    spec = _box_spectrum(2, 4, 4)
    ranked = sorted(keep, key=lambda x: -critical_courant(x, spec))
    best = ranked[0]
    print("alpha key:", [float("%.10g" % v) for v in best[:8]])
    print("b key:    ", [float("%.10g" % v) for v in best[8:]])
    for dim, nc, k, printed in [(2, 4, 1, 0.55), (2, 4, 4, 0.87), (3, 3, 1, 0.36)]:
        print(f"Cr_crit {dim}D k={k}: {critical_courant(best, _box_spectrum(dim, nc, k)):.3f} (Table 2: {printed})")


if __name__ == "__main__":
    main()
