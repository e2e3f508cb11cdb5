"""Pins of the oracle's LSRK5(9) (Sec. 2.2: nine stages, order five, two
registers; the coefficients of the paper's reference are not printed, the
root of the order-5 conditions taken is named by a 10-digit key in
oracle/timestep.py).  Pins: the two-register tableau structure and the
conditions at the refined root; fifth order measured on a linear system
against the matrix exponential and on a driven nonlinear pendulum against a
tight library integrator (the nonlinear trees are invisible to linear
problems); the printed critical Courant numbers of Table 2 (LSRK5(9) column)
within 10 % on the upwind DG operator."""
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

import workloads as W
from oracle import Mesh, apply_operator
from oracle import timestep as ts


def test_two_register_tableau_at_the_key():
    a, b, c = ts.lsrk59_tableau()
    assert a.shape == (9, 9) and np.all(np.triu(a) == 0)
    for i in range(2, 9):
        assert np.array_equal(a[i, :i - 1], b[:i - 1])
    assert np.max(np.abs(ts.order5_conditions(a, b))) < 1e-14
    key = np.array(ts.LSRK59_KEY_ALPHA + ts.LSRK59_KEY_B)
    got = np.concatenate([np.diag(a, -1), b])
    assert np.max(np.abs(got - key)) < 1e-9
    assert c.min() >= 0.0 and c.max() <= 1.0 and np.abs(got).max() < 0.63
    # stability polynomial: Taylor coefficients of exp(z) up to z^5
    g, v = [], np.ones(9)
    for j in range(6):
        g.append(b @ v)
        v = a @ v
    assert np.allclose(np.array(g[:5]), [1, 1 / 2, 1 / 6, 1 / 24, 1 / 120], rtol=1e-13)


def _orders(errs):
    return [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_fifth_order_linear():
    rng = np.random.default_rng(4)
    S = rng.standard_normal((6, 6))
    M = S - S.T - 0.3 * np.eye(6)
    y0 = rng.standard_normal(6)
    T = 2.0
    errs = []
    for n in (10, 20, 40):
        y = y0
        for s in range(n):
            y = ts.lsrk59_step(lambda u, t: M @ u, y, s * T / n, T / n)
        errs.append(np.linalg.norm(y - expm(T * M) @ y0))
    assert min(_orders(errs)) > 4.7


def test_fifth_order_nonlinear_nonautonomous():
    def f(u, t):
        return np.array([u[1], -np.sin(u[0]) - 0.2 * u[1] + 0.5 * np.cos(1.3 * t)])
    y0, T = np.array([1.0, 0.3]), 3.0
    ref = solve_ivp(lambda t, u: f(u, t), (0, T), y0, method="DOP853", rtol=3e-14, atol=1e-14).y[:, -1]
    errs = []
    for n in (15, 30, 60):
        y = y0
        for s in range(n):
            y = ts.lsrk59_step(f, y, s * T / n, T / n)
        errs.append(np.linalg.norm(y - ref))
    assert min(_orders(errs)) > 4.6
    # the LSRK(5,4) of the same module is of order four only
    errs4 = []
    for n in (15, 30, 60):
        y = y0
        for s in range(n):
            y = ts.lsrk_step(f, y, s * T / n, T / n)
        errs4.append(np.linalg.norm(y - ref))
    assert max(_orders(errs4)) < 4.5


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_critical_courant.txt")


def _table2_lsrk59():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            d, k, _, rk59, _ = line.split()
            out[(int(d), int(k))] = float(rk59)
    return out


@pytest.mark.parametrize("dim,nc,k", [(2, 4, 1), (2, 4, 4), (3, 3, 1)])
def test_critical_courant_numbers_lsrk59(dim, nc, k):
    """Stability judged as a run would (amplification over unit time at most
    2, as for the other columns) on the dense upwind operator of a periodic
    Cartesian box; the stability function of the tableau is
    R(z) = sum_j (b a^(j-1) 1) z^j."""
    ref = _table2_lsrk59()[(dim, k)]
    m = Mesh(dim, k, W.box_nodes(dim, nc, k, 0.0), W.box_neighbors(dim, nc), W.ConstantMaterial())
    N = m.nc * (dim + 1) * m.np_
    L = np.column_stack([apply_operator(m, e.reshape(m.nc, dim + 1, m.np_)).ravel() for e in np.eye(N)])
    lam = np.linalg.eigvals(L)
    a, b, _ = ts.lsrk59_tableau()
    g, v = [1.0], np.ones(9)
    for j in range(9):
        g.append(b @ v)
        v = a @ v
    h = 1.0 / nc

    def stable(cr):
        dt = cr * h / k ** 1.5
        R = np.polyval(np.array(g)[::-1], dt * lam)
        return np.max(np.abs(R)) ** (1.0 / dt) <= 2.0
    assert stable(0.9 * ref) and not stable(1.1 * ref)
