"""Parity tolerances derived from the arithmetic.

FP64 time steps from the same state: 1e-12 relative (coefficient 2-norm).
A single FP64 operator application: max(1e-12, 4 eps kappa_1D(k)^d), where
kappa_1D is the condition number of the 1D Gauss-Lobatto mass matrix (Gauss
quadrature): the oracle inverts the dense d-dimensional mass matrix by
Cholesky, whose rounding error grows with kappa_1D^d (7.7e-13 for k = 7 in
3D), and the operator output has no damping factor dt in front of it.
"""
import numpy as np

STEP_TOL = 1e-12


def op_tol(k, dim):
    from oracle import basis
    n = k + 1
    xg, wg = basis.gauss(n)
    S = basis.lagrange(basis.gauss_lobatto(n)[0], xg)
    kappa = np.linalg.cond(S.T @ np.diag(wg) @ S) ** dim
    return max(STEP_TOL, 4 * np.finfo(float).eps * kappa)
