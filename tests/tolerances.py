"""Parity tolerances.

FP64 time steps from the same state and single FP64 operator applications:
1e-12 relative, both in the coefficient 2-norm and element by element per
state component.  The oracle's own rounding stays far below that bar: its
dense float64 Cholesky mass solve agrees with the same solve in extended
precision to about 2e-15 even for k = 7 in 3D, where the condition number
kappa_1D^d of the mass matrix is about 3.5e3
(tests/test_oracle_operator.py::test_mass_solve_matches_extended_precision).
"""
STEP_TOL = 1e-12


def op_tol(k, dim):
    """Bar of a single operator application (the same for every degree)."""
    return STEP_TOL
