"""Tolerances of the GPU step comparisons (shared by the step tests)."""


# Tolerance of a full step against another solver's step or the oracle's, on
# phi and the velocity: both stop at the 1e-8 relative Newton residual, at
# different iterates; the field difference is that residual times the
# Jacobian's conditioning (observed 1e-9 in FP64, 4.5e-8 for the mixed
# coupled solve).  mu and p are determined through their midpoints only and
# are not compared.
def step_tol(precision):
    return 1e-7 if precision == 0 else 2e-7
