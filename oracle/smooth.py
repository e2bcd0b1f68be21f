"""Relaxed matrix-splitting iteration on the fine grid (Algo. 4 step 6).

The paper applies one iteration of an implicit matrix-splitting procedure
with relaxation alpha = 0.5 to the corrected fine state (implementation
notes after Algo. 4; rationale in Sec. 3: a deliberately loose tolerance
keeps the memory of the estimate while the model regularises it).  It does
not name the splitting, the right-hand side or the diagonal.

Reading: damped Jacobi on the implicit-Euler system of the last time step,
x - dt F(x) = x_{k-1}, with the nonlinear coefficients frozen at the current
iterate (Picard):  x <- x + alpha D^-1 (x_{k-1} + dt F(x) - x), where F is
the fine model's spatial operator and D the scalar viscous diagonal of
I - dt dF/dx (see ``Model.diag_coeff``).
"""

from __future__ import annotations

import numpy as np


def sweep(x, x_prev, model, alpha):
    x = np.asarray(x, dtype=np.float64)
    D = model.diag_coeff()
    return x + (alpha / D) * (np.asarray(x_prev, dtype=np.float64) + model.dt * model.rhs(x) - x)


def smooth(x, x_prev, model, n_sweeps, alpha=0.5):
    for _ in range(n_sweeps):
        x = sweep(x, x_prev, model, alpha)
    return x
