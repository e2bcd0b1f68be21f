"""Stochastic ensemble Kalman filter analysis with normalised anomaly matrices.

Follows Algo. 1 (stochastic EnKF, steps 2-7) in the coarse-grid form of
Algo. 3 (state part: steps 3, 4, 7, 8) and the fine-grid correction of
Algo. 4 step 5:

  y^(i)   = H(x^(i))                           model counterparts
  yo^(i)  = y^o + eps^(i)                      perturbed observations (uncentred)
  xbar, ybar, epsbar                           ensemble means
  X = [x^(i) - xbar]/sqrt(N-1),  Y, E likewise normalised anomalies
  K = X Y^T (Y Y^T + E E^T)^-1                 ensemble gain
  x^a(i) = x^(i) + K (yo^(i) - y^(i))          member update
  x^C'   = x* + K (y^o - H(x*)),  delta^C = x^C' - x*

Readings (the paper is silent or inconsistent):
* ``mode="exact_r"`` (default) uses S = Y Y^T + R with the exact diagonal
  R = sigma^2 I.  The literal Y Y^T + E E^T has rank <= 2(N-1) and is
  singular whenever N_y > 2N - 2; it is kept as ``mode="sample_ee"``.
* The uncentred R^e of Algos. 2-3 is never used; E is centred (Algo. 1).
* The product K d is evaluated as X (Y^T S^-1 d), i.e. the gain's own
  factors applied right to left; S^-1 via LAPACK Cholesky.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


def anomalies(A):
    """Columns (a^(i) - mean)/sqrt(N-1) of a member-major array A (N, m) -> (m, N)."""
    A = np.asarray(A, dtype=np.float64)
    N = A.shape[0]
    return (A - A.mean(axis=0)).T / math.sqrt(N - 1)


def analysis(members, xstar, y_obs, eps, H, sigma, mode="exact_r"):
    """One EnKF analysis on the coarse level.

    members : (N, ...) forecast member states
    xstar   : (...)    Pi_C of the fine forecast
    y_obs   : (N_y,)   observations
    eps     : (N, N_y) observation perturbations
    H       : callable mapping (..., state) -> (..., N_y)
    Returns dict with the analysed members, delta^C and the intermediates.
    """
    members = np.asarray(members, dtype=np.float64)
    N = members.shape[0]
    shape = members.shape[1:]
    Xf = members.reshape(N, -1)
    yf = np.asarray(H(members), dtype=np.float64)          # (N, N_y)
    ystar = np.asarray(H(np.asarray(xstar, dtype=np.float64)), dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    yo = np.asarray(y_obs, dtype=np.float64)[None, :] + eps

    X = anomalies(Xf)                                      # (n, N)
    Y = anomalies(yf)                                      # (N_y, N)
    n_y = Y.shape[0]
    if mode == "exact_r":
        S = Y @ Y.T + (sigma ** 2) * np.eye(n_y)
    elif mode == "sample_ee":
        E = anomalies(eps)
        S = Y @ Y.T + E @ E.T
    else:
        raise ValueError(mode)

    cf = sla.cho_factor(S, lower=True)
    D = (yo - yf).T                                        # (N_y, N) innovations
    dstar = np.asarray(y_obs, dtype=np.float64) - ystar    # (N_y,)
    W = sla.cho_solve(cf, np.concatenate([D, dstar[:, None]], axis=1))
    Z = Y.T @ W                                            # (N, N+1)
    inc = X @ Z                                            # (n, N+1)
    Xa = Xf + inc[:, :N].T
    delta = inc[:, N]
    return {
        "members": Xa.reshape((N,) + shape),
        "delta": delta.reshape(shape),
        "S": S, "Z": Z, "Y": Y, "D": D, "dstar": dstar,
        "yf": yf, "ystar": ystar,
    }


def gain_matrix(members, H, sigma, eps=None, mode="exact_r"):
    """Explicit K^e = X Y^T S^-1 (small cases only)."""
    members = np.asarray(members, dtype=np.float64)
    N = members.shape[0]
    X = anomalies(members.reshape(N, -1))
    Y = anomalies(np.asarray(H(members), dtype=np.float64))
    if mode == "exact_r":
        S = Y @ Y.T + (sigma ** 2) * np.eye(Y.shape[0])
    else:
        E = anomalies(eps)
        S = Y @ Y.T + E @ E.T
    return X @ Y.T @ np.linalg.inv(S)
