"""Diagnostics: relative RMSE (Sec. 4, RMSE definition), ensemble spread
(trace of the ensemble error covariance of Sec. 2.1.2) and the
conservativity residual Gamma (Sec. 6, transversal-momentum conservation
indicator).

TEST INFRASTRUCTURE ONLY (see the package docstring)."""

from __future__ import annotations

import numpy as np


def rel_rmse(xa, xt):
    """sqrt( sum (xa - xt)^2 / sum xt^2 ): discrete form of the integral ratio."""
    xa = np.asarray(xa, dtype=np.float64)
    xt = np.asarray(xt, dtype=np.float64)
    return float(np.sqrt(np.sum((xa - xt) ** 2) / np.sum(xt ** 2)))


def velocity_rmse(qa, qt):
    """Joint (u, v) relative RMSE of 2D conservative states (reading for 2D)."""
    ua = np.stack([qa[1] / qa[0], qa[2] / qa[0]])
    ut = np.stack([qt[1] / qt[0], qt[2] / qt[0]])
    return rel_rmse(ua, ut)


def observed_quantity(states, dim, obs_field=0):
    """The quantity the RMSE and the spread are taken on, per state:
    u (1D Burgers, field 0), rho u (1D Euler, field 1), or the velocity pair
    (u, v) = (rho u / rho, rho v / rho) in 2D.  states: (nb, F, ...) ->
    (nb, n_comp, ...)."""
    s = np.asarray(states, dtype=np.float64)
    if dim == 2:
        return np.stack([s[:, 1] / s[:, 0], s[:, 2] / s[:, 0]], axis=1)
    return s[:, obs_field:obs_field + 1]


def rmse_sums(xa, xt, dim, obs_field=0):
    """(sum (qa - qt)^2, sum qt^2) over the observed quantity of one state
    each; sqrt of their ratio is the relative RMSE of Sec. 4."""
    qa = observed_quantity(np.asarray(xa)[None], dim, obs_field)
    qt = observed_quantity(np.asarray(xt)[None], dim, obs_field)
    return float(np.sum((qa - qt) ** 2)), float(np.sum(qt ** 2))


def spread_sums(members, dim, obs_field=0):
    """(trace of the ensemble covariance, sum of the squared ensemble mean)
    of the observed quantity.

    The paper estimates the error covariance from the ensemble as
    P^e = X X^T with normalised anomalies X = (x^(i) - mean)/sqrt(N_e - 1)
    (Sec. 2.1.2).  Its trace over the observed quantity,
    sum_points sum_i (q^(i) - mean q)^2 / (N_e - 1), is the ensemble spread
    squared; the second number normalises it like the relative RMSE, so
    sqrt(first / second) compares with ``rel_rmse`` of the mean."""
    q = observed_quantity(members, dim, obs_field)
    N = q.shape[0]
    mean = q.sum(axis=0) / N
    dev = q - mean[None]
    return float(np.sum(dev * dev) / (N - 1)), float(np.sum(mean * mean))


def ensemble_spread(members, dim, obs_field=0):
    """Relative ensemble spread sqrt(trace P^e / sum mean^2) of the observed quantity."""
    a, b = spread_sums(members, dim, obs_field)
    return float(np.sqrt(a / b))


def gamma_rhov(q_k, q_km1, model):
    """Gamma = ((rho v)_k - (rho v)_{k-1})/dt - F_{rho v}(q_k), per node.

    The spatial terms are evaluated at the new state (the implicit-Euler
    reading used for the smoothing iteration).
    """
    q_k = np.asarray(q_k, dtype=np.float64)
    q_km1 = np.asarray(q_km1, dtype=np.float64)
    return (q_k[2] - q_km1[2]) / model.dt - model.rhs(q_k)[2]


def gamma_normalised(q_k, q_km1, model):
    """Gamma scaled by the largest time derivative of rho v over the step,
    max |((rho v)_k - (rho v)_{k-1})/dt| (the normalisation of Sec. 6)."""
    g = gamma_rhov(q_k, q_km1, model)
    C = np.max(np.abs((q_k[2] - q_km1[2]) / model.dt))
    return g / C
