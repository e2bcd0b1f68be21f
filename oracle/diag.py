"""Diagnostics: relative RMSE (Sec. 4, RMSE definition) and conservativity
residual Gamma (Sec. 6, transversal-momentum conservation indicator)."""

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


def gamma_rhov(q_k, q_km1, model):
    """Gamma = ((rho v)_k - (rho v)_{k-1})/dt - F_{rho v}(q_k), per node.

    The spatial terms are evaluated at the new state (the implicit-Euler
    reading used for the smoothing iteration).
    """
    q_k = np.asarray(q_k, dtype=np.float64)
    q_km1 = np.asarray(q_km1, dtype=np.float64)
    return (q_k[2] - q_km1[2]) / model.dt - model.rhs(q_k)[2]


def gamma_normalised(q_k, q_km1, model):
    g = gamma_rhov(q_k, q_km1, model)
    C = np.max(np.abs((q_k[2] - q_km1[2]) / model.dt))
    return g / C
