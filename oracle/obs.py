"""Observation operators (observation model of Sec. 2.1.1: y = H(x) + eps).

Probes sit at fine-grid nodes (the paper's sensors are mesh nodes of the
fine grid, Sec. 4).  A probe is (fine node linear index, component):
component 0 observes u, component 1 observes v.  In 1D the state is u
itself; in 2D the velocity is momentum over density, which is nonlinear
in the state, so the ensemble uses secant anomalies of H(x^(i)) (the EnKF
variant the paper adopts in its appendix) rather than a tangent-linear H.

Reading for the coarse operator H^C (the paper is silent on how coarse
members are observed): H^C = H^F o Pi_F, evaluated at the probe nodes.
Only the probe rows of the dense Pi_F matrix are used, which is the same
operator restricted to the observed nodes.
"""

from __future__ import annotations

import numpy as np

from . import grids


def observe_fine(x, idx, comp, dim):
    """H^F applied to fine states of shape (..., F, nx) or (..., F, ny, nx)."""
    x = np.asarray(x, dtype=np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    comp = np.asarray(comp, dtype=np.int64)
    if dim == 1:
        flat = x.reshape(x.shape[:-2] + (-1,))
        return flat[..., idx]
    lead = x.shape[:-3]
    flat = x.reshape(lead + (4, -1))
    rho = flat[..., 0, :][..., idx]
    mom = np.where(comp == 0, flat[..., 1, :][..., idx], flat[..., 2, :][..., idx])
    return mom / rho


def _rows(P, fine_idx):
    """Nonzero columns and weights of rows ``fine_idx`` of a dense Pi_F matrix."""
    cols = []
    wts = []
    for i in fine_idx:
        nz = np.nonzero(P[i])[0]
        c = np.zeros(4, dtype=np.int64)
        w = np.zeros(4)
        c[:len(nz)] = nz
        w[:len(nz)] = P[i, nz]
        cols.append(c)
        wts.append(w)
    return np.array(cols), np.array(wts)


def prolong_at(xc, fine_idx, ratio, dim, nx_fine):
    """(Pi_F xc) evaluated at fine linear nodes ``fine_idx``; xc has shape (..., nyc, nxc) or (..., nxc)."""
    xc = np.asarray(xc, dtype=np.float64)
    fine_idx = np.asarray(fine_idx, dtype=np.int64)
    if dim == 1:
        Px = grids.prolong_matrix(xc.shape[-1], ratio)
        c, w = _rows(Px, fine_idx)
        return np.einsum("...pk,pk->...p", xc[..., c], w)
    nyc, nxc = xc.shape[-2], xc.shape[-1]
    Px = grids.prolong_matrix(nxc, ratio)
    Py = grids.prolong_matrix(nyc, ratio)
    cx, wx = _rows(Px, fine_idx % nx_fine)
    cy, wy = _rows(Py, fine_idx // nx_fine)
    g = xc[..., cy[:, :, None], cx[:, None, :]]            # (..., p, 4, 4)
    return np.einsum("...pab,pa,pb->...p", g, wy, wx)


def observe_coarse(xc, idx, comp, dim, ratio, nx_fine):
    """H^C = H^F o Pi_F at the probe nodes, for coarse states (..., F, [nyc,] nxc)."""
    idx = np.asarray(idx, dtype=np.int64)
    comp = np.asarray(comp, dtype=np.int64)
    xc = np.asarray(xc, dtype=np.float64)
    if dim == 1:
        return prolong_at(xc[..., 0, :], idx, ratio, 1, nx_fine)
    rho = prolong_at(xc[..., 0, :, :], idx, ratio, 2, nx_fine)
    mx = prolong_at(xc[..., 1, :, :], idx, ratio, 2, nx_fine)
    my = prolong_at(xc[..., 2, :, :], idx, ratio, 2, nx_fine)
    return np.where(comp == 0, mx, my) / rho
