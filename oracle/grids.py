"""Two-grid projection operators Pi_C (fine -> coarse) and Pi_F (coarse -> fine).

Paper, Sec. 2.2 (two-grid FAS description): both projections are
fourth-order Lagrange interpolators.  Reading taken (the paper gives no grid
placement): periodic, vertex-centred, nested grids, fine node r*j coincides
with coarse node j.

* Pi_C evaluated at a coincident node returns that node's value, so the
  fourth-order Lagrange restriction is injection.
* Pi_F uses the four-point (cubic) Lagrange interpolant through coarse
  nodes j-1, j, j+1, j+2 at the fine node r*j + m (local coordinate
  s = m / r), applied per direction (tensor product in 2D).

Everything is written as explicit dense matrices so that it can be read
against the definition.
"""

from __future__ import annotations

import numpy as np


def lagrange4_weights(s: float) -> np.ndarray:
    """Cubic Lagrange basis through nodes at -1, 0, 1, 2, evaluated at s."""
    nodes = np.array([-1.0, 0.0, 1.0, 2.0])
    w = np.empty(4)
    for a in range(4):
        num = 1.0
        den = 1.0
        for b in range(4):
            if b != a:
                num *= (s - nodes[b])
                den *= (nodes[a] - nodes[b])
        w[a] = num / den
    return w


def prolong_matrix(n_coarse: int, ratio: int) -> np.ndarray:
    """Dense (n_coarse*ratio) x n_coarse periodic 1D Pi_F."""
    n_fine = n_coarse * ratio
    P = np.zeros((n_fine, n_coarse))
    for j in range(n_coarse):
        for m in range(ratio):
            w = lagrange4_weights(m / ratio)
            for q, wq in zip((-1, 0, 1, 2), w):
                P[j * ratio + m, (j + q) % n_coarse] += wq
    return P


def restrict_matrix(n_fine: int, ratio: int) -> np.ndarray:
    """Dense (n_fine/ratio) x n_fine injection Pi_C."""
    n_coarse = n_fine // ratio
    R = np.zeros((n_coarse, n_fine))
    for j in range(n_coarse):
        R[j, j * ratio] = 1.0
    return R


def restrict(xf: np.ndarray, ratio: int, dim: int) -> np.ndarray:
    """Pi_C on a state of shape (..., nx) [1D] or (..., ny, nx) [2D]."""
    xf = np.asarray(xf, dtype=np.float64)
    Rx = restrict_matrix(xf.shape[-1], ratio)
    if dim == 1:
        return xf @ Rx.T
    Ry = restrict_matrix(xf.shape[-2], ratio)
    return Ry @ xf @ Rx.T


def prolong(xc: np.ndarray, ratio: int, dim: int) -> np.ndarray:
    """Pi_F on a coarse state of shape (..., nxc) [1D] or (..., nyc, nxc) [2D]."""
    xc = np.asarray(xc, dtype=np.float64)
    Px = prolong_matrix(xc.shape[-1], ratio)
    if dim == 1:
        return xc @ Px.T
    Py = prolong_matrix(xc.shape[-2], ratio)
    return Py @ xc @ Px.T
