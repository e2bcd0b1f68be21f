"""Closed-form Kalman filter analysis (Sec. 2.1.1, gain / state / covariance update).

Used only to pin the ensemble gain: for a linear observation operator H,
K = P H^T (H P H^T + R)^-1, x^a = x^f + K (y^o - H x^f), P^a = (I - K H) P,
with an explicit matrix inverse (brute force, tiny sizes only).
"""

from __future__ import annotations

import numpy as np


def kalman_gain(P, H, R):
    P = np.asarray(P, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    return P @ H.T @ np.linalg.inv(H @ P @ H.T + R)


def kalman_update(xf, P, H, R, y):
    K = kalman_gain(P, H, R)
    xa = xf + K @ (y - H @ xf)
    Pa = (np.eye(P.shape[0]) - K @ H) @ P
    return xa, Pa, K
