"""1D inviscid Euler equations of the acoustic-wave case, inlet-forced.

Test oracle: plain FP64 NumPy, used by the tests only.

Paper: Sec. 5 (conservative 1D Euler equations for rho, rho u, rho E;
second-order centred differences in space, a first-order time scheme and a
centred sixth-order filter; Dirichlet inlet u(0, t) = u0 (1 + theta(t)
sin(omega t)) with rho and E fixed at their reference values; outlet
extrapolated from the nearest points; ideal gas, gamma = 1.4, inlet Mach
0.4; L = 10, 800 cells, dt = 6e-4 in characteristic units), and the
implementation notes after Algo. 4 (explicit forecasts between analyses, a
single matrix-splitting iteration at the analysis step, one relaxed
iteration with alpha = 0.5 on the corrected fine state).

Readings (the paper leaves them open):
* units: velocities in u_c = u0 + a, lengths in lambda, densities in rho0,
  so a = 1 / (1 + M), u0 = M a, rho0 = 1, p0 = rho0 a^2 / gamma,
  E0 = p0 / ((gamma - 1) rho0) + u0^2 / 2; omega = 2 pi.
* grid: nodes x_i = i h, h = L / n, as in the inlet-forced Burgers case.
* time: forward Euler.  The single damped-Jacobi iteration of the
  implicit-Euler system x - dt R(x) = x_{k-1} at an analysis step, started
  from x_{k-1} with relaxation 1, is the forward-Euler step itself: the
  centred inviscid operator has no diagonal.  So every step is
  x' = x + dt R(x), R = -D1 F(x), F = (rho u, rho u^2 + p, (rho E + p) u),
  p = (gamma - 1) (rho E - (rho u)^2 / (2 rho)).
* one step: the interior nodes 1..n-2 advance; node 0 takes the inlet
  state (rho0, rho0 u_in(t + dt), rho0 E0); then the filter (below) acts
  on nodes 1..n-2 and node n-1 takes the linear extrapolation
  2 x_{n-2} - x_{n-3} of each field.
* filter: the centred explicit filter of order 2p,
  x <- x + (-1)^(p+1) sigma_f delta^(2p) x / 4^p with delta^(2p) the
  undivided difference, transfer function 1 - sigma_f sin^(2p)(k h / 2):
  order 6 on nodes 3..n-4, order 4 on nodes 2 and n-3, order 2 on nodes 1
  and n-2 (the paper cites an optimised filter whose coefficients it does
  not print; without the reduced orders next to the boundaries the fully
  prescribed inlet drives a node-to-node mode that grows within one time
  unit).  sigma_f = 1: grid-scale modes are removed each step, the
  80-cell inlet wave loses less than 1e-3 of its amplitude over the run.
* the relaxed iteration on the corrected fine state:
  x <- x + alpha (x_{k-1} + dt R(x) - x) at the interior (diagonal 1),
  inlet node kept, outlet extrapolated; no filter.
* observed quantity: the momentum rho u (field 1) at the sensor nodes.
"""

from __future__ import annotations

import numpy as np


def reference_state(gamma, mach):
    """(a, u0, rho0, p0, E0) of the characteristic units."""
    a = 1.0 / (1.0 + mach)
    u0 = mach * a
    rho0 = 1.0
    p0 = rho0 * a * a / gamma
    E0 = p0 / ((gamma - 1.0) * rho0) + 0.5 * u0 * u0
    return a, u0, rho0, p0, E0


def uniform(n, gamma, mach, nb=0):
    """The uniform inlet state on n nodes: (3, n), or (nb, 3, n)."""
    _, u0, rho0, _, E0 = reference_state(gamma, mach)
    x = np.empty((3, n))
    x[0], x[1], x[2] = rho0, rho0 * u0, rho0 * E0
    return x if nb == 0 else np.repeat(x[None], nb, axis=0)


def flux(x, gamma):
    """F(x) for states (..., 3, n)."""
    rho, m, e = x[..., 0, :], x[..., 1, :], x[..., 2, :]
    u = m / rho
    p = (gamma - 1.0) * (e - 0.5 * m * u)
    return np.stack([m, m * u + p, (e + p) * u], axis=-2)


def rhs(x, gamma, h):
    """R(x) = -D1 F(x) at the interior nodes (rows of the boundary nodes 0)."""
    f = flux(x, gamma)
    r = np.zeros_like(x)
    r[..., 1:-1] = -(f[..., 2:] - f[..., :-2]) / (2.0 * h)
    return r


_DIFF = {1: (1.0, -2.0, 1.0), 2: (1.0, -4.0, 6.0, -4.0, 1.0), 3: (1.0, -6.0, 15.0, -20.0, 15.0, -6.0, 1.0)}


def undivided(x, p, lo, hi):
    """delta^(2p) x at the nodes lo..hi-1 (needs p neighbours on each side)."""
    c = _DIFF[p]
    d = np.zeros_like(x[..., lo:hi])
    for k, ck in enumerate(c):
        d = d + ck * x[..., lo - p + k:hi - p + k]
    return d


def filter_open(x, sigma):
    """The filter of one step on nodes 1..n-2 (orders 2, 4, 6, 6, ..., 4, 2);
    nodes 0 and n-1 unchanged."""
    n = x.shape[-1]
    y = x.copy()
    for p, (lo, hi) in ((3, (3, n - 3)), (2, (2, 3)), (2, (n - 3, n - 2)), (1, (1, 2)), (1, (n - 2, n - 1))):
        sign = 1.0 if p % 2 == 1 else -1.0
        y[..., lo:hi] = x[..., lo:hi] + sign * sigma * undivided(x, p, lo, hi) / 4.0 ** p
    return y


def inlet_state(t, theta, gamma, mach, omega):
    """(rho0, rho0 u_in, rho0 E0) with u_in = u0 (1 + theta_1 sin(omega t + theta_2));
    theta (..., 2) -> (..., 3)."""
    _, u0, rho0, _, E0 = reference_state(gamma, mach)
    th = np.asarray(theta, dtype=np.float64)
    uin = u0 * (1.0 + th[..., 0] * np.sin(omega * t + th[..., 1]))
    return np.stack(np.broadcast_arrays(rho0 + 0.0 * uin, rho0 * uin, rho0 * E0 + 0.0 * uin), axis=-1)


def _extrapolate_outlet(x):
    x[..., -1] = 2.0 * x[..., -2] - x[..., -3]


def step(x, t, dt, theta, h, gamma, mach, omega, sigma_f):
    """One forward-Euler step from time t: interior update, inlet state,
    filter, outlet extrapolation."""
    y = x + dt * rhs(x, gamma, h)
    y[..., 0] = inlet_state(t + dt, theta, gamma, mach, omega)
    y = filter_open(y, sigma_f)
    _extrapolate_outlet(y)
    return y


def forecast(x, t0, nsteps, dt, theta, h, gamma, mach, omega, sigma_f, theta_of_t=None):
    """nsteps steps from t0 for states (..., 3, n); theta (..., 2) per state,
    or theta_of_t(t) -> (..., 2) evaluated at every step's end time (the
    truth's time-varying amplitude).  Returns (final, state one step earlier)."""
    x = np.asarray(x, dtype=np.float64).copy()
    prev = x.copy()
    for s in range(nsteps):
        t = t0 + s * dt
        th = theta_of_t(t + dt) if theta_of_t is not None else theta
        prev = x
        x = step(x, t, dt, th, h, gamma, mach, omega, sigma_f)
    return x, prev


def sweep(x, x_prev, dt, h, gamma, alpha, n_sweeps):
    """Relaxed iteration of x - dt R(x) = x_prev (diagonal 1), inlet kept,
    outlet extrapolated."""
    x = np.asarray(x, dtype=np.float64).copy()
    xp = np.asarray(x_prev, dtype=np.float64)
    for _ in range(n_sweeps):
        y = x + alpha * (xp + dt * rhs(x, gamma, h) - x)
        y[..., 0] = x[..., 0]
        _extrapolate_outlet(y)
        x = y
    return x


def amplitude_truth(t, theta0, omega_theta):
    """theta(t) = theta0 (1 + sin(omega_theta t)) of the reference run."""
    return theta0 * (1.0 + np.sin(omega_theta * t))
