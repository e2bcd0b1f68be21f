"""Dual EnKF parameter estimation on the inlet-forced 1D cases (Burgers of
Sec. 4; the Euler acoustic case of Sec. 5 through oracle.euler1d).

Test oracle: plain FP64 NumPy, used by the tests only.

Paper: Sec. 2.1.3 (dual estimation: parameters and states updated by two
successive filters), Algo. 2 (Dual EnKF) applied on the coarse grid as in
Algo. 3, with the fine simulation of Algo. 4 driven by the mean of the
analysed parameters; the Burgers application of Sec. 4: Dirichlet inlet
u(0, t) = u0 (1 + theta_1 sin(omega t + theta_2)), outlet extrapolated
from the nearest points, parameters theta = (amplitude, phase).

Readings (the paper leaves them open):
* grid: nodes x_i = i h, i = 0..n-1, h = L / n (L = 10, n = 800 gives the
  paper's dx = 0.0125 and N_x = 800); coarse node j sits on fine node r j.
* space/time: second-order centred differences, three-stage SSP-RK3 (the
  workloads' explicit scheme); the inlet node takes the Dirichlet value of
  each Runge-Kutta stage at that stage's time (t + dt, t + dt/2, t + dt),
  the outlet node the linear extrapolation 2 u_{n-2} - u_{n-3}.
* the paper's own first-order scheme (time_scheme "first_order"; Sec. 4
  and the implementation notes after Algo. 4): explicit (forward-Euler)
  steps between analyses, and at the analysis step, the last of a
  forecast window, a single iteration of a matrix splitting of the
  implicit-Euler system Psi x_k = x_{k-1}, Psi x = x - dt L_{x^0}(x) with
  the convective coefficient frozen at the starting iterate x^0 = x_{k-1}.
  Reading: the splitting is Jacobi, D = diag Psi = 1 + 2 nu dt / h^2 (the
  centred convection has a zero diagonal), no relaxation (the paper names
  a relaxation coefficient only for the final fine-grid iteration), so the
  step is x_k = x_{k-1} + D^-1 dt L(x_{k-1}) at the interior nodes, with the
  inlet value at t_k and the outlet extrapolated as in the other steps.
* Pi_F on the open grid: the cubic Lagrange interpolant through the four
  coarse nodes b..b+3 with b = min(max(j - 1, 0), n_c - 4) for the fine
  node r j + m (one-sided near both ends, including the r - 1 fine nodes
  past the last coarse node); Pi_C is injection, so Pi_C o Pi_F = I.
* the fine correction and the sweeps leave the inlet node alone (its value
  is the boundary condition's, not an estimate); the sweeps extrapolate the
  outlet node from the swept interior like the forecast does.
* parameter random walk tau ~ N(0, diag(sigma_theta^2)) (Sigma^theta is not
  given), drawn with Philox4x32-10 and Box-Muller like the observation
  perturbations, counter (param, member, cycle, 0x5041).
* the perturbed observations of a cycle are drawn once and serve both the
  parameter and the state update (Algo. 2 step 2).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import enkf, rng

STREAM_PARAM = 0x5041


# ------------------------------------------------------------------ open grids
def prolong_matrix_open(n_coarse: int, ratio: int) -> np.ndarray:
    """Dense (n_coarse*ratio) x n_coarse Pi_F on the open grid."""
    n_fine = n_coarse * ratio
    P = np.zeros((n_fine, n_coarse))
    nodes = np.array([0.0, 1.0, 2.0, 3.0])
    for x in range(n_fine):
        j = x // ratio
        b = min(max(j - 1, 0), n_coarse - 4)
        t = x / ratio - b
        for a in range(4):
            num = np.prod([t - nodes[c] for c in range(4) if c != a])
            den = np.prod([nodes[a] - nodes[c] for c in range(4) if c != a])
            P[x, b + a] = num / den
    return P


def restrict_open(xf, ratio):
    """Pi_C = injection on the open grid: coarse node j = fine node r j."""
    return np.asarray(xf, dtype=np.float64)[..., ::ratio]


def prolong_open(xc, ratio):
    xc = np.asarray(xc, dtype=np.float64)
    return xc @ prolong_matrix_open(xc.shape[-1], ratio).T


def observe_coarse_open(xc, idx, ratio, field=0):
    """H^C = H^F o Pi_F at the probe nodes for coarse states (..., F, n_c):
    the observed field (u for Burgers, rho u for Euler) prolonged and sampled."""
    P = prolong_matrix_open(np.asarray(xc).shape[-1], ratio)
    return np.asarray(xc, dtype=np.float64)[..., field, :] @ P[np.asarray(idx, dtype=np.int64)].T


def observed_field(cfg):
    return 1 if getattr(cfg, "eq", "burgers") == "euler" else 0


def model_forecast(cfg, x, t0, nsteps, theta, level):
    """The inlet-forced forecast of the configuration's equations on a level."""
    n = cfg.nx if level == "fine" else cfg.nxc
    h = cfg.length / n
    if getattr(cfg, "eq", "burgers") == "euler":
        from . import euler1d
        return euler1d.forecast(x, t0, nsteps, cfg.dt, theta, h, cfg.gamma, cfg.mach, cfg.omega, cfg.filter_sigma)
    if getattr(cfg, "time_scheme", "ssprk3") == "first_order":
        return inlet_forecast_first_order(x, t0, nsteps, cfg.dt, theta, cfg.nu, h, cfg.u0, cfg.omega)
    return inlet_forecast(x, t0, nsteps, cfg.dt, theta, cfg.nu, h, cfg.u0, cfg.omega)


def model_smooth(cfg, x, x_prev, n_sweeps, alpha):
    if getattr(cfg, "eq", "burgers") == "euler":
        from . import euler1d
        return euler1d.sweep(x, x_prev, cfg.dt, cfg.length / cfg.nx, cfg.gamma, alpha, n_sweeps)
    return smooth_open(x, x_prev, cfg, n_sweeps, alpha)


# ------------------------------------------------------------------ model
def inlet_value(t, theta, u0, omega):
    """u(0, t) = u0 (1 + theta_1 sin(omega t + theta_2)); theta (..., 2)."""
    theta = np.asarray(theta, dtype=np.float64)
    return u0 * (1.0 + theta[..., 0] * np.sin(omega * t + theta[..., 1]))


def _with_bc(u, g):
    u = u.copy()
    u[..., 0] = g
    u[..., -1] = 2.0 * u[..., -2] - u[..., -3]
    return u


def _rhs(u, nu, h):
    """-u u_x + nu u_xx at the interior nodes (boundary rows 0)."""
    r = np.zeros_like(u)
    r[..., 1:-1] = (-u[..., 1:-1] * (u[..., 2:] - u[..., :-2]) / (2.0 * h)
                    + nu * (u[..., 2:] - 2.0 * u[..., 1:-1] + u[..., :-2]) / (h * h))
    return r


def inlet_step(u, t, dt, theta, nu, h, u0, omega):
    """One SSP-RK3 step of the inlet-forced Burgers equation from time t."""
    u1 = _with_bc(u + dt * _rhs(u, nu, h), inlet_value(t + dt, theta, u0, omega))
    u2 = _with_bc(0.75 * u + 0.25 * (u1 + dt * _rhs(u1, nu, h)), inlet_value(t + 0.5 * dt, theta, u0, omega))
    return _with_bc(u / 3.0 + (2.0 / 3.0) * (u2 + dt * _rhs(u2, nu, h)), inlet_value(t + dt, theta, u0, omega))


def inlet_forecast(u, t0, nsteps, dt, theta, nu, h, u0, omega):
    """Advance nsteps from t0; returns (final state, state one step earlier).
    u: (..., 1, n) states; theta: (..., 2) (broadcast over the leading axes)."""
    u = np.asarray(u, dtype=np.float64)[..., 0, :].copy()
    th = np.asarray(theta, dtype=np.float64)
    prev = u.copy()
    for s in range(nsteps):
        prev = u
        u = inlet_step(u, t0 + s * dt, dt, th, nu, h, u0, omega)
    return u[..., None, :], prev[..., None, :]


def jacobi_diagonal(dt, nu, h):
    """Diagonal of Psi = I - dt L at an interior node: the centred second
    difference contributes 2 nu dt / h^2, the centred convection nothing."""
    return 1.0 + 2.0 * nu * dt / (h * h)


def inlet_forecast_first_order(u, t0, nsteps, dt, theta, nu, h, u0, omega):
    """The paper's first-order scheme over one forecast window: nsteps - 1
    forward-Euler steps, then the analysis step as one Jacobi iteration of
    the implicit-Euler system started from x_{k-1}.  Returns (final state,
    state one step earlier), shapes as inlet_forecast."""
    u = np.asarray(u, dtype=np.float64)[..., 0, :].copy()
    th = np.asarray(theta, dtype=np.float64)
    D = jacobi_diagonal(dt, nu, h)
    prev = u.copy()
    for s in range(nsteps):
        prev = u
        g = inlet_value(t0 + (s + 1) * dt, th, u0, omega)
        if s < nsteps - 1:
            u = _with_bc(u + dt * _rhs(u, nu, h), g)                 # explicit step
        else:
            u = _with_bc(u + (dt / D) * _rhs(u, nu, h), g)           # x^1 = x^0 + D^-1 (c - Psi x^0), x^0 = c
    return u[..., None, :], prev[..., None, :]


def correct_open(xf, delta, ratio):
    """x' = x^F_f + Pi_F(delta^C) (Algo. 4 step 5) at every node but the
    inlet, whose value the boundary condition prescribes."""
    x = np.asarray(xf, dtype=np.float64) + prolong_open(delta, ratio)
    x[..., 0] = np.asarray(xf, dtype=np.float64)[..., 0]
    return x


def smooth_open(x, x_prev, cfg, n_sweeps, alpha):
    """Relaxed Jacobi sweeps of the implicit-Euler system of the last step
    (as for the periodic case, Algo. 4 step 6) at the interior nodes; the
    inlet node keeps its value and the outlet node is extrapolated from
    the swept interior."""
    h = cfg.length / cfg.nx
    D = 1.0 + cfg.dt * cfg.nu * 2.0 / (h * h)
    u = np.asarray(x, dtype=np.float64)[..., 0, :]
    up = np.asarray(x_prev, dtype=np.float64)[..., 0, :]
    for _ in range(n_sweeps):
        u = _with_bc(u + (alpha / D) * (up + cfg.dt * _rhs(u, cfg.nu, h) - u), u[..., 0])
    return u[..., None, :]


# ------------------------------------------------------------------ parameters
def param_perturbations(seed: int, cycle: int, n_members: int, sigmas):
    """tau[i, p] ~ N(0, sigmas[p]^2), shape (n_members, P), FP64 (Philox as
    for the observation perturbations, last counter word 0x5041)."""
    sig = np.asarray(sigmas, dtype=np.float64)
    P = sig.shape[0]
    i = np.arange(n_members, dtype=np.uint64)[:, None]
    p = np.arange(P, dtype=np.uint64)[None, :]
    shape = (n_members, P)
    ctr = (np.broadcast_to(p >> np.uint64(1), shape), np.broadcast_to(i, shape),
           np.full(shape, cycle & rng.MASK, dtype=np.uint64), np.full(shape, STREAM_PARAM, dtype=np.uint64))
    key = (np.uint64(seed & rng.MASK), np.uint64((seed >> 32) & rng.MASK))
    r0, r1, r2, r3 = rng.philox4x32_10(ctr, key)
    u1, u2 = rng._u53(r0, r1), rng._u53(r2, r3)
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.where((p % np.uint64(2)) == 0, rad * np.cos(2.0 * np.pi * u2), rad * np.sin(2.0 * np.pi * u2))
    return sig[None, :] * z


def param_update(theta_f, Z):
    """theta^a(j) = theta^f(j) + sum_i Theta_i Z[i, j] (Algo. 2 step 5):
    Theta the normalised parameter anomalies, Z = Y^T S^-1 D of the
    parameter forecast (members as columns of D)."""
    theta_f = np.asarray(theta_f, dtype=np.float64)
    N = theta_f.shape[0]
    Th = (theta_f - theta_f.mean(axis=0)) / np.sqrt(N - 1.0)     # (N, P): row i = Theta_i
    return theta_f + (Th.T @ Z[:, :N]).T


# ------------------------------------------------------------------ one cycle
@dataclasses.dataclass
class DualState:
    fine: np.ndarray        # (1, n)
    members: np.ndarray     # (N, 1, n_c)
    theta: np.ndarray       # (N, 2)
    t: float = 0.0
    cycle: int = 0


def dual_cycle(cfg, st: DualState, y_obs, idx, n_sweeps=1, alpha=0.5, seed=None):
    """One analysis of the dual MEnKF (Algo. 3 on the coarse grid, Algo. 4
    for the fine simulation).  Returns the new state and the parameter mean."""
    c = st.cycle + 1
    seed = cfg.seed + 5 if seed is None else seed
    N, r = cfg.n_members, cfg.ratio
    eps = rng.perturbations(seed, c, N, cfg.n_probes, cfg.obs_sigma)

    fld = observed_field(cfg)

    def H(xc):
        return observe_coarse_open(xc, idx, r, fld)

    # parameter forecast, member forecast with theta^f, parameter update
    theta_f = st.theta + param_perturbations(seed, c, N, cfg.theta_walk)
    mem_f, _ = model_forecast(cfg, st.members, st.t, cfg.n_obs, theta_f, "coarse")
    xstar0 = restrict_open(st.fine, r)     # any x*: the parameter update uses only the D columns
    res_p = enkf.analysis(mem_f, xstar0, y_obs, eps, H, cfg.obs_sigma)
    theta_a = param_update(theta_f, res_p["Z"])
    theta_bar = theta_a.mean(axis=0)
    # member forecast again with theta^a, fine forecast with the mean
    mem_f2, _ = model_forecast(cfg, st.members, st.t, cfg.n_obs, theta_a, "coarse")
    xf, xprev = model_forecast(cfg, st.fine, st.t, cfg.n_obs, theta_bar, "fine")
    xstar = restrict_open(xf, r)
    res = enkf.analysis(mem_f2, xstar, y_obs, eps, H, cfg.obs_sigma)
    x = correct_open(xf, res["delta"], r)
    x = model_smooth(cfg, x, xprev, n_sweeps, alpha)
    return DualState(fine=x, members=res["members"], theta=theta_a, t=st.t + cfg.n_obs * cfg.dt, cycle=c), theta_bar
