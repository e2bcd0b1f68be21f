"""Dynamical models: discretised conservation laws and explicit time advance.

Paper: explicit transition x_k = Phi_k x_{k-1} (Sec. 2.2, explicit
discretised form), Burgers' equation (Sec. 4, Burgers equation) and the
compressible Navier-Stokes system (Sec. 6, mass / momentum / energy
equations).  The paper discretises with second-order centred differences
and implicit first-order time stepping; the workloads here prescribe:

* 1D Burgers, advective form u_t = -u D1 u + nu D2 u with second-order
  centred D1, D2 on a periodic grid, advanced by the three-stage
  strong-stability-preserving Runge-Kutta scheme of Shu & Osher.
* 2D compressible Navier-Stokes in conservative variables
  (rho, rho u, rho v, E) on a periodic box, fourth-order centred
  differences, classical four-stage Runge-Kutta.

Reading for the 2D operator (the paper states the equations, not a
discretisation order): non-dimensional with rho0 = U0 = T0 = 1,
p = (gamma-1)(E - rho|u|^2/2), T = gamma Ma^2 p / rho, mu = 1/Re,
kappa = mu c_p / Pr with c_p = 1/((gamma-1) Ma^2), Stokes stress
tau = mu (grad u + grad u^T - 2/3 div u I).
  * convection and pressure: D1 of the nodal fluxes;
  * momentum viscous term written as mu (4/3 u_xx + u_yy + 1/3 v_xy) and
    mu (v_xx + 4/3 v_yy + 1/3 u_xy): pure second derivatives with the
    fourth-order D2 stencil, mixed derivatives as D1_x(D1_y .);
  * viscous work: D1 of the nodal flux tau.u (tau from D1 of u, v);
  * heat flux: kappa (D2_x T + D2_y T).
"""

from __future__ import annotations

import numpy as np


# ------------------------------------------------------------------ difference ops
def d1_2(f, h, axis=-1):
    """Second-order centred first derivative, periodic."""
    return (np.roll(f, -1, axis) - np.roll(f, 1, axis)) / (2.0 * h)


def d2_2(f, h, axis=-1):
    """Second-order centred second derivative, periodic."""
    return (np.roll(f, -1, axis) - 2.0 * f + np.roll(f, 1, axis)) / (h * h)


def d1_4(f, h, axis):
    """Fourth-order centred first derivative (f_{i-2} - 8f_{i-1} + 8f_{i+1} - f_{i+2})/(12h)."""
    return (np.roll(f, 2, axis) - 8.0 * np.roll(f, 1, axis)
            + 8.0 * np.roll(f, -1, axis) - np.roll(f, -2, axis)) / (12.0 * h)


def d2_4(f, h, axis):
    """Fourth-order centred second derivative (-f_{i-2} + 16f_{i-1} - 30f_i + 16f_{i+1} - f_{i+2})/(12h^2)."""
    return (-np.roll(f, 2, axis) + 16.0 * np.roll(f, 1, axis) - 30.0 * f
            + 16.0 * np.roll(f, -1, axis) - np.roll(f, -2, axis)) / (12.0 * h * h)


# ------------------------------------------------------------------ Burgers
def burgers_rhs(u, nu, h):
    """L(u) = -u du/dx + nu d2u/dx2 (Burgers equation, Sec. 4), FD2, periodic.

    ``u`` has shape (..., nx).
    """
    return -u * d1_2(u, h) + nu * d2_2(u, h)


def ssprk3_step(u, dt, rhs):
    """Shu-Osher SSP-RK3: u1 = u + dt L(u); u2 = 3/4 u + 1/4 (u1 + dt L(u1));
    u^{n+1} = 1/3 u + 2/3 (u2 + dt L(u2))."""
    u1 = u + dt * rhs(u)
    u2 = 0.75 * u + 0.25 * (u1 + dt * rhs(u1))
    return u / 3.0 + (2.0 / 3.0) * (u2 + dt * rhs(u2))


# ------------------------------------------------------------------ Navier-Stokes
class NSParams:
    def __init__(self, gamma, mach, reynolds, prandtl, hx, hy, inviscid=False):
        self.gamma = gamma
        self.mach = mach
        self.mu = 0.0 if inviscid else 1.0 / reynolds
        cp = 1.0 / ((gamma - 1.0) * mach * mach)
        self.kappa = 0.0 if inviscid else self.mu * cp / prandtl
        self.tfac = gamma * mach * mach          # T = tfac * p / rho
        self.hx = hx
        self.hy = hy


def ns_primitives(q, prm: NSParams):
    rho, m, n, E = q[..., 0, :, :], q[..., 1, :, :], q[..., 2, :, :], q[..., 3, :, :]
    u = m / rho
    v = n / rho
    p = (prm.gamma - 1.0) * (E - 0.5 * (m * u + n * v))
    T = prm.tfac * p / rho
    return rho, m, n, E, u, v, p, T


def ns_rhs(q, prm: NSParams):
    """Right-hand side of the 2D compressible Navier-Stokes system (Sec. 6).

    ``q`` has shape (..., 4, ny, nx) holding (rho, rho u, rho v, E); axis -1
    is x, axis -2 is y.
    """
    hx, hy = prm.hx, prm.hy
    X, Y = -1, -2
    rho, m, n, E, u, v, p, T = ns_primitives(q, prm)
    mu, kappa = prm.mu, prm.kappa

    ux, uy = d1_4(u, hx, X), d1_4(u, hy, Y)
    vx, vy = d1_4(v, hx, X), d1_4(v, hy, Y)
    div = ux + vy
    txx = mu * (2.0 * ux - (2.0 / 3.0) * div)
    tyy = mu * (2.0 * vy - (2.0 / 3.0) * div)
    txy = mu * (uy + vx)

    r_rho = -(d1_4(m, hx, X) + d1_4(n, hy, Y))
    r_m = -(d1_4(m * u + p, hx, X) + d1_4(m * v, hy, Y))
    r_n = -(d1_4(n * u, hx, X) + d1_4(n * v + p, hy, Y))
    r_E = -(d1_4((E + p) * u, hx, X) + d1_4((E + p) * v, hy, Y))
    if mu != 0.0 or kappa != 0.0:
        uxy = d1_4(uy, hx, X)
        vxy = d1_4(vy, hx, X)
        r_m = r_m + mu * ((4.0 / 3.0) * d2_4(u, hx, X) + d2_4(u, hy, Y) + (1.0 / 3.0) * vxy)
        r_n = r_n + mu * (d2_4(v, hx, X) + (4.0 / 3.0) * d2_4(v, hy, Y) + (1.0 / 3.0) * uxy)
        r_E = r_E + d1_4(txx * u + txy * v, hx, X) + d1_4(txy * u + tyy * v, hy, Y) \
            + kappa * (d2_4(T, hx, X) + d2_4(T, hy, Y))
    return np.stack([r_rho, r_m, r_n, r_E], axis=-3)


def rk4_step(q, dt, rhs):
    """Classical four-stage Runge-Kutta."""
    k1 = rhs(q)
    k2 = rhs(q + 0.5 * dt * k1)
    k3 = rhs(q + 0.5 * dt * k2)
    k4 = rhs(q + dt * k3)
    return q + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


# ------------------------------------------------------------------ model wrapper
class Model:
    """The explicit forecast operator M of the state-evolution equation for one grid level."""

    def __init__(self, cfg, level: str, inviscid: bool = False):
        self.cfg = cfg
        self.dim = cfg.dim
        if cfg.dim == 1:
            n = cfg.nx if level == "fine" else cfg.nxc
            self.h = cfg.length / n
            self.nu = cfg.nu
        else:
            nx = cfg.nx if level == "fine" else cfg.nxc
            ny = cfg.ny if level == "fine" else cfg.nyc
            self.prm = NSParams(cfg.gamma, cfg.mach, cfg.reynolds, cfg.prandtl,
                                cfg.length / nx, cfg.length / ny, inviscid=inviscid)
        self.dt = cfg.dt

    def rhs(self, q):
        q = np.asarray(q, dtype=np.float64)
        if self.dim == 1:
            return burgers_rhs(q, self.nu, self.h)
        return ns_rhs(q, self.prm)

    def step(self, q):
        if self.dim == 1:
            return ssprk3_step(q, self.dt, self.rhs)
        return rk4_step(q, self.dt, self.rhs)

    def forecast(self, q, nsteps: int):
        """Advance ``nsteps`` steps; returns (final state, state one step earlier).

        The earlier state is the right-hand side x_{k-1} of the implicit
        system that the relaxed fine-grid iteration regularises against.
        """
        q = np.asarray(q, dtype=np.float64).copy()
        prev = q.copy()
        for _ in range(nsteps):
            prev = q
            q = self.step(q)
        return q, prev

    def diag_coeff(self) -> float:
        """Diagonal of I - dt dF/dx used by the relaxed Jacobi iteration.

        Reading: centred convection has a zero diagonal, so D is the
        viscous part, 1 + dt nu c sum_dims 1/h^2 with c = 2 for the
        second-order D2 stencil and c = 30/12 for the fourth-order one
        (nu = mu / rho0, rho0 = 1); one scalar for all fields.
        """
        if self.dim == 1:
            return 1.0 + self.dt * self.nu * 2.0 / (self.h * self.h)
        p = self.prm
        return 1.0 + self.dt * p.mu * (30.0 / 12.0) * (1.0 / p.hx ** 2 + 1.0 / p.hy ** 2)
