"""Seeded initial conditions, probe placements and observation noise.

Seeds are ``cfg.seed + offset``: truth +1, model +2, members +3, observation
noise +4, probe placement +6.  Every array is float64; callers cast.

Initial conditions (synthetic stand-ins for the paper's self-generated
reference simulations):

* 1D truth: sin(x) plus white noise of amplitude ``truth_sigma`` smoothed by
  a periodic Gaussian of standard deviation ``smooth_width`` (weights
  normalised to sum one).  Model: sin(x).  Members: sin at the coarse nodes
  plus white noise of amplitude ``member_sigma`` per coarse node.
* 2D truth: Taylor-Green vortex plus solenoidal random-phase modes with
  integer wavevectors 1 <= |k| <= 8 and equal energy per mode, scaled to a
  velocity RMS of ``truth_sigma``.  Model: Taylor-Green only.  Members: the
  Taylor-Green vortex at the coarse nodes plus their own random-phase modes
  at RMS ``member_sigma``, pressure unchanged.
"""

from __future__ import annotations

import math

import numpy as np

from .configs import Config


def _grid(n: int, length: float) -> np.ndarray:
    return np.arange(n, dtype=np.float64) * (length / n)


# ----------------------------------------------------------------------------- 1D
def burgers_truth_ic(cfg: Config) -> np.ndarray:
    rng = np.random.default_rng(cfg.seed + 1)
    x = _grid(cfg.nx, cfg.length)
    h = cfg.length / cfg.nx
    noise = rng.standard_normal(cfg.nx)
    d = np.minimum(x, cfg.length - x)             # periodic distance to node 0
    w = np.exp(-0.5 * (d / cfg.smooth_width) ** 2)
    w /= w.sum()
    smooth = np.real(np.fft.ifft(np.fft.fft(noise) * np.fft.fft(w)))
    del h
    return (np.sin(x) + cfg.truth_sigma * smooth).reshape(1, cfg.nx)


def burgers_model_ic(cfg: Config) -> np.ndarray:
    return np.sin(_grid(cfg.nx, cfg.length)).reshape(1, cfg.nx)


def burgers_member_ics(cfg: Config) -> np.ndarray:
    rng = np.random.default_rng(cfg.seed + 3)
    xc = _grid(cfg.nxc, cfg.length)
    base = np.sin(xc)
    out = base[None, :] + cfg.member_sigma * rng.standard_normal((cfg.n_members, cfg.nxc))
    return out.reshape(cfg.n_members, 1, cfg.nxc)


# ----------------------------------------------------------------------------- 2D
def _p0(cfg: Config) -> float:
    return 1.0 / (cfg.gamma * cfg.mach ** 2)


def ns_tgv_primitives(cfg: Config, n_x: int, n_y: int):
    """Taylor-Green vortex (rho, u, v, p) on an n_y x n_x periodic grid."""
    x = _grid(n_x, cfg.length)[None, :]
    y = _grid(n_y, cfg.length)[:, None]
    p0 = _p0(cfg)
    u = np.sin(x) * np.cos(y)
    v = -np.cos(x) * np.sin(y)
    p = p0 + 0.25 * (np.cos(2 * x) + np.cos(2 * y))
    rho = p / p0
    return rho, u, v, p


def _random_modes(rng, n_x: int, n_y: int, length: float, rms: float, kmax: int = 8):
    """Solenoidal velocity from the streamfunction sum over 1 <= |k| <= kmax of
    cos(k.x + phase_k) / |k|, random phases, scaled to the given RMS.  Each
    mode factorises as exp(i kx x) exp(i (ky y + phase)), so the sum is
    Im(E_y C E_x) with small matrices of complex exponentials."""
    ks = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(0, kmax + 1)
          if (ky > 0 or kx > 0) and 1 <= kx * kx + ky * ky <= kmax * kmax]
    x = _grid(n_x, length) * (2 * math.pi / length)
    y = _grid(n_y, length) * (2 * math.pi / length)
    phases = rng.uniform(0.0, 2 * math.pi, size=len(ks))
    cu = np.zeros((kmax + 1, 2 * kmax + 1), dtype=np.complex128)
    cv = np.zeros_like(cu)
    for (kx, ky), ph in zip(ks, phases):
        kn = math.hypot(kx, ky)
        # streamfunction psi = cos(k.x + ph)/|k|: u = d psi/dy, v = -d psi/dx
        e = np.exp(1j * ph)
        cu[ky, kx + kmax] += -(ky / kn) * e
        cv[ky, kx + kmax] += (kx / kn) * e
    ey = np.exp(1j * np.outer(y, np.arange(kmax + 1)))                 # (n_y, kmax+1)
    ex = np.exp(1j * np.outer(np.arange(-kmax, kmax + 1), x))          # (2kmax+1, n_x)
    u = np.imag(ey @ cu @ ex)
    v = np.imag(ey @ cv @ ex)
    scale = rms / math.sqrt(np.mean(u * u + v * v))
    return u * scale, v * scale


def _conservative(cfg: Config, rho, u, v, p) -> np.ndarray:
    E = p / (cfg.gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E])


def ns_truth_ic(cfg: Config) -> np.ndarray:
    rng = np.random.default_rng(cfg.seed + 1)
    rho, u, v, p = ns_tgv_primitives(cfg, cfg.nx, cfg.ny)
    du, dv = _random_modes(rng, cfg.nx, cfg.ny, cfg.length, cfg.truth_sigma)
    return _conservative(cfg, rho, u + du, v + dv, p)


def ns_model_ic(cfg: Config) -> np.ndarray:
    rho, u, v, p = ns_tgv_primitives(cfg, cfg.nx, cfg.ny)
    return _conservative(cfg, rho, u, v, p)


def ns_member_ics(cfg: Config) -> np.ndarray:
    rng = np.random.default_rng(cfg.seed + 3)
    rho, u, v, p = ns_tgv_primitives(cfg, cfg.nxc, cfg.nyc)
    out = np.empty((cfg.n_members, 4, cfg.nyc, cfg.nxc))
    for i in range(cfg.n_members):
        du, dv = _random_modes(rng, cfg.nxc, cfg.nyc, cfg.length, cfg.member_sigma)
        out[i] = _conservative(cfg, rho, u + du, v + dv, p)
    return out


# ----------------------------------------------------------------------------- both
def truth_ic(cfg: Config) -> np.ndarray:
    return burgers_truth_ic(cfg) if cfg.dim == 1 else ns_truth_ic(cfg)


def model_ic(cfg: Config) -> np.ndarray:
    return burgers_model_ic(cfg) if cfg.dim == 1 else ns_model_ic(cfg)


def member_ics(cfg: Config) -> np.ndarray:
    return burgers_member_ics(cfg) if cfg.dim == 1 else ns_member_ics(cfg)


def probes_for(cfg: Config):
    """(fine node linear index, observed component) for every scalar probe.

    1D: equispaced fine nodes (every nx / N_y-th node), component 0 (u).
    2D: N_y distinct random fine nodes; probe p observes u if p is even and
    v if p is odd.
    """
    if cfg.dim == 1 and getattr(cfg, "bc", "periodic") == "inlet":
        # the first n_probes fine nodes (80 sensors on [0, 1) in the Sec. 4 case)
        idx = np.arange(cfg.n_probes, dtype=np.int64)
        comp = np.zeros(cfg.n_probes, dtype=np.int64)
    elif cfg.dim == 1:
        step = cfg.nx // cfg.n_probes
        assert step * cfg.n_probes == cfg.nx
        idx = np.arange(cfg.n_probes, dtype=np.int64) * step
        comp = np.zeros(cfg.n_probes, dtype=np.int64)
    else:
        rng = np.random.default_rng(cfg.seed + 6)
        idx = np.sort(rng.choice(cfg.nx * cfg.ny, size=cfg.n_probes, replace=False)).astype(np.int64)
        comp = (np.arange(cfg.n_probes) % 2).astype(np.int64)
    return idx.astype(np.int32), comp.astype(np.int32)


def obs_noise(cfg: Config, cycle: int) -> np.ndarray:
    """Observation noise obs_sigma * xi added to the sampled truth at a cycle."""
    rng = np.random.default_rng([cfg.seed + 4, cycle])
    return cfg.obs_sigma * rng.standard_normal(cfg.n_probes)


def random_members_like(cfg: Config, seed_offset: int = 11, amplitude: float = 1.0) -> np.ndarray:
    """Member states with the workload's structure for tests of one analysis:
    the member initial conditions with an extra seeded random-phase (2D) or
    smooth (1D) perturbation so that anomalies are not those of the ICs."""
    base = member_ics(cfg)
    rng = np.random.default_rng(cfg.seed + seed_offset)
    if cfg.dim == 1:
        xc = _grid(cfg.nxc, cfg.length)
        ph = rng.uniform(0, 2 * math.pi, size=(cfg.n_members, 1))
        a = rng.standard_normal((cfg.n_members, 1)) * 0.02 * amplitude
        return base + (a * np.sin(2 * xc[None, :] + ph))[:, None, :]
    out = base.copy()
    for i in range(cfg.n_members):
        du, dv = _random_modes(rng, cfg.nxc, cfg.nyc, cfg.length, 0.02 * amplitude, kmax=4)
        rho = out[i, 0]
        u = out[i, 1] / rho + du
        v = out[i, 2] / rho + dv
        ke_old = 0.5 * (out[i, 1] ** 2 + out[i, 2] ** 2) / rho
        p_int = out[i, 3] - ke_old
        out[i, 1] = rho * u
        out[i, 2] = rho * v
        out[i, 3] = p_int + 0.5 * rho * (u * u + v * v)
    return out


# ----------------------------------------------------------------------------- inlet case
def inlet_theta_ics(cfg: Config) -> np.ndarray:
    """Member parameters theta^(i) ~ N(theta_prior, diag(theta_prior_sigma^2)), (N, 2)."""
    rng = np.random.default_rng(cfg.seed + 3)
    return (np.asarray(cfg.theta_prior)[None, :]
            + np.asarray(cfg.theta_prior_sigma)[None, :] * rng.standard_normal((cfg.n_members, 2)))


def inlet_uniform(cfg: Config, level: str = "fine", nb: int = 0) -> np.ndarray:
    """The uniform inlet state everywhere: u = u0 (Burgers, (1, n)) or
    (rho0, rho0 u0, rho0 E0) of the characteristic units (Euler, (3, n));
    (nb, F, n) for nb states."""
    n = cfg.nx if level == "fine" else cfg.nxc
    if cfg.eq == "euler":
        a = 1.0 / (1.0 + cfg.mach)
        u0 = cfg.mach * a
        p0 = a * a / cfg.gamma
        e0 = p0 / (cfg.gamma - 1.0) + 0.5 * u0 * u0
        u = np.empty((3, n))
        u[0], u[1], u[2] = 1.0, u0, e0
    else:
        u = np.full((1, n), cfg.u0)
    return u if nb == 0 else np.repeat(u[None], nb, axis=0)
