"""Workload configurations (sizes, constants, seeds).

The five named workloads are synthetic stand-ins for the paper's cases: a
1D periodic viscous Burgers flow (shapes after the Burgers case of Sec. 4)
and a 2D periodic compressible Navier-Stokes box (stand-in for the mixing
layer of Sec. 6).  Time steps not fixed by the workload descriptions are
stability-derived (acoustic CFL about 0.35, diffusion number well below the
explicit limit).
"""

from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    dim: int                 # 1 (Burgers) or 2 (compressible Navier-Stokes)
    nx: int                  # fine points along x
    ny: int                  # fine points along y (1 in 1D)
    ratio: int               # coarsening ratio r_C per direction
    n_members: int           # ensemble size N_e
    n_obs: int               # time steps between two analyses
    n_probes: int            # scalar observations N_y
    dt: float
    n_cycles: int
    obs_sigma: float         # observation noise std (R = obs_sigma^2 I)
    member_sigma: float      # member perturbation amplitude
    precision: str = "f32"   # "f64" = all-double path, "f32" = mixed path
    nu: float = 0.0          # Burgers viscosity
    gamma: float = 1.4
    mach: float = 0.3
    reynolds: float = 1000.0
    prandtl: float = 0.71
    length: float = 2.0 * math.pi
    seed: int = 2012
    truth_sigma: float = 0.1  # 1D truth noise amplitude / 2D truth mode RMS
    smooth_width: float = 0.1  # 1D truth noise smoothing (Gaussian std, x units)
    # inlet-forced 1D Burgers (dual parameter estimation); bc "periodic" elsewhere
    bc: str = "periodic"
    u0: float = 1.0
    omega: float = 2.0 * math.pi
    theta_true: tuple = (0.2, 0.0)
    theta_prior: tuple = (0.0, 0.3)
    theta_prior_sigma: tuple = (0.05, 0.05)
    theta_walk: tuple = (0.005, 0.005)
    t_spinup: float = 10.0
    # 1D equations: "burgers" or "euler" (inviscid 1D Euler, acoustic case)
    eq: str = "burgers"
    filter_sigma: float = 1.0      # strength of the explicit filter (Euler case)
    # inlet-forced Burgers: "ssprk3" or "first_order" (the paper's scheme)
    time_scheme: str = "ssprk3"
    theta_b: float = 10.0          # truth amplitude theta0 (1 + sin(omega t / b)) (Euler case)

    @property
    def nfields(self) -> int:
        if self.dim == 2:
            return 4
        return 3 if self.eq == "euler" else 1

    @property
    def nxc(self) -> int:
        return self.nx // self.ratio

    @property
    def nyc(self) -> int:
        return 1 if self.dim == 1 else self.ny // self.ratio

    @property
    def n_fine(self) -> int:
        return self.nx * self.ny

    @property
    def n_coarse(self) -> int:
        return self.nxc * self.nyc

    @property
    def fine_shape(self):
        return (self.nfields, self.nx) if self.dim == 1 else (self.nfields, self.ny, self.nx)

    @property
    def coarse_shape(self):
        return (self.nfields, self.nxc) if self.dim == 1 else (self.nfields, self.nyc, self.nxc)

    @property
    def mu(self) -> float:
        return 1.0 / self.reynolds

    def with_(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


C1 = Config(name="burgers1d_256_64_n40", dim=1, nx=256, ny=1, ratio=4, n_members=40,
            n_obs=10, n_probes=32, dt=1e-3, n_cycles=20, obs_sigma=0.02,
            member_sigma=0.05, precision="f64", nu=0.01)

C2 = Config(name="burgers1d_16384_4096_n256", dim=1, nx=16384, ny=1, ratio=4,
            n_members=256, n_obs=5, n_probes=1024, dt=5e-5, n_cycles=400,
            obs_sigma=0.02, member_sigma=0.05, precision="f32", nu=1e-3)

C3 = Config(name="ns2d_1024_256_n64", dim=2, nx=1024, ny=1024, ratio=4, n_members=64,
            n_obs=20, n_probes=4096, dt=5e-4, n_cycles=100, obs_sigma=0.01,
            member_sigma=0.05, precision="f32")

C4 = Config(name="ns2d_512_128_n32", dim=2, nx=512, ny=512, ratio=4, n_members=32,
            n_obs=20, n_probes=1024, dt=1e-3, n_cycles=100, obs_sigma=0.01,
            member_sigma=0.05, precision="f32")

CONFIGS = {"C1": C1, "C2": C2, "C3": C3, "C4": C4}


def inlet_burgers(ratio: int = 4, precision: str = "f64", **kw) -> Config:
    """The Burgers case of Sec. 4: [0, 10], dx = 0.0125 (800 nodes), Re = 200,
    dt = 2e-4, inlet u0 (1 + theta_1 sin(2 pi t + theta_2)), truth theta =
    (0.2, 0), 80 sensors on [0, 1) observed every 30 steps with variance
    0.0025, N_e = 100, prior theta ~ N((0, 0.3), 0.0025 I)."""
    base = Config(name=f"burgers1d_inlet_800_r{ratio}_n100", dim=1, nx=800, ny=1, ratio=ratio,
                  n_members=100, n_obs=30, n_probes=80, dt=2e-4, n_cycles=3166, obs_sigma=0.05,
                  member_sigma=0.0, precision=precision, nu=1.0 / 200.0, length=10.0, bc="inlet")
    return base.with_(**kw)


def euler_inlet(ratio: int = 4, n_obs: int = 30, precision: str = "f64", **kw) -> Config:
    """The acoustic case of Sec. 5: inviscid 1D Euler on [0, 10], 800 cells,
    dt = 6e-4, inlet Mach 0.4, inlet velocity u0 (1 + theta(t) sin(2 pi t))
    with the truth theta(t) = 0.015 (1 + sin(2 pi t / 10)), 80 sensors on
    [0, 1) observing rho u, N_e = 100, r_C = 4, prior theta ~ N(0, 6.4e-5),
    random walk variance 1e-10 per analysis, assimilation over t in [0, 110]
    after a 10-unit spin-up of the truth.  n_obs = 30, 167, 833 give the
    analysis frequencies f_a = 55, 10, 2 per characteristic time.  The
    observation noise is the paper's variance 0.09 read in SI units of
    momentum (rho0 = 1.17 kg/m^3, T0 = 300 K, air) and converted to
    rho0 (u0 + a) units."""
    a_si = math.sqrt(1.4 * 287.05 * 300.0)
    sigma = 0.3 / (1.17 * (1.0 + 0.4) * a_si)
    mach = 0.4
    base = Config(name=f"euler1d_inlet_800_r{ratio}_n100_nobs{n_obs}", dim=1, nx=800, ny=1, ratio=ratio,
                  n_members=100, n_obs=n_obs, n_probes=80, dt=6e-4, n_cycles=int(110.0 / (n_obs * 6e-4)),
                  obs_sigma=sigma, member_sigma=0.0, precision=precision, length=10.0, bc="inlet", eq="euler",
                  gamma=1.4, mach=mach, u0=mach / (1.0 + mach), omega=2.0 * math.pi,
                  theta_true=(0.015, 0.0), theta_prior=(0.0, 0.0), theta_prior_sigma=(0.008, 0.0),
                  theta_walk=(1e-5, 0.0), t_spinup=10.0, filter_sigma=1.0, theta_b=10.0)
    return base.with_(**kw)


def tiny_1d(precision: str = "f64", **kw) -> Config:
    base = Config(name="burgers1d_tiny", dim=1, nx=128, ny=1, ratio=4, n_members=12,
                  n_obs=4, n_probes=8, dt=1e-3, n_cycles=3, obs_sigma=0.02,
                  member_sigma=0.05, precision=precision, nu=0.02)
    return base.with_(**kw)


def tiny_2d(precision: str = "f32", **kw) -> Config:
    base = Config(name="ns2d_tiny", dim=2, nx=64, ny=64, ratio=4, n_members=8,
                  n_obs=2, n_probes=24, dt=2e-3, n_cycles=2, obs_sigma=0.01,
                  member_sigma=0.05, precision=precision, reynolds=200.0)
    return base.with_(**kw)


def ragged_2d(precision: str = "f32", **kw) -> Config:
    """Non-square grid whose sides are not multiples of any power-of-two tile."""
    base = Config(name="ns2d_ragged", dim=2, nx=200, ny=72, ratio=4, n_members=24,
                  n_obs=2, n_probes=40, dt=2e-3, n_cycles=2, obs_sigma=0.01,
                  member_sigma=0.05, precision=precision, reynolds=500.0,
                  length=2.0 * math.pi)
    return base.with_(**kw)


def uneven_batch(n_instances: int = 48, seed: int = 2012 + 7) -> List[Config]:
    """Independent 2D instances with uneven fine grids, ensemble sizes and probe
    counts: fine side in {256, 512, 768}, coarse = fine / 4, N in {16, 32, 64, 128},
    N_y uniform in [256, 2048], time step at a fixed acoustic CFL."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_instances):
        side = int(rng.choice([256, 512, 768]))
        n = int(rng.choice([16, 32, 64, 128]))
        ny_obs = int(rng.integers(256, 2049))
        dt = 5e-4 * 1024.0 / side          # same CFL as the 1024^2 case
        out.append(Config(name=f"batch{i:02d}_{side}_n{n}", dim=2, nx=side, ny=side,
                          ratio=4, n_members=n, n_obs=20, n_probes=ny_obs, dt=dt,
                          n_cycles=10, obs_sigma=0.01, member_sigma=0.05,
                          precision="f32", seed=2012 + 100 + i))
    return out
