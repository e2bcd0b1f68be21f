"""Pins of the oracle's dynamical models against closed forms and physics:
Cole-Hopf Burgers solution, discrete conservation, convected entropy wave,
Taylor-Green decay, Stokes-Kirchhoff sound attenuation and viscous heating."""

import math

import numpy as np
import pytest

from oracle import models
from synthetic import configs


def cole_hopf(nx, nu, t, nfine=2048):
    """u = -2 nu phi_x / phi with phi_t = nu phi_xx, phi0 = exp(cos x / (2 nu)),
    solved spectrally in FP64 for u0 = sin x on [0, 2pi)."""
    x = np.arange(nfine) * 2 * math.pi / nfine
    phi0 = np.exp(np.cos(x) / (2 * nu))
    k = np.fft.fftfreq(nfine, d=1.0 / nfine)
    ph = np.fft.fft(phi0) * np.exp(-nu * k * k * t)
    phi = np.real(np.fft.ifft(ph))
    phix = np.real(np.fft.ifft(1j * k * ph))
    u = -2 * nu * phix / phi
    return u[:: nfine // nx]


@pytest.mark.parametrize("nu", [0.1, 0.5])
def test_burgers_matches_cole_hopf_second_order(nu):
    errs = []
    T = 0.5
    for nx in (32, 64, 128):
        h = 2 * math.pi / nx
        dt = 0.2 * min(h, h * h / nu)
        nsteps = int(round(T / dt))
        dt = T / nsteps
        u = np.sin(np.arange(nx) * h)
        rhs = lambda v: models.burgers_rhs(v, nu, h)
        for _ in range(nsteps):
            u = models.ssprk3_step(u, dt, rhs)
        errs.append(np.max(np.abs(u - cole_hopf(nx, nu, T))))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-3
    assert all(1.8 < o < 2.3 for o in orders), (errs, orders)


def test_burgers_conserves_sum():
    cfg = configs.tiny_1d()
    m = models.Model(cfg, "fine")
    rng = np.random.default_rng(0)
    u = np.sin(np.arange(cfg.nx) * m.h)[None] + 0.1 * rng.standard_normal((3, 1, cfg.nx))
    s0 = u.sum(axis=-1)
    u1, _ = m.forecast(u, 100)
    np.testing.assert_allclose(u1.sum(axis=-1), s0, rtol=0, atol=1e-12 * np.abs(u).sum())


def _ns_cfg(**kw):
    return configs.tiny_2d(**kw)


def test_ns_conserves_all_four_totals():
    cfg = _ns_cfg(nx=48, ny=40, reynolds=100.0)
    from synthetic import fields
    q = fields.ns_truth_ic(cfg.with_(truth_sigma=0.3))
    m = models.Model(cfg, "fine")
    q1, _ = m.forecast(q, 10)
    tot0 = q.sum(axis=(-1, -2))
    tot1 = q1.sum(axis=(-1, -2))
    np.testing.assert_allclose(tot1, tot0, rtol=0, atol=1e-12 * np.abs(q).sum(axis=(-1, -2)).max())


def _entropy_wave(n, t, u0=0.7, v0=0.4):
    cfg = _ns_cfg(nx=n, ny=n)
    h = 2 * math.pi / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    p = 1.0 / (cfg.gamma * cfg.mach ** 2)
    def state(tt):
        rho = 1.0 + 0.2 * np.sin((X - u0 * tt) + (Y - v0 * tt))
        E = p / (cfg.gamma - 1) + 0.5 * rho * (u0 * u0 + v0 * v0)
        return np.stack([rho, rho * u0, rho * v0, E])
    m = models.Model(cfg.with_(dt=0.05 * h), "fine", inviscid=True)
    nsteps = int(round(t / m.dt))
    m.dt = t / nsteps
    q, _ = m.forecast(state(0.0), nsteps)
    return np.max(np.abs(q[0] - state(t)[0]))


def test_ns_entropy_wave_fourth_order():
    errs = [_entropy_wave(n, 0.5) for n in (16, 32, 64)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.6 < o < 4.4 for o in orders), (errs, orders)


def test_ns_taylor_green_energy_decay():
    from synthetic import fields
    cfg = _ns_cfg(nx=64, ny=64, reynolds=100.0, mach=0.1, dt=2e-3)
    q = fields.ns_model_ic(cfg)
    m = models.Model(cfg, "fine")
    ke = lambda s: np.sum(0.5 * (s[1] ** 2 + s[2] ** 2) / s[0])
    T = 1.0
    q1, _ = m.forecast(q, int(round(T / cfg.dt)))
    ratio = ke(q1) / ke(q)
    expected = math.exp(-4.0 * cfg.mu * T)
    assert abs(ratio / expected - 1) < 5e-3, (ratio, expected)


@pytest.mark.parametrize("kvec", [(1, 0), (1, 1)])
def test_ns_sound_attenuation_stokes_kirchhoff(kvec):
    """Small plane acoustic wave: speed 1/Ma and amplitude decay rate
    |k|^2/2 [4/3 nu + (gamma - 1) nu / Pr] (classical sound absorption)."""
    n = 32
    cfg = _ns_cfg(nx=n, ny=n, reynolds=20.0, mach=0.5)
    h = 2 * math.pi / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    kx, ky = kvec
    kn = math.hypot(kx, ky)
    c = 1.0 / cfg.mach
    p0 = 1.0 / (cfg.gamma * cfg.mach ** 2)
    eps = 1e-5
    ph = np.cos(kx * X + ky * Y)
    rho = 1.0 + eps * ph
    un = c * eps * ph                        # velocity along k for a wave travelling along k
    u, v = un * kx / kn, un * ky / kn
    p = p0 + c * c * eps * ph
    E = p / (cfg.gamma - 1) + 0.5 * rho * (u * u + v * v)
    q = np.stack([rho, rho * u, rho * v, E])
    m = models.Model(cfg.with_(dt=0.02 * h / c), "fine")
    T = 1.0
    nsteps = int(round(T / m.dt))
    m.dt = T / nsteps
    q1, _ = m.forecast(q, nsteps)
    u1 = q1[1] / q1[0]
    v1 = q1[2] / q1[0]
    p1 = (cfg.gamma - 1) * (q1[3] - 0.5 * q1[0] * (u1 * u1 + v1 * v1))
    w = (p1 - p0) / c + (u1 * kx + v1 * ky) / kn    # right-running characteristic (rho0 = 1)
    coef = np.sum(w * np.exp(-1j * (kx * X + ky * Y))) / (n * n) * 2
    amp0 = 2 * c * eps
    nu = cfg.mu
    beta = 0.5 * kn * kn * ((4.0 / 3.0) * nu + (cfg.gamma - 1) * nu / cfg.prandtl)
    assert abs(abs(coef) / amp0 - math.exp(-beta * T)) < 0.02 * (1 - math.exp(-beta * T))
    phase = -np.angle(coef)
    expected = (c * kn * T) % (2 * math.pi)
    dphi = (phase - expected + math.pi) % (2 * math.pi) - math.pi
    assert abs(dphi) < 2e-3


def test_ns_viscous_heating_of_shear_wave():
    """u = U sin y, v = 0: internal energy rises at the dissipation rate mu u_y^2,
    so p_t = (gamma - 1) mu U^2 cos^2 y at t = 0 (uniform T, no conduction yet)."""
    n = 64
    cfg = _ns_cfg(nx=n, ny=n, reynolds=50.0)
    h = 2 * math.pi / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    U = 0.2
    p0 = 1.0 / (cfg.gamma * cfg.mach ** 2)
    rho = np.ones_like(X)
    u = U * np.sin(Y)
    q = np.stack([rho, rho * u, 0 * rho, p0 / (cfg.gamma - 1) + 0.5 * rho * u * u])
    m = models.Model(cfg, "fine")
    r = m.rhs(q)
    # p_t = (gamma - 1)(E_t - d/dt(rho u^2 / 2)) with rho_t = 0 and (rho u)_t = r_m
    dke = u * r[1]
    pt = (cfg.gamma - 1) * (r[3] - dke)
    expected = (cfg.gamma - 1) * cfg.mu * U * U * np.cos(Y) ** 2
    np.testing.assert_allclose(pt, expected, atol=1e-3 * np.max(expected))
    # and the shear decays at nu: (rho u)_t = mu u_yy = -mu u
    np.testing.assert_allclose(r[1], -cfg.mu * u, atol=1e-6 * U)
