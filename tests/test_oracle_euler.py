"""Pins of the inlet-forced 1D Euler oracle (the acoustic case): the filter's
transfer functions on Fourier modes, the telescoping sum of the centred
flux differences, the uniform inlet state as a fixed point, the acoustic
speeds u0 +- a of a small pulse, and the relaxed iteration converging to
the implicit-Euler solution."""

import numpy as np

from oracle import dual, euler1d as E
from synthetic import configs, fields

G, M = 1.4, 0.4


def test_filter_transfer_functions_on_a_fourier_mode():
    n = 64
    for kh in (0.3, 1.1, 2.0, np.pi):
        for sig in (0.2, 1.0):
            x = np.cos(kh * np.arange(n) + 0.4)[None, :]
            y = E.filter_open(x, sig)
            s2 = np.sin(kh / 2) ** 2
            np.testing.assert_allclose(y[0, 3:n - 3], (1 - sig * s2 ** 3) * x[0, 3:n - 3], atol=1e-14)
            for i in (2, n - 3):
                np.testing.assert_allclose(y[0, i], (1 - sig * s2 ** 2) * x[0, i], atol=1e-14)
            for i in (1, n - 2):
                np.testing.assert_allclose(y[0, i], (1 - sig * s2) * x[0, i], atol=1e-14)
            assert y[0, 0] == x[0, 0] and y[0, -1] == x[0, -1]


def test_centred_flux_differences_telescope():
    """sum over the interior of R(x) h = -(F_{n-1} + F_{n-2} - F_1 - F_0) / 2:
    what leaves the domain through the two end cells."""
    g = np.random.default_rng(4)
    n, h = 50, 0.1
    x = E.uniform(n, G, M) * (1 + 0.05 * g.standard_normal((3, n)))
    f = E.flux(x, G)
    lhs = E.rhs(x, G, h).sum(axis=-1) * h
    rhs = -(f[:, -1] + f[:, -2] - f[:, 1] - f[:, 0]) / 2.0
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)
    # the flux itself: a state at rest has F = (0, p, 0)
    rest = np.stack([np.full(3, 1.3), np.zeros(3), np.full(3, 2.0)])
    np.testing.assert_allclose(E.flux(rest, G), np.stack([np.zeros(3), np.full(3, 0.4 * 2.0), np.zeros(3)]))


def test_uniform_inlet_state_is_a_fixed_point():
    x = E.uniform(120, G, M)
    out, prev = E.forecast(x, 0.3, 200, 6e-4, np.array([0.0, 0.0]), 0.0125, G, M, 2 * np.pi, 1.0)
    np.testing.assert_allclose(out, x, rtol=0, atol=1e-15)
    a, u0, rho0, p0, E0 = E.reference_state(G, M)
    assert abs(u0 + a - 1.0) < 1e-15 and abs(u0 / a - M) < 1e-15
    assert abs((G - 1) * (rho0 * E0 - 0.5 * rho0 * u0 * u0) - p0) < 1e-15


def test_small_pulse_splits_at_the_acoustic_speeds():
    """A small density/pressure bump in the uniform flow splits into two
    pulses moving at u0 + a = 1 and u0 - a; their centroids after T = 2
    land within 2 % of those distances."""
    n, L = 2000, 10.0
    h = L / n
    xs = np.arange(n) * h
    a, u0, rho0, p0, E0 = E.reference_state(G, M)
    bump = 1e-4 * np.exp(-((xs - 5.0) / 0.15) ** 2)
    x = E.uniform(n, G, M)
    x[0] += bump                       # rho' at fixed velocity u0
    x[1] += u0 * bump
    p = p0 + a * a * bump              # isentropic p'
    x[2] = p / (G - 1) + 0.5 * x[1] ** 2 / x[0]
    dt, T = 1e-3, 2.0
    out, _ = E.forecast(x, 0.0, int(round(T / dt)), dt, np.array([0.0, 0.0]), h, G, M, 2 * np.pi, 1.0)
    d = out[0] - rho0
    right = xs > 5.0 + u0 * T
    left = xs < 5.0 + u0 * T
    cr = (xs[right] * d[right]).sum() / d[right].sum()
    cl = (xs[left] * d[left]).sum() / d[left].sum()
    assert abs((cr - 5.0) - (u0 + a) * T) < 0.02 * (u0 + a) * T, cr
    assert abs((cl - 5.0) - (u0 - a) * T) < 0.02 * abs(u0 - a) * T, cl


def test_relaxed_iteration_solves_the_implicit_system():
    cfg = configs.euler_inlet()
    g = np.random.default_rng(8)
    n, h = 100, 0.0125
    x = E.uniform(n, G, M) * (1 + 0.01 * np.sin(np.arange(n) / 5.0))[None, :]
    xp = x - 1e-4 * g.standard_normal((3, n))
    y = E.sweep(x, xp, cfg.dt, h, G, 1.0, 300)
    r = xp + cfg.dt * E.rhs(y, G, h) - y
    assert np.abs(r[:, 1:-1]).max() < 1e-14
    assert np.all(y[:, 0] == x[:, 0])
    np.testing.assert_allclose(y[:, -1], 2 * y[:, -2] - y[:, -3], atol=1e-15)
    # one relaxed iteration with alpha = 0.5 moves halfway to the plain iterate
    y1 = E.sweep(x, xp, cfg.dt, h, G, 0.5, 1)
    full = x + (xp + cfg.dt * E.rhs(x, G, h) - x)
    np.testing.assert_allclose(y1[:, 1:-1], 0.5 * (x + full)[:, 1:-1], atol=1e-15)


def test_euler_observation_is_the_momentum():
    cfg = configs.euler_inlet(n_members=3)
    idx, _ = fields.probes_for(cfg)
    xc = fields.inlet_uniform(cfg, "coarse", 3) * 1.01
    y = dual.observe_coarse_open(xc, idx, cfg.ratio, dual.observed_field(cfg))
    a, u0, rho0, p0, E0 = E.reference_state(cfg.gamma, cfg.mach)
    np.testing.assert_allclose(y, 1.01 * rho0 * u0, rtol=1e-14)
