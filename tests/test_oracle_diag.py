"""Pins of the oracle's diagnostics against closed forms: the relative RMSE
(Sec. 4), the ensemble spread (trace of the ensemble covariance of
Sec. 2.1.2), the conservativity indicator Gamma (Sec. 6) and the filter's
only external sanity check, assimilated RMSE below the free run's."""

import math

import numpy as np
import pytest

from oracle import cycle, diag, enkf
from oracle.models import Model
from synthetic import configs, fields


def _ns_state(rho, u, v, p, gamma=1.4):
    """Conservative (rho, rho u, rho v, E) from primitives, independent of the oracle."""
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E])


# ----------------------------------------------------------------- RMSE
def test_velocity_rmse_known_error():
    """Truth u = 1, v = 0 everywhere; analysis off by (+0.03, -0.04) on half
    the nodes and exact elsewhere: RMSE = sqrt(n/2 * 0.05^2 / n)."""
    ny, nx = 6, 10
    one = np.ones((ny, nx))
    qt = _ns_state(2.0 * one, one, 0 * one, 5.0 * one)
    ua, va = one.copy(), 0 * one
    ua[:, ::2] += 0.03
    va[:, ::2] -= 0.04
    qa = _ns_state(0.5 + one, ua, va, 7.0 * one)        # other density/pressure: velocity only counts
    assert diag.velocity_rmse(qa, qt) == pytest.approx(math.sqrt(0.5) * 0.05, rel=1e-13)


def test_velocity_rmse_counts_both_components():
    """Truth (u, v) = (3, 4) (|u| = 5), analysis (3, 4 + d): RMSE = d / 5."""
    one = np.ones((4, 4))
    qt = _ns_state(one, 3 * one, 4 * one, one)
    qa = _ns_state(one, 3 * one, (4 + 0.2) * one, one)
    assert diag.velocity_rmse(qa, qt) == pytest.approx(0.2 / 5.0, rel=1e-13)


def test_rel_rmse_scales():
    x = np.linspace(1.0, 2.0, 50)
    assert diag.rel_rmse(1.1 * x, x) == pytest.approx(0.1, rel=1e-13)
    assert diag.rel_rmse(x, x) == 0.0


# ----------------------------------------------------------------- spread
def test_spread_closed_form_1d():
    """Members c(x) + s_i phi(x) with sum_i s_i = 0: the ensemble mean is c
    and the covariance trace is sum_x phi^2 * sum_i s_i^2 / (N - 1)."""
    n = 37
    x = np.linspace(0, 2 * np.pi, n, endpoint=False)
    c = 1.0 + 0.5 * np.sin(x)
    phi = np.cos(2 * x) + 0.25
    s = np.array([0.3, -0.1, -0.5, 0.2, 0.1])
    mem = (c[None] + s[:, None] * phi[None])[:, None, :]
    a, b = diag.spread_sums(mem, 1)
    assert a == pytest.approx(np.sum(phi ** 2) * np.sum(s ** 2) / 4.0, rel=1e-13)
    assert b == pytest.approx(np.sum(c ** 2), rel=1e-13)
    assert diag.ensemble_spread(mem, 1) == pytest.approx(math.sqrt(a / b), rel=1e-15)


def test_spread_is_trace_of_anomaly_covariance():
    """trace(X X^T) with the analysis's own normalised anomalies."""
    cfg = configs.tiny_1d()
    mem = fields.member_ics(cfg)
    X = enkf.anomalies(mem.reshape(cfg.n_members, -1))
    a, _ = diag.spread_sums(mem, 1)
    assert a == pytest.approx(float(np.sum(X * X)), rel=1e-12)


def test_spread_2d_uses_velocity_and_euler_uses_momentum():
    one = np.ones((5, 8))
    s = np.array([0.2, -0.2, 0.05, -0.05])
    mem = np.stack([_ns_state(3.0 * one, (1.0 + si) * one, -0.5 * one, 2.0 * one) for si in s])
    a, b = diag.spread_sums(mem, 2)
    assert a == pytest.approx(40 * np.sum(s ** 2) / 3.0, rel=1e-13)      # v has no spread
    assert b == pytest.approx(40 * (1.0 + 0.25), rel=1e-13)
    eul = np.zeros((3, 3, 6))
    eul[:, 1] = np.array([1.0, 2.0, 3.0])[:, None]                       # rho u of three members
    eul[:, 0] = 7.0
    a, b = diag.spread_sums(eul, 1, obs_field=1)
    assert a == pytest.approx(6 * 2.0 / 2.0, rel=1e-13)                 # deviations -1, 0, 1
    assert b == pytest.approx(6 * 4.0, rel=1e-13)


# ----------------------------------------------------------------- Gamma
def _tiny_ns(n=12):
    return configs.tiny_2d(nx=n, ny=n, precision="f64")


def test_gamma_vanishes_on_the_implicit_euler_step():
    """Gamma = 0 when x_k solves x_k - dt F(x_k) = x_{k-1} (the paper: Gamma
    is zero after a model step); the step is found by fixed-point iteration
    to roundoff, independently of the sweep code."""
    cfg = _tiny_ns()
    m = Model(cfg, "fine")
    xp = fields.truth_ic(cfg)
    z = xp.copy()
    for _ in range(60):
        z = xp + m.dt * m.rhs(z)
    g = diag.gamma_rhov(z, xp, m)
    scale = np.max(np.abs(m.rhs(z)[2]))
    assert np.max(np.abs(g)) < 1e-9 * scale
    # a non-solution (the explicit step) leaves a residual of order dt |F'F|
    ze = xp + m.dt * m.rhs(xp)
    assert np.max(np.abs(diag.gamma_rhov(ze, xp, m))) > 1e3 * np.max(np.abs(g))


def test_gamma_closed_form_on_a_density_wave():
    """Uniform u, v, p and rho = 1 + a sin(x + 2y): every viscous term of the
    rho v equation vanishes and F_{rho v} = -(u v d_x rho + v^2 d_y rho),
    with the fourth-order difference of sin(k x) equal to
    k kappa(k h) cos(k x), kappa(t) = (8 sin t - sin 2t) / (6 t).  With
    x_{k-1} = x_k - dt G the indicator is G_{rho v} - F_{rho v}(x_k)."""
    n = 16
    cfg = _tiny_ns(n)
    m = Model(cfg, "fine")
    h = cfg.length / n
    xs = np.arange(n) * h
    X, Y = np.meshgrid(xs, xs)
    a, u0, v0, p0 = 0.2, 0.3, -0.4, 5.0
    ph = X + 2 * Y
    q = _ns_state(1 + a * np.sin(ph), u0 + 0 * X, v0 + 0 * X, p0 + 0 * X, cfg.gamma)
    G = np.zeros_like(q)
    G[2] = 0.7 * np.cos(X)
    qp = q - m.dt * G
    kap = lambda k: (8 * np.sin(k * h) - np.sin(2 * k * h)) / (6 * k * h)
    drho_x = a * 1 * kap(1) * np.cos(ph)
    drho_y = a * 2 * kap(2) * np.cos(ph)
    F_rv = -(u0 * v0 * drho_x + v0 * v0 * drho_y)
    np.testing.assert_allclose(diag.gamma_rhov(q, qp, m), G[2] - F_rv, rtol=0, atol=1e-11)
    gn = diag.gamma_normalised(q, qp, m)
    np.testing.assert_allclose(gn, (G[2] - F_rv) / 0.7, rtol=0, atol=1e-11)


# ----------------------------------------------------------------- filter sanity
def test_assimilation_beats_the_free_run_c1():
    """All 20 cycles of the 1D FP64 workload: the analysed fine state's
    relative RMSE (second-half mean, Sec. 4 RMSE) is below the free run's
    (same model and initial state, no analysis) by more than 10 %, and the
    ensemble spread shrinks as observations are assimilated."""
    cfg = configs.CONFIGS["C1"]
    idx, comp = fields.probes_for(cfg)
    truth = fields.truth_ic(cfg)
    st = cycle.State(fine=fields.model_ic(cfg), members=fields.member_ics(cfg))
    free = cycle.free_run(cfg, fields.model_ic(cfg), cfg.n_cycles)
    mt = Model(cfg, "fine")
    ra, rf, sp = [], [], [diag.ensemble_spread(st.members, 1)]
    for c in range(1, cfg.n_cycles + 1):
        truth, _ = mt.forecast(truth, cfg.n_obs)
        y = cycle.observe_truth(cfg, truth, idx, comp) + fields.obs_noise(cfg, c)
        st = cycle.cycle(cfg, st, y, idx, comp, n_sweeps=1, seed=cfg.seed + 5)
        ra.append(diag.rel_rmse(st.fine, truth))
        rf.append(diag.rel_rmse(free[c - 1], truth))
        sp.append(diag.ensemble_spread(st.members, 1))
    half = cfg.n_cycles // 2
    assert np.mean(ra[half:]) < 0.9 * np.mean(rf[half:]), (np.mean(ra[half:]), np.mean(rf[half:]))
    assert sp[-1] < 0.5 * sp[0]


def test_rmse_sums_agree_with_the_rmse_functions():
    cfg = configs.tiny_2d(precision="f64")
    qt = fields.truth_ic(cfg)
    qa = fields.model_ic(cfg)
    a, b = diag.rmse_sums(qa, qt, 2)
    assert math.sqrt(a / b) == pytest.approx(diag.velocity_rmse(qa, qt), rel=1e-14)
    x = np.linspace(0.5, 1.5, 20)[None]
    a, b = diag.rmse_sums(1.2 * x, x, 1)
    assert (a, b) == (pytest.approx(0.04 * np.sum(x ** 2), rel=1e-14), pytest.approx(np.sum(x ** 2), rel=1e-14))
