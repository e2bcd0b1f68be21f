"""Pins of the oracle's EnKF analysis and MEnKF cycle against the closed-form
Kalman filter, brute-force inverses, invariants and special cases."""

import math

import numpy as np
import pytest

from oracle import cycle, enkf, grids, kf, obs
from synthetic import configs, fields


def _linear_case(n=6, ny=3, N=10, seed=0):
    rng = np.random.default_rng(seed)
    members = rng.standard_normal((N, n))
    Hm = rng.standard_normal((ny, n))
    return members, Hm


def test_ensemble_gain_equals_brute_force_kalman_gain():
    members, Hm = _linear_case()
    sigma = 0.3
    H = lambda x: np.asarray(x) @ Hm.T
    K_e = enkf.gain_matrix(members, H, sigma)
    X = enkf.anomalies(members)
    Pe = X @ X.T
    K_kf = kf.kalman_gain(Pe, Hm, sigma ** 2 * np.eye(Hm.shape[0]))
    np.testing.assert_allclose(K_e, K_kf, rtol=0, atol=1e-12)


def test_analysis_update_uses_that_gain():
    members, Hm = _linear_case(seed=3)
    sigma = 0.2
    H = lambda x: np.asarray(x) @ Hm.T
    rng = np.random.default_rng(5)
    y = rng.standard_normal(Hm.shape[0])
    eps = sigma * rng.standard_normal((members.shape[0], Hm.shape[0]))
    xstar = rng.standard_normal(members.shape[1])
    res = enkf.analysis(members, xstar, y, eps, H, sigma)
    X = enkf.anomalies(members)
    K = kf.kalman_gain(X @ X.T, Hm, sigma ** 2 * np.eye(Hm.shape[0]))
    expected = members + ((y + eps - members @ Hm.T) @ K.T)
    np.testing.assert_allclose(res["members"], expected, atol=1e-12)
    np.testing.assert_allclose(res["delta"], K @ (y - Hm @ xstar), atol=1e-12)


def test_sample_mode_gain_equals_brute_force():
    members, Hm = _linear_case(N=12)
    rng = np.random.default_rng(7)
    eps = 0.1 * rng.standard_normal((12, Hm.shape[0]))
    H = lambda x: np.asarray(x) @ Hm.T
    K_e = enkf.gain_matrix(members, H, None, eps=eps, mode="sample_ee")
    X = enkf.anomalies(members)
    E = enkf.anomalies(eps)
    K_bf = (X @ X.T) @ Hm.T @ np.linalg.inv(Hm @ X @ X.T @ Hm.T + E @ E.T)
    np.testing.assert_allclose(K_e, K_bf, atol=1e-11)


def test_sample_mode_singular_when_too_many_observations():
    """Reading 1: rank(YY^T + EE^T) <= 2(N-1) < N_y makes S singular."""
    N, n_y = 4, 9
    rng = np.random.default_rng(1)
    members = rng.standard_normal((N, 12))
    Hm = rng.standard_normal((n_y, 12))
    eps = rng.standard_normal((N, n_y))
    with pytest.raises(np.linalg.LinAlgError):
        enkf.analysis(members, members[0], np.zeros(n_y), eps, lambda x: np.asarray(x) @ Hm.T,
                      None, mode="sample_ee")


def test_large_ensemble_gain_converges_to_kalman_gain():
    """K^e -> K as N grows, error ~ c / sqrt(N) (sampling error, Sec. 2.1.2)."""
    rng = np.random.default_rng(11)
    n, ny = 3, 2
    A = rng.standard_normal((n, n))
    P = A @ A.T + 0.5 * np.eye(n)
    Hm = rng.standard_normal((ny, n))
    R = 0.3 * np.eye(ny)
    K = kf.kalman_gain(P, Hm, R)
    errs = []
    for N in (1000, 100000):
        members = rng.multivariate_normal(np.zeros(n), P, size=N)
        Ke = enkf.gain_matrix(members, lambda x: np.asarray(x) @ Hm.T, math.sqrt(0.3))
        errs.append(np.max(np.abs(Ke - K)))
    assert errs[1] < 0.05
    assert errs[1] < errs[0]


def test_stochastic_update_reproduces_analysis_covariance():
    """Perturbed observations make the analysed ensemble covariance (I - KH)P."""
    rng = np.random.default_rng(21)
    n, ny, N = 3, 2, 4000
    A = rng.standard_normal((n, n))
    P = A @ A.T + 0.5 * np.eye(n)
    Hm = rng.standard_normal((ny, n))
    sigma = 0.5
    members = rng.multivariate_normal(np.zeros(n), P, size=N)
    eps = sigma * rng.standard_normal((N, ny))
    res = enkf.analysis(members, members.mean(0), np.zeros(ny), eps,
                        lambda x: np.asarray(x) @ Hm.T, sigma)
    Pa = np.cov(res["members"].T)
    Pf = np.cov(members.T)
    K = kf.kalman_gain(Pf, Hm, sigma ** 2 * np.eye(ny))
    expected = (np.eye(n) - K @ Hm) @ Pf
    np.testing.assert_allclose(Pa, expected, atol=0.08 * np.max(np.abs(expected)))


def test_anomaly_columns_conserve_spatial_sums():
    """Zero-spatial-mean member perturbations: every anomaly column sums to 0,
    so the analysis keeps each member's total and delta^C sums to 0."""
    cfg = configs.tiny_1d(n_members=10, n_probes=8)
    rng = np.random.default_rng(2)
    base = np.sin(np.arange(cfg.nxc) * cfg.length / cfg.nxc)
    pert = rng.standard_normal((cfg.n_members, cfg.nxc))
    pert -= pert.mean(axis=1, keepdims=True)
    members = (base + 0.05 * pert)[:, None, :]
    idx, comp = fields.probes_for(cfg)
    H = cycle.make_H(cfg, idx, comp)
    y = rng.standard_normal(cfg.n_probes) * 0.1
    eps = 0.02 * rng.standard_normal((cfg.n_members, cfg.n_probes))
    res = enkf.analysis(members, members.mean(0), y, eps, H, cfg.obs_sigma)
    np.testing.assert_allclose(res["members"].sum(axis=-1), members.sum(axis=-1), atol=1e-12)
    assert abs(res["delta"].sum()) < 1e-12


def test_unit_ratio_without_sweeps_is_plain_enkf_on_the_fine_grid():
    """r_C = 1 and no smoothing: x^F_a = x^F_f + K^e (y^o - H x^F_f) exactly."""
    cfg = configs.tiny_1d(ratio=1, nx=64, n_probes=8, n_members=10)
    idx, comp = fields.probes_for(cfg)
    rng = np.random.default_rng(4)
    fine = fields.burgers_model_ic(cfg)
    members = fine[None] + 0.05 * rng.standard_normal((cfg.n_members, 1, cfg.nx))
    st = cycle.State(fine=fine, members=members)
    y = rng.standard_normal(cfg.n_probes) * 0.1
    new, parts = cycle.cycle(cfg, st, y, idx, comp, n_sweeps=0, return_parts=True)
    H = cycle.make_H(cfg, idx, comp)
    K = enkf.gain_matrix(parts["members_f"], H, cfg.obs_sigma)
    xf = parts["xf"]
    expected = xf.reshape(-1) + K @ (y - obs.observe_fine(xf, idx, comp, 1))
    np.testing.assert_allclose(new.fine.reshape(-1), expected, atol=1e-12)


def test_coarse_observation_is_fine_observation_of_prolongation():
    cfg = configs.tiny_2d()
    idx, comp = fields.probes_for(cfg)
    rng = np.random.default_rng(8)
    xc = fields.ns_member_ics(cfg)[:3] + 0.01 * rng.standard_normal((3, 4, cfg.nyc, cfg.nxc))
    full = obs.observe_fine(grids.prolong(xc, cfg.ratio, 2), idx, comp, 2)
    fast = obs.observe_coarse(xc, idx, comp, 2, cfg.ratio, cfg.nx)
    np.testing.assert_allclose(fast, full, rtol=1e-13)
