"""Pins of the oracle's smoothing iteration, random numbers, diagnostics and
learned-prolongation network."""

import math
import os

import numpy as np
import pytest
import scipy.optimize

from oracle import cycle, diag, enkf, grids, net, rng, smooth
from oracle.models import Model
from synthetic import configs, fields


# ----------------------------------------------------------------- smoothing
def test_sweeps_converge_to_the_implicit_euler_step():
    cfg = configs.tiny_1d(nx=32, nu=0.05, dt=2e-3)
    m = Model(cfg, "fine")
    x_prev = np.sin(np.arange(32) * m.h)[None] + 0.2 * np.cos(3 * np.arange(32) * m.h)[None]
    direct = scipy.optimize.fsolve(lambda z: z - m.dt * m.rhs(z[None])[0] - x_prev[0],
                                   x_prev[0], xtol=1e-14)
    x = x_prev + 0.3
    x = smooth.smooth(x, x_prev, m, 400, alpha=0.5)
    np.testing.assert_allclose(x[0], direct, atol=1e-11)


def test_sweep_fixed_point_is_implicit_euler_solution():
    cfg = configs.tiny_1d(nx=32, nu=0.05, dt=2e-3)
    m = Model(cfg, "fine")
    xp = np.cos(np.arange(32) * m.h)[None]
    sol = scipy.optimize.fsolve(lambda z: z - m.dt * m.rhs(z[None])[0] - xp[0], xp[0], xtol=1e-14)
    out = smooth.sweep(sol[None], xp, m, 0.5)
    np.testing.assert_allclose(out[0], sol, atol=1e-13)


def test_one_sweep_on_linear_diffusion_is_the_jacobi_matrix():
    """Zero-amplitude-advection limit: F = nu D2, so a sweep is
    x + alpha/D (b + dt nu D2 x - x) with D = 1 + 2 dt nu / h^2."""
    cfg = configs.tiny_1d(nx=16, nu=0.1, dt=1e-2)
    m = Model(cfg, "fine")
    n = 16
    D2 = (np.roll(np.eye(n), 1, 0) - 2 * np.eye(n) + np.roll(np.eye(n), -1, 0)) / m.h ** 2
    A = np.eye(n) - m.dt * cfg.nu * D2
    Dd = np.diag(A)[0]
    assert abs(Dd - m.diag_coeff()) < 1e-14
    rng_ = np.random.default_rng(0)
    x = 1e-9 * rng_.standard_normal(n)          # advection term u u_x ~ 1e-18: negligible
    b = 1e-9 * rng_.standard_normal(n)
    expected = x + 0.5 / Dd * (b - A @ x)
    got = smooth.sweep(x[None], b[None], m, 0.5)[0]
    np.testing.assert_allclose(got, expected, rtol=1e-7, atol=0)


def test_gamma_decreases_with_sweeps():
    """Conservativity residual after an analysis shrinks with more sweeps (Sec. 6)."""
    cfg = configs.tiny_2d(nx=32, ny=32, n_members=8, n_probes=16)
    idx, comp = fields.probes_for(cfg)
    truth = fields.ns_truth_ic(cfg)
    st = cycle.State(fine=fields.ns_model_ic(cfg), members=fields.ns_member_ics(cfg))
    mt = Model(cfg, "fine")
    truth, _ = mt.forecast(truth, cfg.n_obs)
    y = cycle.observe_truth(cfg, truth, idx, comp) + fields.obs_noise(cfg, 1)
    g = []
    for ns in (0, 1, 3):
        new, parts = cycle.cycle(cfg, st, y, idx, comp, n_sweeps=ns, return_parts=True)
        g.append(np.sqrt(np.mean(diag.gamma_rhov(new.fine, parts["xf_prev"], mt) ** 2)))
    assert g[0] > g[1] > g[2], g


# ----------------------------------------------------------------- rng
def _kat(golden_dir):
    out = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            out.append((v[:4], v[4:6], v[6:]))
    return out


def test_philox_known_answers(golden_dir):
    for ctr, key, expected in _kat(golden_dir):
        got = rng.philox4x32_10([np.uint64(c) for c in ctr], [np.uint64(k) for k in key])
        assert [int(g) for g in got] == expected


def test_perturbation_moments():
    e = rng.perturbations(1234, 7, 64, 4096, 1.0)
    n = e.size
    assert abs(e.mean()) < 4 / math.sqrt(n)
    assert abs(e.var() - 1) < 4 * math.sqrt(2 / n)
    assert abs(np.mean(e ** 4) - 3) < 0.05
    e2 = rng.perturbations(1234, 8, 64, 4096, 1.0)
    assert abs(np.corrcoef(e.ravel(), e2.ravel())[0, 1]) < 4 / math.sqrt(n)


def test_perturbations_scale_and_are_deterministic():
    a = rng.perturbations(99, 3, 5, 10, 0.02)
    b = rng.perturbations(99, 3, 5, 10, 1.0)
    np.testing.assert_array_equal(a, 0.02 * b)
    np.testing.assert_array_equal(a, rng.perturbations(99, 3, 5, 10, 0.02))


# ----------------------------------------------------------------- diagnostics
def test_rel_rmse_definition():
    xt = np.array([3.0, 4.0])
    assert diag.rel_rmse(xt, xt) == 0.0
    assert abs(diag.rel_rmse(np.array([3.0, 0.0]), xt) - 4.0 / 5.0) < 1e-15


# ----------------------------------------------------------------- network
def _brute_conv(x, w, b):
    C, H, W = x.shape
    O = w.shape[0]
    out = np.zeros((O, H, W))
    for o in range(O):
        for yy in range(H):
            for xx in range(W):
                s = b[o]
                for c in range(C):
                    for a in range(3):
                        for bb in range(3):
                            s += w[o, c, a, bb] * x[c, (yy + a - 1) % H, (xx + bb - 1) % W]
                out[o, yy, xx] = s
    return out


def test_conv_matches_brute_force_loops():
    r = np.random.default_rng(0)
    x = r.standard_normal((3, 5, 4))
    w = r.standard_normal((2, 3, 3, 3))
    b = r.standard_normal(2)
    np.testing.assert_allclose(net.conv(x, w, b), _brute_conv(x, w, b), atol=1e-13)


def test_network_gradients_match_central_differences():
    cfg = configs.tiny_2d()
    p = net.init_params(cfg, seed=3, zero_last=False)
    r = np.random.default_rng(1)
    inp = r.standard_normal((2, 8, 6, 5))
    tgt = r.standard_normal((2, 4, 6, 5))
    out, cache = net.forward(p, inp)
    loss, g = net.mse(out, tgt)
    grads, dinp = net.backward(p, cache, g)
    h = 1e-6
    for ti, t in enumerate(p.tensors()):
        flat = t.reshape(-1)
        for j in r.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[j]
            flat[j] = old + h
            lp, _ = net.mse(net.forward(p, inp)[0], tgt)
            flat[j] = old - h
            lm, _ = net.mse(net.forward(p, inp)[0], tgt)
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            an = grads[ti].reshape(-1)[j]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (ti, j, fd, an)
    flat = inp.reshape(-1)
    for j in r.choice(flat.size, size=6, replace=False):
        old = flat[j]
        flat[j] = old + h
        lp, _ = net.mse(net.forward(p, inp)[0], tgt)
        flat[j] = old - h
        lm, _ = net.mse(net.forward(p, inp)[0], tgt)
        flat[j] = old
        assert abs((lp - lm) / (2 * h) - dinp.reshape(-1)[j]) < 1e-7


def test_zero_last_layer_is_plain_prolongation():
    cfg = configs.tiny_2d()
    p = net.init_params(cfg, seed=0, zero_last=True)
    r = np.random.default_rng(2)
    dc = 0.01 * r.standard_normal((4, cfg.nyc, cfg.nxc))
    dproj = grids.prolong(dc, cfg.ratio, 2)
    xf = fields.ns_model_ic(cfg)
    np.testing.assert_array_equal(net.learned_correction(p, dproj, xf), dproj)


def test_adam_first_step_is_lr_times_sign():
    t = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -0.1, 1e-3])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    net.adam_update(t, g, m, v, 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(t[0], [0.99, -1.99, 2.99], atol=1e-15)
