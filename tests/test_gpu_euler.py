"""GPU parity of the inlet-forced 1D Euler model (the acoustic case,
MENKF_EULER1D_INLET) against the oracle: forecasts with the filter and the
inlet/outlet rows, the momentum observation, the fine correction and
relaxed iterations, whole dual cycles, and tracking of the time-varying
inlet amplitude at the Sec. 5 size."""

import numpy as np
import pytest
import torch

from oracle import dual, euler1d as E
from synthetic import configs, fields
from tests.gpu_helpers import make_ctx, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu

F64 = torch.float64


def _dt(cfg):
    return torch.float64 if cfg.precision == "f64" else torch.float32


def _round(x, cfg):
    x = np.asarray(x, dtype=np.float64)
    return x if cfg.precision == "f64" else x.astype(np.float32).astype(np.float64)


def _states(cfg, level, nb, seed):
    """Uniform inlet states plus small smooth acoustic-like perturbations."""
    n = cfg.nx if level == "fine" else cfg.nxc
    g = np.random.default_rng(seed)
    x = np.arange(n) * (cfg.length / n)
    out = fields.inlet_uniform(cfg, level, nb).copy()
    for k in range(1, 4):
        for f in range(3):
            a = 2e-3 / k * g.standard_normal((nb, 1))
            ph = g.uniform(0, 2 * np.pi, (nb, 1))
            out[:, f] *= 1 + a * np.sin(2 * np.pi * k * x / cfg.length + ph)
    return _round(out, cfg)


def _thetas(nb, seed):
    g = np.random.default_rng(seed)
    return np.stack([0.015 + 0.008 * g.standard_normal(nb), np.zeros(nb)], axis=1)


def _forecast(cfg, x, t0, nsteps, theta, level):
    h = cfg.length / (cfg.nx if level == "fine" else cfg.nxc)
    return E.forecast(x, t0, nsteps, cfg.dt, theta, h, cfg.gamma, cfg.mach, cfg.omega, cfg.filter_sigma)


CASES = [
    (configs.euler_inlet(nx=200, ratio=4, n_members=12, n_probes=16), 1e-12),
    (configs.euler_inlet(n_members=100), 1e-12),                                 # Sec. 5 size, F64
    (configs.euler_inlet(nx=1600, ratio=8, n_members=6, n_probes=16), 1e-12),    # 2 nodes per thread
    (configs.euler_inlet(precision="f32", n_members=100), None),
]
CASE_IDS = ["200r4-f64", "800r4-f64", "1600r8-f64", "800r4-f32"]


@pytest.mark.parametrize("cfg,tol", CASES, ids=CASE_IDS)
@pytest.mark.parametrize("nsteps", [1, 37, 300])
def test_euler_forecast_matches_oracle(cfg, tol, nsteps):
    if tol is None:
        # FP32: a few roundings per step (update, filter), of one sign when
        # the increments vary slowly
        tol = 1e-6 + 4 * nsteps * 2.0 ** -24
    ctx, _, _ = make_ctx(cfg)
    dt = _dt(cfg)
    t0 = 0.37
    t0_d = torch.tensor([t0], dtype=F64, device="cuda")
    for level, nb in (("fine", 1), ("coarse", cfg.n_members)):
        say(f"euler forecast {cfg.name} {cfg.precision} {level} nb={nb} nsteps={nsteps}")
        x0 = _states(cfg, level, nb, 3 + nb)
        th = _thetas(nb, 7 + nb)
        want, want_prev = _forecast(cfg, x0, t0, nsteps, th, level)
        x_d = to_dev(x0 if level == "coarse" else x0[0], dt)
        prev_d = torch.empty_like(x_d)
        ctx.forecast_inlet(0 if level == "fine" else 1, x_d, nsteps, to_dev(th, F64), t0_d, prev=prev_d)
        got = to_np(x_d).reshape(want.shape)
        gprev = to_np(prev_d).reshape(want.shape)
        assert rel_l2(got, want) < tol, (level, rel_l2(got, want))
        assert rel_l2(gprev, want_prev) < tol, (level, rel_l2(gprev, want_prev))
        # inlet row: (rho0, rho0 u_in(t_end), rho0 E0)
        a, u0, rho0, p0, E0 = E.reference_state(cfg.gamma, cfg.mach)
        t_end = (t0 + (nsteps - 1) * cfg.dt) + cfg.dt
        uin = u0 * (1.0 + th[:, 0] * np.sin(cfg.omega * t_end + th[:, 1]))
        rt = 1e-15 if cfg.precision == "f64" else 1e-7
        np.testing.assert_allclose(got[:, 1, 0], rho0 * uin, rtol=rt)
        np.testing.assert_allclose(got[:, 0, 0], rho0, rtol=rt)
        np.testing.assert_allclose(got[:, 2, 0], rho0 * E0, rtol=rt)
        if cfg.precision == "f64":
            np.testing.assert_allclose(got[..., -1], 2 * got[..., -2] - got[..., -3], rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("cfg,tol", [CASES[0], CASES[1], CASES[3]], ids=[CASE_IDS[0], CASE_IDS[1], CASE_IDS[3]])
def test_euler_observes_the_momentum(cfg, tol):
    ctx, _, _ = make_ctx(cfg)
    g = np.random.default_rng(1)
    ends = np.array([0, 1, 2, cfg.nx - 3, cfg.nx - 2, cfg.nx - 1])
    rest = g.choice(np.arange(3, cfg.nx - 3), cfg.n_probes - len(ends), replace=False)
    idx = np.sort(np.concatenate([ends, rest])).astype(np.int32)
    ctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.zeros(cfg.n_probes, dtype=torch.int32, device="cuda"))
    mem = _states(cfg, "coarse", cfg.n_members, 5)
    say(f"euler observation {cfg.name} {cfg.precision}")
    y = to_np(ctx.observe(1, to_dev(mem, _dt(cfg))))
    want = dual.observe_coarse_open(mem, idx, cfg.ratio, field=1)
    assert rel_l2(y, want) < 1e-14, rel_l2(y, want)
    xf = _states(cfg, "fine", 1, 9)[0]
    yf = to_np(ctx.observe(0, to_dev(xf, _dt(cfg))))
    np.testing.assert_array_equal(yf[0], xf[1, idx])
    # diagnostics read the same field
    out = to_np(ctx.diagnostics(to_dev(xf, _dt(cfg)), to_dev(0.5 * xf, _dt(cfg))))
    np.testing.assert_allclose(out[0], ((0.5 * xf[1]) ** 2).sum(), rtol=1e-12)
    np.testing.assert_allclose(out[1], ((0.5 * xf[1]) ** 2).sum(), rtol=1e-12)


@pytest.mark.parametrize("cfg,tol", [CASES[0], CASES[1], CASES[3]], ids=[CASE_IDS[0], CASE_IDS[1], CASE_IDS[3]])
@pytest.mark.parametrize("n_sweeps", [0, 1, 2, 3])
def test_euler_correction_and_sweeps_match_oracle(cfg, tol, n_sweeps):
    tol = tol or 2e-6
    ctx, _, _ = make_ctx(cfg)
    dt = _dt(cfg)
    xf = _states(cfg, "fine", 1, 11)[0]
    xprev = _round(xf * (1 - 1e-4 * np.cos(np.arange(cfg.nx) / 7.0))[None, :], cfg)
    delta = _round(1e-3 * np.random.default_rng(2).standard_normal((3, cfg.nxc)), cfg)
    say(f"euler prolong+smooth {cfg.name} {cfg.precision} sweeps={n_sweeps}")
    x_d = to_dev(xf, dt)
    ctx.prolong_smooth(to_dev(delta, dt), x_d, to_dev(xprev, dt), n_sweeps=n_sweeps, alpha=0.5)
    x = dual.correct_open(xf, delta, cfg.ratio)
    want = E.sweep(x, xprev, cfg.dt, cfg.length / cfg.nx, cfg.gamma, 0.5, n_sweeps)
    got = to_np(x_d)
    assert rel_l2(got, want) < tol, rel_l2(got, want)
    assert np.all(got[:, 0] == xf[:, 0])


def _truth_fn(cfg):
    return lambda t: np.array([E.amplitude_truth(t, cfg.theta_true[0], cfg.omega / cfg.theta_b), 0.0])


def _spun_up_truth(cfg):
    th = _truth_fn(cfg)
    x, _ = E.forecast(fields.inlet_uniform(cfg), 0.0, int(round(cfg.t_spinup / cfg.dt)), cfg.dt, None,
                      cfg.length / cfg.nx, cfg.gamma, cfg.mach, cfg.omega, cfg.filter_sigma, theta_of_t=th)
    return x


class _Dev:
    def __init__(self, ctx, cfg, st):
        dt = _dt(cfg)
        self.fine = to_dev(st.fine, dt)
        self.prev = torch.empty_like(self.fine)
        self.mem = to_dev(st.members, dt)
        self.xs = torch.empty((3, cfg.nxc), dtype=dt, device="cuda")
        self.dc = torch.empty_like(self.xs)
        self.theta = to_dev(st.theta, F64)
        self.tm = torch.empty(2, dtype=F64, device="cuda")
        self.clock = torch.tensor([st.t], dtype=F64, device="cuda")
        self.y = torch.empty(cfg.n_probes, dtype=F64, device="cuda")
        self.ctx, self.cfg = ctx, cfg

    def cycle(self, seed, c, n_sweeps, stream=None, aux_stream=None):
        self.ctx.dual_cycle(self.fine, self.prev, self.mem, self.xs, self.dc, self.y, self.theta, self.tm,
                            self.clock, seed, c, self.cfg.n_obs, n_sweeps=n_sweeps, alpha=0.5, stream=stream,
                            aux_stream=aux_stream)


@pytest.mark.parametrize("cfg,tol,ncyc", [
    (configs.euler_inlet(nx=200, ratio=2, n_members=40, n_probes=20), 1e-10, 6),
    (configs.euler_inlet(n_members=100), 1e-10, 3),
    (configs.euler_inlet(precision="f32", n_members=100), None, 3),
], ids=["200r2-f64", "800r4-f64", "800r4-f32"])
def test_euler_dual_cycles_match_oracle(cfg, tol, ncyc):
    ctx, idx, _ = make_ctx(cfg)
    truth = _spun_up_truth(cfg.with_(t_spinup=1.0))
    st = dual.DualState(fine=fields.inlet_uniform(cfg), members=_states(cfg, "coarse", cfg.n_members, 4),
                        theta=fields.inlet_theta_ics(cfg), t=0.0)
    dev = _Dev(ctx, cfg, st)
    th = _truth_fn(cfg)
    hf = cfg.length / cfg.nx
    seed = cfg.seed + 5
    t = 0.0
    for c in range(1, ncyc + 1):
        truth, _ = E.forecast(truth, t, cfg.n_obs, cfg.dt, None, hf, cfg.gamma, cfg.mach, cfg.omega,
                              cfg.filter_sigma, theta_of_t=th)
        t += cfg.n_obs * cfg.dt
        y = truth[1, idx] + fields.obs_noise(cfg, c)
        say(f"euler dual cycle {cfg.name} {cfg.precision} cycle {c}")
        st, tb = dual.dual_cycle(cfg, st, y, idx, n_sweeps=1, seed=seed)
        dev.y.copy_(torch.as_tensor(y, dtype=F64))
        dev.cycle(seed, c, 1, aux_stream=torch.cuda.Stream() if c % 2 else None)
        assert ctx.get_status() == 0
        tol_theta = tol
        if cfg.precision == "f32":
            # states: the forecast bound over the c windows so far; parameters:
            # the innovations are ~sigma_obs while the observed momentum is
            # ~rho0 u0, so a relative state error e moves them by
            # e rho0 u0 / sigma_obs relative
            tol = 1e-5 + 4 * cfg.n_obs * c * 2.0 ** -24
            a, u0, rho0, _, _ = E.reference_state(cfg.gamma, cfg.mach)
            tol_theta = tol * rho0 * u0 / cfg.obs_sigma
        assert rel_l2(to_np(dev.theta), st.theta) < tol_theta, (c, rel_l2(to_np(dev.theta), st.theta))
        assert rel_l2(to_np(dev.tm), tb) < tol_theta, c
        assert rel_l2(to_np(dev.fine), st.fine) < tol, (c, rel_l2(to_np(dev.fine), st.fine))
        assert rel_l2(to_np(dev.mem), st.members) < tol, (c, rel_l2(to_np(dev.mem), st.members))
        assert to_np(dev.clock)[0] == st.t


def test_euler_dual_tracks_the_time_varying_amplitude():
    """Sec. 5 size, f_a = 55 (an analysis every 30 steps): from the prior
    theta ~ N(0, 6.4e-5) the mean estimate follows the truth
    theta(t) = 0.015 (1 + sin(2 pi t / 10)) through its first maximum with a
    lag of under 1.5 time units, and the momentum error shrinks as the
    corrected flow fills the domain.  Truth and observations come from the
    oracle's model on the CPU."""
    cfg = configs.euler_inlet(n_members=100)
    ctx, idx, _ = make_ctx(cfg)
    truth = _spun_up_truth(cfg)
    st = dual.DualState(fine=fields.inlet_uniform(cfg), members=fields.inlet_uniform(cfg, "coarse", cfg.n_members),
                        theta=fields.inlet_theta_ics(cfg), t=0.0)
    dev = _Dev(ctx, cfg, st)
    th = _truth_fn(cfg)
    hf = cfg.length / cfg.nx
    t = 0.0
    times, est, errs = [], [], []
    base = fields.inlet_uniform(cfg)[1]
    for c in range(1, 401):
        truth, _ = E.forecast(truth, t, cfg.n_obs, cfg.dt, None, hf, cfg.gamma, cfg.mach, cfg.omega,
                              cfg.filter_sigma, theta_of_t=th)
        t += cfg.n_obs * cfg.dt
        dev.y.copy_(torch.as_tensor(truth[1, idx] + fields.obs_noise(cfg, c), dtype=F64))
        dev.cycle(cfg.seed + 5, c, 1)
        if c % 10 == 0:
            times.append(t)
            est.append(to_np(dev.tm)[0])
            errs.append(rel_l2(to_np(dev.fine)[1] - base, truth[1] - base))
            if c % 50 == 0:
                say(f"euler tracking cycle {c} t={t:.2f}: theta {est[-1]:.5f} truth {th(t)[0]:.5f} "
                    f"momentum-fluctuation error {errs[-1]:.3f}")
    assert ctx.get_status() == 0
    times, est = np.array(times), np.array(est)
    # the estimate rises from 0 and peaks within 1.5 time units after the truth's maximum (t = 2.5)
    assert est.max() > 0.025, est
    t_peak = times[np.argmax(est)]
    assert 2.5 <= t_peak <= 4.0, t_peak
    # and then comes down with the truth
    assert est[-1] < 0.7 * est.max(), est
    assert errs[-1] < 0.5 * errs[0], errs
