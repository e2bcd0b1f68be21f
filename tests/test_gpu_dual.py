"""GPU parity of the dual EnKF on the inlet-forced Burgers case (the
MENKF_BURGERS1D_INLET model) against the oracle: the inlet forecast, the
open-grid observation operator and fine correction, the parameter random
walk and update, whole dual cycles (eager and replayed from a captured
graph), and the parameter estimate found at the Sec. 4 size."""

import numpy as np
import pytest
import torch

from oracle import dual, enkf, rng
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
    """Inlet-case states with structure: u0 plus a few smooth random modes."""
    n = cfg.nx if level == "fine" else cfg.nxc
    h = cfg.length / n
    g = np.random.default_rng(seed)
    x = np.arange(n) * h
    out = np.full((nb, 1, n), cfg.u0)
    for k in range(1, 5):
        a = 0.03 / k * g.standard_normal((nb, 1, 1))
        ph = g.uniform(0, 2 * np.pi, (nb, 1, 1))
        out += a * np.sin(2 * np.pi * k * x / cfg.length + ph)
    return _round(out, cfg)


def _thetas(nb, seed):
    g = np.random.default_rng(seed)
    return np.stack([0.2 + 0.05 * g.standard_normal(nb), 0.3 * g.standard_normal(nb)], axis=1)


CASES = [
    (configs.inlet_burgers(nx=200, ratio=4, n_members=12, n_probes=16), 1e-12),
    (configs.inlet_burgers(n_members=100), 1e-12),                                   # Sec. 4 size, F64
    (configs.inlet_burgers(nx=2400, ratio=8, n_members=6, n_probes=16), 1e-12),      # 3 points per thread
    (configs.inlet_burgers(precision="f32", n_members=100), 2e-6),
    # the paper's first-order scheme (forward Euler, Jacobi analysis step)
    (configs.inlet_burgers(nx=200, ratio=4, n_members=12, n_probes=16, time_scheme="first_order"), 1e-12),
    (configs.inlet_burgers(n_members=100, time_scheme="first_order"), 1e-12),
]
CASE_IDS = ["200r4-f64", "800r4-f64", "2400r8-f64", "800r4-f32", "200r4-f64-first-order", "800r4-f64-first-order"]


@pytest.mark.parametrize("cfg,tol", CASES, ids=CASE_IDS)
@pytest.mark.parametrize("nsteps", [1, 37, 300])
def test_inlet_forecast_matches_oracle(cfg, tol, nsteps):
    if cfg.precision == "f32":
        # one half-ulp rounding per Runge-Kutta stage update, of one sign when
        # the increments vary slowly: the error can grow linearly in the steps
        tol = 1e-6 + 3 * nsteps * 2.0 ** -24
    ctx, _, _ = make_ctx(cfg)
    dt = _dt(cfg)
    t0 = 0.37
    t0_d = torch.tensor([t0], dtype=F64, device="cuda")
    for level, n, nb in (("fine", cfg.nx, 1), ("coarse", cfg.nxc, cfg.n_members)):
        say(f"inlet forecast {cfg.name} {cfg.precision} {level} nb={nb} nsteps={nsteps}")
        x0 = _states(cfg, level, nb, 3 + nb)
        th = _thetas(nb, 7 + nb)
        h = cfg.length / n
        want, want_prev = dual.model_forecast(cfg, x0, t0, nsteps, th, level)
        x_d = to_dev(x0 if level == "coarse" else x0[0], dt)
        prev_d = torch.empty_like(x_d)
        lv = 0 if level == "fine" else 1
        ctx.forecast_inlet(lv, x_d, nsteps, to_dev(th, F64), t0_d, prev=prev_d)
        got = to_np(x_d).reshape(want.shape)
        gprev = to_np(prev_d).reshape(want.shape)
        assert rel_l2(got, want) < tol, (level, rel_l2(got, want))
        assert rel_l2(gprev, want_prev) < tol, (level, rel_l2(gprev, want_prev))
        # the boundary rows follow their definitions exactly
        g_end = cfg.u0 * (1.0 + th[:, 0] * np.sin(cfg.omega * ((t0 + (nsteps - 1) * cfg.dt) + cfg.dt) + th[:, 1]))
        np.testing.assert_allclose(got[:, 0, 0], g_end, rtol=1e-15 if cfg.precision == "f64" else 1e-7)
        if cfg.precision == "f64":
            np.testing.assert_allclose(got[:, 0, -1], 2 * got[:, 0, -2] - got[:, 0, -3], rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("cfg,tol", CASES[:2] + CASES[3:4], ids=[CASE_IDS[0], CASE_IDS[1], CASE_IDS[3]])
def test_open_observation_matches_oracle(cfg, tol):
    ctx, _, _ = make_ctx(cfg)
    # probes at both ends and across the grid (the one-sided stencils at both ends)
    g = np.random.default_rng(1)
    ends = np.array([0, 1, 2, cfg.nx - 3, cfg.nx - 2, cfg.nx - 1])
    rest = g.choice(np.arange(3, cfg.nx - 3), cfg.n_probes - len(ends), replace=False)
    idx = np.sort(np.concatenate([ends, rest])).astype(np.int32)
    ctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.zeros(cfg.n_probes, dtype=torch.int32, device="cuda"))
    mem = _states(cfg, "coarse", cfg.n_members, 5)
    say(f"open observation {cfg.name} {cfg.precision}")
    y = to_np(ctx.observe(1, to_dev(mem, _dt(cfg))))
    want = dual.observe_coarse_open(mem, idx, cfg.ratio)
    assert rel_l2(y, want) < 1e-14, rel_l2(y, want)    # FP64 arithmetic on the same state values
    xf = _states(cfg, "fine", 1, 9)[0]
    yf = to_np(ctx.observe(0, to_dev(xf, _dt(cfg))))
    np.testing.assert_array_equal(yf[0], xf[0, idx])


@pytest.mark.parametrize("cfg,tol", [CASES[0], CASES[1], CASES[3]], ids=[CASE_IDS[0], CASE_IDS[1], CASE_IDS[3]])
@pytest.mark.parametrize("n_sweeps", [0, 1, 2, 3])
def test_open_correction_and_sweeps_match_oracle(cfg, tol, n_sweeps):
    ctx, _, _ = make_ctx(cfg)
    dt = _dt(cfg)
    xf = _states(cfg, "fine", 1, 11)
    xprev = _round(xf - 0.001 * np.cos(np.arange(cfg.nx) / 7.0), cfg)
    delta = _round(0.02 * np.random.default_rng(2).standard_normal((1, 1, cfg.nxc)), cfg)[0]
    say(f"open prolong+smooth {cfg.name} {cfg.precision} sweeps={n_sweeps}")
    x_d = to_dev(xf[0], dt)
    ctx.prolong_smooth(to_dev(delta, dt), x_d, to_dev(xprev[0], dt), n_sweeps=n_sweeps, alpha=0.5)
    want = dual.smooth_open(dual.correct_open(xf[0], delta, cfg.ratio), xprev[0], cfg, n_sweeps, 0.5)
    got = to_np(x_d)
    assert rel_l2(got, want) < tol, rel_l2(got, want)
    assert got[0, 0] == xf[0, 0, 0]


def test_param_perturb_matches_oracle_and_reads_the_device_counter():
    cfg = configs.inlet_burgers(n_members=100)
    ctx, _, _ = make_ctx(cfg)
    th = _thetas(cfg.n_members, 3)
    th_d = to_dev(th, F64)
    out = torch.empty_like(th_d)
    seed = 1234567890123
    for c in (1, 7, 2 ** 33 + 5):
        say(f"param perturb cycle {c}")
        ctx.param_perturb(th_d, out, seed, c)
        want = th + dual.param_perturbations(seed, c, cfg.n_members, cfg.theta_walk)
        np.testing.assert_allclose(to_np(out), want, rtol=0, atol=1e-15)
    from paper_2012_10091_amd import MENKF_CYCLE_DEVICE
    ctx.set_cycle(9)
    ctx.param_perturb(th_d, out, seed, MENKF_CYCLE_DEVICE)
    a = to_np(out)
    ctx.param_perturb(th_d, out, seed, MENKF_CYCLE_DEVICE)   # not advanced by the perturbation
    np.testing.assert_array_equal(to_np(out), a)
    np.testing.assert_allclose(a, th + dual.param_perturbations(seed, 9, cfg.n_members, cfg.theta_walk),
                               rtol=0, atol=1e-15)
    # in place
    ctx.param_perturb(th_d, th_d, seed, 9)
    np.testing.assert_array_equal(to_np(th_d), a)


def test_param_update_matches_oracle():
    """Gain on members forecast with theta^f, then the parameter update, vs
    the oracle's analysis and update on the same inputs."""
    cfg = configs.inlet_burgers(n_members=100)
    ctx, idx, _ = make_ctx(cfg)
    mem = _states(cfg, "coarse", cfg.n_members, 21)
    xs = _states(cfg, "coarse", 1, 22)[0]
    thf = _thetas(cfg.n_members, 23)
    y = dual.observe_coarse_open(xs, idx, cfg.ratio) + 0.01       # (N_y,)
    seed, c = 99, 4
    say("param update")
    ctx.gain(to_dev(mem, F64), to_dev(xs, F64), to_dev(y, F64), seed, c)
    thf_d = to_dev(thf, F64)
    tha_d = torch.empty_like(thf_d)
    tm_d = torch.empty(2, dtype=F64, device="cuda")
    ctx.param_update(thf_d, tha_d, tm_d)
    eps = rng.perturbations(seed, c, cfg.n_members, cfg.n_probes, cfg.obs_sigma)
    res = enkf.analysis(mem, xs, y, eps, lambda x: dual.observe_coarse_open(x, idx, cfg.ratio), cfg.obs_sigma)
    want = dual.param_update(thf, res["Z"])
    np.testing.assert_allclose(to_np(tha_d), want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(to_np(tm_d), want.mean(axis=0), rtol=0, atol=1e-12)
    # aliasing theta_a with theta_f gives the same result
    ctx.param_update(thf_d, thf_d, tm_d)
    np.testing.assert_array_equal(to_np(thf_d), to_np(tha_d))


def _spun_up(cfg, steps):
    hf, hc = cfg.length / cfg.nx, cfg.length / cfg.nxc
    theta = fields.inlet_theta_ics(cfg)
    truth, _ = dual.inlet_forecast(fields.inlet_uniform(cfg), 0.0, steps, cfg.dt, np.array(cfg.theta_true), cfg.nu,
                                   hf, cfg.u0, cfg.omega)
    fine, _ = dual.inlet_forecast(fields.inlet_uniform(cfg), 0.0, steps, cfg.dt, theta.mean(0), cfg.nu, hf, cfg.u0,
                                  cfg.omega)
    mem, _ = dual.inlet_forecast(fields.inlet_uniform(cfg, "coarse", cfg.n_members), 0.0, steps, cfg.dt, theta,
                                 cfg.nu, hc, cfg.u0, cfg.omega)
    return truth, dual.DualState(fine=_round(fine, cfg), members=_round(mem, cfg), theta=theta, t=steps * cfg.dt)


class _Dev:
    def __init__(self, ctx, cfg, st):
        dt = _dt(cfg)
        self.fine = to_dev(st.fine, dt)          # (1, n): one state of one field
        self.prev = torch.empty_like(self.fine)
        self.mem = to_dev(st.members, dt)
        self.xs = torch.empty((1, cfg.nxc), dtype=dt, device="cuda")
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
    (configs.inlet_burgers(nx=200, ratio=2, n_members=40, n_probes=20), 1e-10, 6),
    (configs.inlet_burgers(n_members=100), 1e-10, 3),
    (configs.inlet_burgers(precision="f32", n_members=100), None, 3),
    (configs.inlet_burgers(nx=200, ratio=2, n_members=40, n_probes=20, time_scheme="first_order"), 1e-10, 6),
    (configs.inlet_burgers(n_members=100, time_scheme="first_order"), 1e-10, 3),
], ids=["200r2-f64", "800r4-f64", "800r4-f32", "200r2-f64-first-order", "800r4-f64-first-order"])
def test_dual_cycles_match_oracle(cfg, tol, ncyc):
    ctx, idx, _ = make_ctx(cfg)
    truth, st = _spun_up(cfg, 1000)
    dev = _Dev(ctx, cfg, st)
    seed = cfg.seed + 5
    t = st.t
    for c in range(1, ncyc + 1):
        truth, _ = dual.model_forecast(cfg, truth, t, cfg.n_obs, np.array(cfg.theta_true), "fine")
        t += cfg.n_obs * cfg.dt
        y = truth[0, idx] + fields.obs_noise(cfg, c)
        say(f"dual cycle {cfg.name} {cfg.precision} cycle {c}")
        st, tb = dual.dual_cycle(cfg, st, y, idx, n_sweeps=1, seed=seed)
        dev.y.copy_(torch.as_tensor(y, dtype=F64))
        dev.cycle(seed, c, 1)
        assert ctx.get_status() == 0
        if cfg.precision == "f32":   # the forecast bound of the inlet test over the c windows so far
            tol = 1e-5 + 3 * cfg.n_obs * c * 2.0 ** -24
        assert rel_l2(to_np(dev.theta), st.theta) < tol, (c, rel_l2(to_np(dev.theta), st.theta))
        assert rel_l2(to_np(dev.tm), tb) < tol, c
        assert rel_l2(to_np(dev.fine), st.fine[0]) < tol, (c, rel_l2(to_np(dev.fine), st.fine[0]))
        assert rel_l2(to_np(dev.mem), st.members) < tol, (c, rel_l2(to_np(dev.mem), st.members))
        assert to_np(dev.clock)[0] == st.t


@pytest.mark.parametrize("aux", [False, True], ids=["one-stream", "fine-on-second-stream"])
def test_dual_cycle_graph_replays_match_eager_calls(aux):
    from paper_2012_10091_amd import MENKF_CYCLE_DEVICE, Graph
    cfg = configs.inlet_burgers(nx=200, ratio=2, n_members=40, n_probes=20)
    ctx_a, idx, _ = make_ctx(cfg)
    ctx_b, _, _ = make_ctx(cfg)
    truth, st = _spun_up(cfg, 500)
    a, b = _Dev(ctx_a, cfg, st), _Dev(ctx_b, cfg, st)
    seed = 42
    ys = [truth[0, idx] + fields.obs_noise(cfg, c) for c in range(1, 6)]
    s = torch.cuda.Stream()
    s_aux = torch.cuda.Stream() if aux else None
    with torch.cuda.stream(s):
        ctx_b.set_cycle(1, stream=s)
        Graph.begin(s)
        b.cycle(seed, MENKF_CYCLE_DEVICE, 1, stream=s, aux_stream=s_aux)
        g = Graph.end(s)
    torch.cuda.synchronize()
    for c, y in enumerate(ys, start=1):
        say(f"dual graph replay {c} (aux {aux})")
        a.y.copy_(torch.as_tensor(y, dtype=F64))
        a.cycle(seed, c, 1)
        with torch.cuda.stream(s):
            b.y.copy_(torch.as_tensor(y, dtype=F64).to("cuda"))
            g.launch(s)
        torch.cuda.synchronize()
        for name in ("fine", "mem", "theta", "tm", "clock"):
            np.testing.assert_array_equal(to_np(getattr(b, name)), to_np(getattr(a, name)), err_msg=f"{name} {c}")


def test_dual_estimate_converges_at_the_paper_size():
    """Sec. 4 size (800 fine nodes, r = 4, 100 members, 80 sensors every 30
    steps): from the prior (0, 0.3) the amplitude reaches the truth 0.2 and
    the phase moves toward 0, every cycle on the GPU.  Truth and
    observations come from the oracle's model on the CPU."""
    cfg = configs.inlet_burgers(n_members=100)
    ctx, idx, _ = make_ctx(cfg)
    truth, st = _spun_up(cfg, 5000)
    dev = _Dev(ctx, cfg, st)
    hf = cfg.length / cfg.nx
    t = st.t
    hist = []
    for c in range(1, 301):
        truth, _ = dual.model_forecast(cfg, truth, t, cfg.n_obs, np.array(cfg.theta_true), "fine")
        t += cfg.n_obs * cfg.dt
        dev.y.copy_(torch.as_tensor(truth[0, idx] + fields.obs_noise(cfg, c), dtype=F64))
        dev.cycle(cfg.seed + 5, c, 1)
        if c % 50 == 0:
            hist.append(to_np(dev.tm).copy())
            say(f"dual estimate cycle {c}: {hist[-1]}")
    assert ctx.get_status() == 0
    late = np.array(hist[-3:])
    assert np.all(np.abs(late[:, 0] - 0.2) < 0.03), hist
    assert np.all(late[:, 1] < 0.15), hist
    err = rel_l2(to_np(dev.fine), truth[0])
    assert err < 0.02, err
