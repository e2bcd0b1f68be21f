"""GPU parity: every menkf_* call against the FP64 oracle on the same seeded
inputs.  Tolerances: FP64 contexts 1e-10 (relative L2); FP32 forecasts 1e-5
after one observation window; BF16 analysis 1e-3 on the analysed states."""

import ctypes
import os

import numpy as np
import pytest
import torch

from oracle import cycle as ocycle
from oracle import enkf, grids, obs, rng, smooth
from oracle.models import Model
from synthetic import configs, fields
from tests.gpu_helpers import make_ctx, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu

F32 = torch.float32
F64 = torch.float64


def _dt(cfg):
    return F64 if cfg.precision == "f64" else F32


def _round(x, cfg):
    """Inputs as the device sees them (FP32 contexts take float32 states)."""
    return np.asarray(x, dtype=np.float64) if cfg.precision == "f64" else \
        np.asarray(x, dtype=np.float32).astype(np.float64)


# ------------------------------------------------------------------ primitives
def test_philox_known_answers_on_device(golden_dir):
    import paper_2012_10091_amd as m
    lib = m.load_library()
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    inp = torch.tensor([r[:6] for r in rows], dtype=torch.int64).to(torch.int32).cuda()
    out = torch.zeros((len(rows), 4), dtype=torch.int32, device="cuda")
    say("philox KAT on device, n =", len(rows))
    assert lib.menkf_test_philox(ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()), len(rows),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0
    got = out.cpu().numpy().astype(np.uint32)
    assert [[int(v) for v in r] for r in got] == [r[6:] for r in rows]


def test_mfma_lane_layouts():
    import paper_2012_10091_amd as m
    lib = m.load_library()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = torch.Generator().manual_seed(0)
    a = torch.randint(-4, 5, (32, 16), generator=g).to(torch.bfloat16)
    b = torch.randint(-4, 5, (16, 32), generator=g).to(torch.bfloat16)
    out = torch.zeros((32, 32), dtype=torch.float32, device="cuda")
    ad, bd = a.cuda().contiguous(), b.cuda().contiguous()
    say("mfma layout bf16 32x32x16")
    assert lib.menkf_test_mfma(0, ctypes.c_void_p(ad.data_ptr()), ctypes.c_void_p(bd.data_ptr()),
                               ctypes.c_void_p(out.data_ptr()), s) == 0
    np.testing.assert_array_equal(out.cpu().numpy(), (a.float() @ b.float()).numpy())
    a64 = torch.randn((16, 4), generator=g, dtype=torch.float64)
    b64 = torch.randn((4, 16), generator=g, dtype=torch.float64)
    o64 = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    ad, bd = a64.cuda(), b64.cuda()
    say("mfma layout f64 16x16x4")
    assert lib.menkf_test_mfma(1, ctypes.c_void_p(ad.data_ptr()), ctypes.c_void_p(bd.data_ptr()),
                               ctypes.c_void_p(o64.data_ptr()), s) == 0
    np.testing.assert_allclose(o64.cpu().numpy(), (a64 @ b64).numpy(), rtol=1e-14, atol=1e-14)
    a16 = torch.randint(-4, 5, (16, 32), generator=g).to(torch.bfloat16)
    b16 = torch.randint(-4, 5, (32, 16), generator=g).to(torch.bfloat16)
    o16 = torch.zeros((16, 16), dtype=torch.float32, device="cuda")
    ad, bd = a16.cuda().contiguous(), b16.cuda().contiguous()
    say("mfma layout bf16 16x16x32")
    assert lib.menkf_test_mfma(2, ctypes.c_void_p(ad.data_ptr()), ctypes.c_void_p(bd.data_ptr()),
                               ctypes.c_void_p(o16.data_ptr()), s) == 0
    np.testing.assert_array_equal(o16.cpu().numpy(), (a16.float() @ b16.float()).numpy())


# ------------------------------------------------------------------ forecasts
FORECAST_CASES = [
    ("C1-f64", configs.CONFIGS["C1"], 10, 1e-12),
    ("tiny1d-f32", configs.tiny_1d(precision="f32"), 7, 1e-5),
    ("tiny2d-f64", configs.tiny_2d(precision="f64"), 3, 1e-11),
    ("ragged2d-f64", configs.ragged_2d(precision="f64"), 2, 1e-11),
    ("tiny2d-f32", configs.tiny_2d(precision="f32"), 3, 1e-5),
    ("ragged2d-f32", configs.ragged_2d(precision="f32"), 3, 1e-5),
]


@pytest.mark.parametrize("name,cfg,nsteps,tol", FORECAST_CASES, ids=[c[0] for c in FORECAST_CASES])
def test_forecast_fine_and_members(name, cfg, nsteps, tol):
    ctx, _, _ = make_ctx(cfg)
    dt = _dt(cfg)
    xf = _round(fields.truth_ic(cfg), cfg)
    mem = _round(fields.member_ics(cfg), cfg)
    say(f"forecast {name}: fine {xf.shape} coarse {mem.shape} steps {nsteps}")
    xf_d, mem_d = to_dev(xf, dt), to_dev(mem, dt)
    prev_d = torch.empty_like(xf_d)
    ctx.forecast(0, xf_d, nsteps, prev=prev_d)
    ctx.forecast(1, mem_d, nsteps)
    o_f, o_prev = Model(cfg, "fine").forecast(xf, nsteps)
    o_m, _ = Model(cfg, "coarse").forecast(mem, nsteps)
    assert rel_l2(to_np(xf_d), o_f) < tol
    assert rel_l2(to_np(prev_d), o_prev) < tol
    assert rel_l2(to_np(mem_d), o_m) < tol
    for i in (0, cfg.n_members - 1):
        assert rel_l2(to_np(mem_d)[i], o_m[i]) < tol


def test_forecast_c2_shapes_f32():
    cfg = configs.CONFIGS["C2"]
    ctx, _, _ = make_ctx(cfg)
    rs = np.random.default_rng(5)
    mem = _round(fields.member_ics(cfg), cfg)
    xf = _round(fields.truth_ic(cfg), cfg)
    say("forecast C2 shapes: coarse", mem.shape, "fine", xf.shape)
    mem_d, xf_d = to_dev(mem, F32), to_dev(xf, F32)
    prev_d = torch.empty_like(xf_d)
    ctx.forecast(1, mem_d, cfg.n_obs)
    ctx.forecast(0, xf_d, cfg.n_obs, prev=prev_d)
    o_m, _ = Model(cfg, "coarse").forecast(mem, cfg.n_obs)
    o_f, o_p = Model(cfg, "fine").forecast(xf, cfg.n_obs)
    assert rel_l2(to_np(mem_d), o_m) < 1e-5
    assert rel_l2(to_np(xf_d), o_f) < 1e-5
    assert rel_l2(to_np(prev_d), o_p) < 1e-5
    del rs


def test_forecast_c3_shapes_f32():
    """The 2D workload's shapes: the 1024^2 fine state and 8 members on the
    256^2 coarse grid, one whole observation window (20 RK4 steps), FP32
    against the FP64 oracle from the same FP32 inputs."""
    cfg = configs.CONFIGS["C3"].with_(n_members=8)
    ctx, _, _ = make_ctx(cfg)
    xf = _round(fields.truth_ic(cfg), cfg)
    mem = _round(fields.member_ics(cfg), cfg)
    say("forecast C3 shapes: fine", xf.shape, "coarse", mem.shape, "steps", cfg.n_obs)
    xf_d, mem_d = to_dev(xf, F32), to_dev(mem, F32)
    prev_d = torch.empty_like(xf_d)
    ctx.forecast(0, xf_d, cfg.n_obs, prev=prev_d)
    ctx.forecast(1, mem_d, cfg.n_obs)
    o_f, o_p = Model(cfg, "fine").forecast(xf, cfg.n_obs)
    o_m, _ = Model(cfg, "coarse").forecast(mem, cfg.n_obs)
    e = (rel_l2(to_np(xf_d), o_f), rel_l2(to_np(prev_d), o_p), rel_l2(to_np(mem_d), o_m))
    say(f"  rel-L2 fine {e[0]:.2e} prev {e[1]:.2e} members {e[2]:.2e}")
    assert max(e) < 1e-5
    g = to_np(mem_d)
    for i in range(cfg.n_members):
        assert rel_l2(g[i], o_m[i]) < 1e-5, i
    # the row-march schedules of the coarse level (one and two RK stages
    # per launch): the same forecast, bitwise
    for tile in ((0, 16), (0, 32)):
        ctx.set_schedule(1, tile, 0)
        mem2 = to_dev(mem, F32)
        say(f"  coarse level again with the row-march schedule {tile}")
        ctx.forecast(1, mem2, cfg.n_obs)
        np.testing.assert_array_equal(to_np(mem2), g)


def test_forecast_conserves_totals_f64():
    cfg = configs.ragged_2d(precision="f64")
    ctx, _, _ = make_ctx(cfg)
    mem = fields.member_ics(cfg)
    d = to_dev(mem, F64)
    say("conservation ragged2d f64, 20 steps")
    ctx.forecast(1, d, 20)
    out = to_np(d)
    np.testing.assert_allclose(out.sum(axis=(-1, -2)), mem.sum(axis=(-1, -2)), rtol=0,
                               atol=1e-12 * np.abs(mem).sum(axis=(-1, -2)).max())


# ------------------------------------------------------------------ projections, observation
@pytest.mark.parametrize("cfg", [configs.CONFIGS["C1"], configs.ragged_2d(precision="f32"),
                                 configs.tiny_2d(precision="f64")], ids=["C1", "ragged-f32", "tiny-f64"])
def test_restrict_is_exact_and_observe_matches(cfg):
    ctx, idx, comp = make_ctx(cfg)
    dt = _dt(cfg)
    xf = _round(fields.truth_ic(cfg), cfg)
    xf_d = to_dev(xf, dt)
    xc_d = torch.empty((cfg.nfields,) + tuple(cfg.coarse_shape[1:]), dtype=dt, device="cuda")
    say("restrict/observe", cfg.name)
    ctx.restrict(xf_d, xc_d)
    np.testing.assert_array_equal(to_np(xc_d), grids.restrict(xf, cfg.ratio, cfg.dim))
    yf = to_np(ctx.observe(0, xf_d))[0]
    np.testing.assert_allclose(yf, obs.observe_fine(xf, idx, comp, cfg.dim), rtol=1e-12, atol=0)
    mem = _round(fields.member_ics(cfg), cfg)
    yc = to_np(ctx.observe(1, to_dev(mem, dt)))
    np.testing.assert_allclose(yc, obs.observe_coarse(mem, idx, comp, cfg.dim, cfg.ratio, cfg.nx),
                               rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("cfg,tol", [(configs.CONFIGS["C1"], 1e-12), (configs.tiny_2d(precision="f64"), 1e-12),
                                     (configs.ragged_2d(precision="f32"), 1e-5)],
                         ids=["C1", "tiny2d-f64", "ragged2d-f32"])
@pytest.mark.parametrize("n_sweeps", [0, 1, 2, 3])
def test_prolong_smooth_plain(cfg, tol, n_sweeps):
    ctx, _, _ = make_ctx(cfg)
    dt = _dt(cfg)
    r = np.random.default_rng(3)
    xprev = _round(fields.truth_ic(cfg), cfg)
    m = Model(cfg, "fine")
    xf = _round(m.step(xprev), cfg)
    dc = _round(0.01 * r.standard_normal((cfg.nfields,) + tuple(cfg.coarse_shape[1:])), cfg)
    say("prolong_smooth", cfg.name, "sweeps", n_sweeps)
    xf_d, xp_d, dc_d = to_dev(xf, dt), to_dev(xprev, dt), to_dev(dc, dt)
    ctx.prolong_smooth(dc_d, xf_d, xp_d, n_sweeps=n_sweeps, alpha=0.5)
    x = xf + grids.prolong(dc, cfg.ratio, cfg.dim)
    x = smooth.smooth(x, xprev, m, n_sweeps, 0.5)
    assert rel_l2(to_np(xf_d) - xf, x - xf) < (tol * 1e3 if cfg.precision != "f64" else 1e-10)
    assert rel_l2(to_np(xf_d), x) < tol


# ------------------------------------------------------------------ analysis
def _analysis_inputs(cfg, seed_offset=11):
    r = np.random.default_rng(cfg.seed + seed_offset)
    mem = _round(fields.random_members_like(cfg), cfg)
    xstar = _round(mem.mean(axis=0) + 0.01 * r.standard_normal(mem.shape[1:]), cfg)
    idx, comp = fields.probes_for(cfg)
    truth_c = mem.mean(axis=0) + 0.02 * r.standard_normal(mem.shape[1:])
    y = obs.observe_coarse(truth_c, idx, comp, cfg.dim, cfg.ratio, cfg.nx) + cfg.obs_sigma * r.standard_normal(cfg.n_probes)
    return mem, xstar, y


ANALYSIS_CASES = [
    # name, config, Z tol, increment tol, analysed-state tol
    ("C1-f64", configs.CONFIGS["C1"], 1e-10, 1e-10, 1e-10),
    ("tiny2d-f64", configs.tiny_2d(precision="f64"), 1e-10, 1e-10, 1e-10),
    ("ragged2d-f64-N24", configs.ragged_2d(precision="f64"), 1e-10, 1e-10, 1e-10),
    ("tiny1d-f64-N200", configs.tiny_1d(precision="f64", n_members=200, n_probes=32), 1e-10, 1e-10, 1e-10),
    ("tiny1d-f32", configs.tiny_1d(precision="f32", n_members=12, n_probes=8), 1e-9, 1e-4, 1e-5),
    ("ragged2d-f32", configs.ragged_2d(precision="f32"), 1e-9, 1e-4, 1e-5),
    ("tiny2d-f32-N40", configs.tiny_2d(precision="f32", n_members=40, n_probes=70), 1e-9, 1e-4, 1e-5),
    ("C2-f32-N256", configs.CONFIGS["C2"], 1e-9, 1e-4, 1e-5),
    ("ragged2d-f32-plainbf16", configs.ragged_2d(precision="f32").with_(name="plain"), 1e-9, 2e-2, 1e-3),
    # degenerate ends: two members (rank-one anomalies), a single probe
    ("tiny1d-f64-N2-Ny1", configs.tiny_1d(precision="f64", n_members=2, n_probes=1), 1e-10, 1e-10, 1e-10),
    ("tiny2d-f32-N2-Ny3", configs.tiny_2d(precision="f32", n_members=2, n_probes=3), 1e-9, 1e-4, 1e-5),
]


@pytest.mark.parametrize("name,cfg,ztol,inctol,xtol", ANALYSIS_CASES, ids=[c[0] for c in ANALYSIS_CASES])
@pytest.mark.parametrize("rng_on_device", [False, True], ids=["eps-given", "eps-philox"])
def test_gain_and_update(name, cfg, ztol, inctol, xtol, rng_on_device):
    if name.endswith("plainbf16"):
        cfg = _with_terms(cfg, 1)
    ctx, idx, comp = make_ctx(cfg)
    dt = _dt(cfg)
    mem, xstar, y = _analysis_inputs(cfg)
    seed, cyc = 4242, 7
    eps = rng.perturbations(seed, cyc, cfg.n_members, cfg.n_probes, cfg.obs_sigma)
    mem_d, xs_d = to_dev(mem, dt), to_dev(xstar, dt)
    y_d = to_dev(y, F64)
    eps_d = None if rng_on_device else to_dev(eps, F64)
    say(f"gain/update {name} members {mem.shape} probes {cfg.n_probes} device-rng {rng_on_device}")
    ctx.gain(mem_d, xs_d, y_d, seed, cyc, eps=eps_d)
    z = to_np(ctx.get_gain())
    dc_d = torch.empty_like(xs_d)
    ctx.update(mem_d, dc_d)
    assert ctx.get_status() == 0
    H = ocycle.make_H(cfg, idx, comp)
    res = enkf.analysis(mem, xstar, y, eps, H, cfg.obs_sigma)
    zo = res["Z"].T                      # (N+1, N): row j = column j of Z
    assert rel_l2(z, zo) < ztol, rel_l2(z, zo)
    xa = to_np(mem_d)
    assert rel_l2(xa - mem, res["members"] - mem) < inctol, rel_l2(xa - mem, res["members"] - mem)
    assert rel_l2(xa, res["members"]) < xtol
    assert rel_l2(to_np(dc_d), res["delta"]) < max(1e-6 if cfg.precision == "f32" else 1e-10, ztol)


def _with_terms(cfg, terms):
    import dataclasses

    @dataclasses.dataclass(frozen=True)
    class C(type(cfg)):
        anomaly_terms: int = terms
    return C(**dataclasses.asdict(cfg))


def test_gain_and_update_c3_scale():
    """Full C3 analysis shape: 64 members of 4 x 256^2, 4096 probes."""
    cfg = configs.CONFIGS["C3"]
    ctx, idx, comp = make_ctx(cfg)
    mem, xstar, y = _analysis_inputs(cfg)
    seed, cyc = 99, 3
    say("gain/update C3 scale", mem.shape)
    mem_d, xs_d = to_dev(mem, F32), to_dev(xstar, F32)
    ctx.gain(mem_d, xs_d, to_dev(y, F64), seed, cyc)
    z = to_np(ctx.get_gain())
    dc_d = torch.empty_like(xs_d)
    ctx.update(mem_d, dc_d)
    assert ctx.get_status() == 0
    eps = rng.perturbations(seed, cyc, cfg.n_members, cfg.n_probes, cfg.obs_sigma)
    res = enkf.analysis(mem, xstar, y, eps, ocycle.make_H(cfg, idx, comp), cfg.obs_sigma)
    assert rel_l2(z, res["Z"].T) < 1e-8
    xa = to_np(mem_d)
    assert rel_l2(xa - mem, res["members"] - mem) < 1e-4
    assert rel_l2(xa, res["members"]) < 1e-5
    assert rel_l2(to_np(dc_d), res["delta"]) < 1e-5


def test_nonfinite_member_sets_status_and_freezes_outputs():
    cfg = configs.tiny_2d(precision="f32")
    ctx, idx, comp = make_ctx(cfg)
    mem, xstar, y = _analysis_inputs(cfg)
    mem[3, 0, 0, 0] = np.nan
    mem_d, xs_d = to_dev(mem, F32), to_dev(xstar, F32)
    say("status word on a NaN member")
    ctx.gain(mem_d, xs_d, to_dev(y, F64), 1, 1)
    before = to_np(mem_d).copy()
    dc_d = torch.full_like(xs_d, 7.0)
    ctx.update(mem_d, dc_d)
    xf = to_dev(_round(fields.truth_ic(cfg), cfg), F32)
    xf0 = to_np(xf).copy()
    ctx.prolong_smooth(dc_d, xf, xf.clone(), n_sweeps=1)
    info = ctx.get_status(clear=True)
    assert info > 0
    np.testing.assert_array_equal(to_np(mem_d), before)
    assert np.all(to_np(dc_d) == 7.0)
    np.testing.assert_array_equal(to_np(xf), xf0)
    assert ctx.get_status() == 0


# ------------------------------------------------------------------ whole cycles
def _gpu_cycle(ctx, cfg, st, y, c, n_sweeps, seed):
    dt = _dt(cfg)
    xprev = torch.empty_like(st["fine"])
    ctx.forecast(0, st["fine"], cfg.n_obs, prev=xprev)
    ctx.forecast(1, st["members"], cfg.n_obs)
    xs = torch.empty((cfg.nfields,) + tuple(cfg.coarse_shape[1:]), dtype=dt, device="cuda")
    ctx.restrict(st["fine"], xs)
    ctx.gain(st["members"], xs, y, seed, c)
    dc = torch.empty_like(xs)
    ctx.update(st["members"], dc)
    ctx.prolong_smooth(dc, st["fine"], xprev, n_sweeps=n_sweeps, alpha=0.5)


def test_c1_cycles_fp64_match_oracle():
    """The whole C1 workload (20 cycles, all FP64, device Philox perturbations)."""
    cfg = configs.CONFIGS["C1"]
    ctx, idx, comp = make_ctx(cfg)
    truth = fields.truth_ic(cfg)
    fine = fields.model_ic(cfg)
    mem = fields.member_ics(cfg)
    st_o = ocycle.State(fine=fine, members=mem)
    st_g = {"fine": to_dev(fine, F64), "members": to_dev(mem, F64)}
    mt = Model(cfg, "fine")
    seed = cfg.seed + 5
    for c in range(1, cfg.n_cycles + 1):
        truth, _ = mt.forecast(truth, cfg.n_obs)
        y = ocycle.observe_truth(cfg, truth, idx, comp) + fields.obs_noise(cfg, c)
        say(f"C1 cycle {c}")
        st_o = ocycle.cycle(cfg, st_o, y, idx, comp, n_sweeps=1, seed=seed)
        _gpu_cycle(ctx, cfg, st_g, to_dev(y, F64), c, 1, seed)
        assert rel_l2(to_np(st_g["fine"]), st_o.fine) < 1e-10, c
        assert rel_l2(to_np(st_g["members"]), st_o.members) < 1e-10, c
    assert ctx.get_status() == 0


def test_c2_three_cycles_f32():
    """Three whole cycles of the 1D workload at scale (16384 / 4096, N = 256,
    1024 probes every 5 steps; FP32 states, BF16x3 member update, FP64
    Cholesky of the 1024 x 1024 innovation covariance) against the oracle
    run independently from the same initial states, observations and
    perturbations (device Philox on the GPU, its NumPy twin in the oracle).
    The analysed fine state and members stay within the analysis tolerance
    after every cycle, the differences of earlier cycles carried along."""
    cfg = configs.CONFIGS["C2"]
    ctx, idx, comp = make_ctx(cfg)
    truth = fields.truth_ic(cfg)
    fine = _round(fields.model_ic(cfg), cfg)
    mem = _round(fields.member_ics(cfg), cfg)
    st_o = ocycle.State(fine=fine, members=mem)
    st_g = {"fine": to_dev(fine, F32), "members": to_dev(mem, F32)}
    mt = Model(cfg, "fine")
    seed = cfg.seed + 5
    for c in range(1, 4):
        truth, _ = mt.forecast(truth, cfg.n_obs)
        y = ocycle.observe_truth(cfg, truth, idx, comp) + fields.obs_noise(cfg, c)
        say(f"C2 cycle {c}")
        st_o = ocycle.cycle(cfg, st_o, y, idx, comp, n_sweeps=1, seed=seed)
        _gpu_cycle(ctx, cfg, st_g, to_dev(y, F64), c, 1, seed)
        e_f = rel_l2(to_np(st_g["fine"]), st_o.fine)
        e_m = rel_l2(to_np(st_g["members"]), st_o.members)
        say(f"  rel-L2 fine {e_f:.2e} members {e_m:.2e}")
        assert e_f < 1e-3 and e_m < 1e-3, (c, e_f, e_m)
    assert ctx.get_status() == 0


def test_c2_member_window_from_gpu_state_f32():
    """One C2 member window from identical inputs (the FP32 tolerance of a
    forecast is stated for one window from the same states)."""
    cfg = configs.CONFIGS["C2"]
    ctx, _, _ = make_ctx(cfg)
    mem = _round(fields.random_members_like(cfg), cfg)
    d = to_dev(mem, F32)
    say("C2 member window", mem.shape)
    ctx.forecast(1, d, cfg.n_obs)
    o_m, _ = Model(cfg, "coarse").forecast(mem, cfg.n_obs)
    assert rel_l2(to_np(d), o_m) < 1e-5


def test_graph_replay_matches_eager():
    from paper_2012_10091_amd import Graph
    cfg = configs.tiny_2d(precision="f32")
    ctx, idx, comp = make_ctx(cfg)
    fine = to_dev(fields.model_ic(cfg), F32)
    mem = to_dev(fields.member_ics(cfg), F32)
    y = to_dev(np.zeros(cfg.n_probes) + 0.1, F64)
    st_e = {"fine": fine.clone(), "members": mem.clone()}
    st_g = {"fine": fine.clone(), "members": mem.clone()}
    stream = torch.cuda.Stream()
    say("graph capture of one tiny cycle")
    with torch.cuda.stream(stream):
        Graph.begin(stream)
        _gpu_cycle(ctx, cfg, st_g, y, 1, 1, 5)
        g = Graph.end(stream)
    torch.cuda.synchronize()
    for rep in range(3):
        _gpu_cycle(ctx, cfg, st_e, y, 1, 1, 5)
        torch.cuda.synchronize()
        g.launch(stream)
        stream.synchronize()
        np.testing.assert_array_equal(to_np(st_g["fine"]), to_np(st_e["fine"]))
        np.testing.assert_array_equal(to_np(st_g["members"]), to_np(st_e["members"]))
