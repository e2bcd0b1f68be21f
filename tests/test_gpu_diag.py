"""GPU parity of the diagnostics: menkf_diagnostics (the sums of the relative
RMSE of Sec. 4), menkf_residual (the conservativity indicator Gamma of
Sec. 6, Gamma = -r / dt on rho v) and menkf_spread (the trace of the
ensemble error covariance X X^T of Sec. 2.1.2) against the oracle on the
same inputs; and the filter's external sanity check on the GPU: the
assimilated fine state's RMSE below the free run's at the 512^2 workload.

Tolerances: the device reductions accumulate in FP64 from the same (FP32 or
FP64) inputs as the oracle and differ only in summation order (1e-12
relative).  The FP32 residual is bounded elementwise by its rounding: the
inputs are exact; r = (x_{k-1} + dt F(x)) - x rounds at most
2^-24 (|x_{k-1}| + |x|) per node, and F(x) carries the rounding of its
nodal fluxes (at most 8 roundings of values up to max |x|, the energy and
pressure being the largest) amplified by the coefficient sum 18/(12 h) of
the fourth-order difference, applied at most twice, so
|Gamma_gpu - Gamma| <= 2^-24 (2 (|x_{k-1}| + |x|) / dt + 2 * 8 max|x| 18/(12 h))."""

import math

import numpy as np
import pytest
import torch

from oracle import diag
from oracle.models import Model
from synthetic import configs, fields
from tests.gpu_helpers import make_ctx, say, to_dev, to_np

pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64


def _dt(cfg):
    return F64 if cfg.precision == "f64" else F32


def _round(x, cfg):
    return np.asarray(x, dtype=np.float64) if cfg.precision == "f64" else \
        np.asarray(x, dtype=np.float32).astype(np.float64)


def _pair(cfg, seed):
    """A reference state and a perturbed 'analysis' of it (positive density)."""
    r = np.random.default_rng(seed)
    if cfg.dim == 2:
        xt = fields.model_ic(cfg)
        xa = xt + 0.01 * r.standard_normal(xt.shape) * np.array([1, 1, 1, 10.0])[:, None, None]
    elif cfg.eq == "euler":
        n = cfg.nx
        xt = np.stack([1 + 0.1 * r.random(n), 0.3 + 0.05 * r.standard_normal(n), 2 + r.random(n)])
        xa = xt + 0.01 * r.standard_normal(xt.shape)
    else:
        xt = fields.truth_ic(cfg)
        xa = fields.model_ic(cfg)
    return _round(xa, cfg), _round(xt, cfg)


DIAG_CASES = [
    ("C1-f64", configs.CONFIGS["C1"]),
    ("tiny1d-f32", configs.tiny_1d(precision="f32")),
    ("euler-f64", configs.euler_inlet(nx=200, ratio=4, n_members=12, n_probes=16)),
    ("tiny2d-f32", configs.tiny_2d(precision="f32")),
    ("ragged2d-f64", configs.ragged_2d(precision="f64")),
    ("ragged2d-f32", configs.ragged_2d(precision="f32")),
    ("C3-fine-f32", configs.CONFIGS["C3"]),
]


@pytest.mark.parametrize("name,cfg", DIAG_CASES, ids=[c[0] for c in DIAG_CASES])
def test_diagnostics_match_oracle_rmse_sums(name, cfg):
    ctx, _, _ = make_ctx(cfg)
    xa, xt = _pair(cfg, 7)
    obs_field = 1 if cfg.eq == "euler" else 0
    say(f"diagnostics {name}: fine {xa.shape}")
    out = to_np(ctx.diagnostics(to_dev(xa, _dt(cfg)), to_dev(xt, _dt(cfg))))
    a, b = diag.rmse_sums(xa, xt, cfg.dim, obs_field)
    assert out[0] == pytest.approx(a, rel=1e-12)
    assert out[1] == pytest.approx(b, rel=1e-12)
    assert out[2] == 0
    if cfg.dim == 2:
        assert math.sqrt(out[0] / out[1]) == pytest.approx(diag.velocity_rmse(xa, xt), rel=1e-12)
    # non-finite entries are counted (every field in 2D, the observed one in 1D)
    bad = xa.copy()
    f_obs = 3 if cfg.dim == 2 else obs_field
    bad[(f_obs,) + (0,) * (bad.ndim - 1)] = np.nan
    bad[(f_obs,) + (1,) * (bad.ndim - 1)] = np.inf
    out = to_np(ctx.diagnostics(to_dev(bad, _dt(cfg)), to_dev(xt, _dt(cfg))))
    assert out[2] == 2


RESID_CASES = [
    ("tiny2d-f64", configs.tiny_2d(precision="f64")),
    ("ragged2d-f64", configs.ragged_2d(precision="f64")),
    ("tiny2d-f32", configs.tiny_2d(precision="f32")),
    ("C3-fine-f32", configs.CONFIGS["C3"]),
]


@pytest.mark.parametrize("name,cfg", RESID_CASES, ids=[c[0] for c in RESID_CASES])
def test_residual_gives_gamma_of_the_oracle(name, cfg):
    """x = a model step of x_{k-1} plus a correction that the model does not
    satisfy (Gamma clearly non-zero), as after an analysis."""
    ctx, _, _ = make_ctx(cfg)
    m = Model(cfg, "fine")
    r = np.random.default_rng(3)
    xp = _round(fields.model_ic(cfg), cfg)
    x = xp + m.dt * m.rhs(xp)
    x = _round(x + 1e-3 * r.standard_normal(x.shape), cfg)
    say(f"residual {name}: {x.shape}")
    rd = ctx.residual(to_dev(x, _dt(cfg)), to_dev(xp, _dt(cfg)))
    g_gpu = -to_np(rd)[2] / m.dt
    g = diag.gamma_rhov(x, xp, m)
    if cfg.precision == "f64":
        np.testing.assert_allclose(g_gpu, g, rtol=0, atol=1e-10 * np.max(np.abs(g)))
    else:
        h = cfg.length / max(cfg.nx, cfg.ny)
        bound = 2.0 ** -24 * (2 * (np.abs(xp[2]) + np.abs(x[2])) / m.dt + 2 * 8 * np.max(np.abs(x)) * 18 / (12 * h))
        assert np.all(np.abs(g_gpu - g) <= bound), np.max(np.abs(g_gpu - g) / bound)
    # the normalised indicator of Sec. 6 from the device residual
    C = np.max(np.abs((x[2] - xp[2]) / m.dt))
    assert np.max(np.abs(g_gpu / C - diag.gamma_normalised(x, xp, m))) < (1e-10 if cfg.precision == "f64" else 1e-3)


SPREAD_CASES = [
    ("C1-f64", configs.CONFIGS["C1"]),
    ("C2-f32-N256", configs.CONFIGS["C2"]),
    ("euler-f64", configs.euler_inlet(nx=200, ratio=4, n_members=12, n_probes=16)),
    ("tiny2d-f32", configs.tiny_2d(precision="f32")),
    ("ragged2d-f64-N24", configs.ragged_2d(precision="f64")),
    ("C3-members-f32", configs.CONFIGS["C3"]),
]


@pytest.mark.parametrize("name,cfg", SPREAD_CASES, ids=[c[0] for c in SPREAD_CASES])
def test_spread_matches_oracle(name, cfg):
    ctx, _, _ = make_ctx(cfg)
    obs_field = 1 if cfg.eq == "euler" else 0
    if cfg.eq == "euler":
        r = np.random.default_rng(5)
        base = fields.inlet_uniform(cfg, "coarse", cfg.n_members)
        mem = _round(base * (1 + 0.01 * r.standard_normal(base.shape)), cfg)
    else:
        mem = _round(fields.random_members_like(cfg), cfg)
    say(f"spread {name}: members {mem.shape}")
    d = to_dev(mem, _dt(cfg))
    for nb in (cfg.n_members, max(2, cfg.n_members - 3), 2):
        out = to_np(ctx.spread(d[:nb]))
        a, b = diag.spread_sums(mem[:nb], cfg.dim, obs_field)
        assert out[0] == pytest.approx(a, rel=1e-12), nb
        assert out[1] == pytest.approx(b, rel=1e-12), nb
        assert out[2] == 0
    bad = mem.copy()
    bad[(1, 1 if cfg.dim == 2 else obs_field) + (0,) * (bad.ndim - 2)] = np.nan
    out = to_np(ctx.spread(to_dev(bad, _dt(cfg))))
    assert out[2] == 1


def test_assimilation_beats_the_free_run_c4():
    """40 plain MEnKF cycles of the 512^2 / 128^2, N = 32 workload (Pi_F and
    three relaxed sweeps) against a free run of the same fine model from the
    same initial state: the second-half mean velocity RMSE (Sec. 4) of the
    analysis is below the free run's, and the ensemble spread shrinks."""
    cfg = configs.CONFIGS["C4"]
    ctx, _, _ = make_ctx(cfg)
    n_cyc = 40
    truth = to_dev(fields.truth_ic(cfg), F32)
    fine = to_dev(fields.model_ic(cfg), F32)
    free = fine.clone()
    mem = to_dev(fields.member_ics(cfg), F32)
    prev = torch.empty_like(fine)
    xs = torch.empty((4, cfg.nyc, cfg.nxc), dtype=F32, device="cuda")
    dc = torch.empty_like(xs)
    out = torch.zeros(3, dtype=F64, device="cuda")
    ra, rf, sp = [], [], [to_np(ctx.spread(mem))]
    say(f"C4 assimilated vs free run, {n_cyc} cycles")
    for c in range(1, n_cyc + 1):
        ctx.forecast(0, truth, cfg.n_obs)
        y = ctx.observe(0, truth)[0] + to_dev(fields.obs_noise(cfg, c), F64)
        ctx.forecast(0, fine, cfg.n_obs, prev=prev)
        ctx.forecast(1, mem, cfg.n_obs)
        ctx.restrict(fine, xs)
        ctx.gain(mem, xs, y, cfg.seed + 5, c)
        ctx.update(mem, dc)
        ctx.prolong_smooth(dc, fine, prev, n_sweeps=3, alpha=0.5)
        ctx.forecast(0, free, cfg.n_obs)
        o = to_np(ctx.diagnostics(fine, truth, out=out))
        ra.append(math.sqrt(o[0] / o[1]))
        o = to_np(ctx.diagnostics(free, truth, out=out))
        rf.append(math.sqrt(o[0] / o[1]))
        sp.append(to_np(ctx.spread(mem)))
    assert ctx.get_status() == 0
    h = n_cyc // 2
    a, f = float(np.mean(ra[h:])), float(np.mean(rf[h:]))
    say(f"C4: assimilated {a:.5f} free run {f:.5f} (ratio {a / f:.4f}); spread "
        f"{math.sqrt(sp[0][0] / sp[0][1]):.4f} -> {math.sqrt(sp[-1][0] / sp[-1][1]):.4f}")
    assert a < f
    assert sp[-1][0] < 0.5 * sp[0][0]
