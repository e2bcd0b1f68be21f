"""GPU parity of the ensemble-space gain (MENKF_GAIN_ENSEMBLE_SPACE): with
R = s^2 I, Y^T (Y Y^T + s^2 I)^-1 = (s^2 I + Y^T Y)^-1 Y^T exactly, so its Z
must match the oracle's exact-R analysis (an N_y x N_y Cholesky in FP64)
to roundoff times the conditioning, on the same inputs as the exact-R
parity tests, and the whole 1D FP64 workload must follow the oracle."""

import dataclasses

import numpy as np
import pytest
import torch

from oracle import cycle as ocycle
from oracle import enkf, rng
from oracle.models import Model
from synthetic import configs, fields
from tests.gpu_helpers import make_ctx, rel_l2, say, to_dev, to_np
from tests.test_gpu_parity import _analysis_inputs, _dt

pytestmark = pytest.mark.gpu

F64 = torch.float64


def _ens(cfg):
    @dataclasses.dataclass(frozen=True)
    class C(type(cfg)):
        gain_mode: int = 2
    return C(**dataclasses.asdict(cfg))


CASES = [
    # name, config, Z tol, analysed-state tol
    ("C1-f64", configs.CONFIGS["C1"], 1e-10, 1e-10),
    ("tiny2d-f64", configs.tiny_2d(precision="f64"), 1e-10, 1e-10),
    ("ragged2d-f64-N24", configs.ragged_2d(precision="f64"), 1e-10, 1e-10),
    ("tiny1d-f64-N200", configs.tiny_1d(precision="f64", n_members=200, n_probes=32), 1e-10, 1e-10),
    ("ragged2d-f32", configs.ragged_2d(precision="f32"), 1e-9, 1e-5),
    ("C2-f32-N256", configs.CONFIGS["C2"], 1e-9, 1e-5),
    ("C3-f32", configs.CONFIGS["C3"], 1e-8, 1e-5),
]


@pytest.mark.parametrize("name,cfg,ztol,xtol", CASES, ids=[c[0] for c in CASES])
def test_ensemble_space_gain_matches_exact_r_oracle(name, cfg, ztol, xtol):
    ecfg = _ens(cfg)
    ctx, idx, comp = make_ctx(ecfg)
    dt = _dt(cfg)
    mem, xstar, y = _analysis_inputs(cfg)
    seed, cyc = 4242, 7
    say(f"ensemble-space gain {name}: members {mem.shape}, probes {cfg.n_probes}")
    mem_d, xs_d = to_dev(mem, dt), to_dev(xstar, dt)
    ctx.gain(mem_d, xs_d, to_dev(y, F64), seed, cyc)
    z = to_np(ctx.get_gain())
    dc_d = torch.empty_like(xs_d)
    ctx.update(mem_d, dc_d)
    assert ctx.get_status() == 0
    eps = rng.perturbations(seed, cyc, cfg.n_members, cfg.n_probes, cfg.obs_sigma)
    res = enkf.analysis(mem, xstar, y, eps, ocycle.make_H(cfg, idx, comp), cfg.obs_sigma)
    assert rel_l2(z, res["Z"].T) < ztol, rel_l2(z, res["Z"].T)
    assert rel_l2(to_np(mem_d), res["members"]) < xtol
    assert rel_l2(to_np(dc_d), res["delta"]) < max(1e-6 if cfg.precision == "f32" else 1e-10, ztol)


def test_ensemble_space_and_exact_r_agree_on_device():
    cfg = configs.ragged_2d(precision="f64")
    mem, xstar, y = _analysis_inputs(cfg)
    zs = []
    for c in (cfg, _ens(cfg)):
        ctx, _, _ = make_ctx(c)
        ctx.gain(to_dev(mem, F64), to_dev(xstar, F64), to_dev(y, F64), 11, 3)
        zs.append(to_np(ctx.get_gain()))
        assert ctx.get_status() == 0
    assert rel_l2(zs[1], zs[0]) < 1e-11


def test_c1_cycles_fp64_ensemble_space_match_oracle():
    """The whole 1D FP64 workload with the ensemble-space gain on the device
    against the oracle's exact-R cycles (20 cycles, device perturbations)."""
    cfg = configs.CONFIGS["C1"]
    ecfg = _ens(cfg)
    ctx, idx, comp = make_ctx(ecfg)
    truth = fields.truth_ic(cfg)
    st_o = ocycle.State(fine=fields.model_ic(cfg), members=fields.member_ics(cfg))
    fine_d, mem_d = to_dev(st_o.fine, F64), to_dev(st_o.members, F64)
    prev_d = torch.empty_like(fine_d)
    xs_d = torch.empty((cfg.nfields,) + tuple(cfg.coarse_shape[1:]), dtype=F64, device="cuda")
    dc_d = torch.empty_like(xs_d)
    mt = Model(cfg, "fine")
    seed = cfg.seed + 5
    for c in range(1, cfg.n_cycles + 1):
        truth, _ = mt.forecast(truth, cfg.n_obs)
        y = ocycle.observe_truth(cfg, truth, idx, comp) + fields.obs_noise(cfg, c)
        say(f"C1 ensemble-space cycle {c}")
        st_o = ocycle.cycle(cfg, st_o, y, idx, comp, n_sweeps=1, seed=seed)
        ctx.cycle(fine_d, prev_d, mem_d, xs_d, dc_d, to_dev(y, F64), seed, c, cfg.n_obs, n_sweeps=1, alpha=0.5)
        assert rel_l2(to_np(fine_d), st_o.fine) < 1e-10, c
        assert rel_l2(to_np(mem_d), st_o.members) < 1e-10, c
    assert ctx.get_status() == 0
