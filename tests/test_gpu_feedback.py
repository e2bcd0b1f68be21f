"""GPU parity of the fine-to-coarse feedback (members recentred on the
injected fine analysis) against the oracle, alone and inside whole cycles
of the 1D FP64 workload."""

import numpy as np
import pytest
import torch

from oracle import cycle as ocycle
from oracle.models import Model
from synthetic import configs, fields
from tests.gpu_helpers import make_ctx, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg,tol", [(configs.tiny_2d(precision="f64"), 1e-13),
                                     (configs.ragged_2d(precision="f32"), 1e-6),
                                     (configs.CONFIGS["C3"], 1e-6)],
                         ids=["tiny2d-f64", "ragged2d-f32", "C3-f32"])
def test_recentre_matches_oracle(cfg, tol):
    ctx, _, _ = make_ctx(cfg)
    dt = torch.float64 if cfg.precision == "f64" else torch.float32
    rs = np.random.default_rng(17)
    mem = np.asarray(fields.member_ics(cfg), dtype=np.float64)
    fine = np.asarray(fields.truth_ic(cfg), dtype=np.float64) + 0.01 * rs.standard_normal((4, cfg.ny, cfg.nx))
    if cfg.precision != "f64":
        mem = mem.astype(np.float32).astype(np.float64)
        fine = fine.astype(np.float32).astype(np.float64)
    say(f"recentre {cfg.name} {mem.shape}")
    mem_d, fine_d = to_dev(mem, dt), to_dev(fine, dt)
    ctx.recentre(mem_d, fine_d)
    out = ocycle.recentre(mem, fine, cfg)
    assert rel_l2(to_np(mem_d), out) < tol
    got = to_np(mem_d)
    # the mean is the injected fine state to the precision of the states
    assert rel_l2(got.mean(axis=0), fine[:, ::cfg.ratio, ::cfg.ratio]) < (1e-13 if cfg.precision == "f64" else 1e-6)


def test_c1_cycles_fp64_with_feedback_match_oracle():
    cfg = configs.CONFIGS["C1"]
    ctx, idx, comp = make_ctx(cfg)
    truth = fields.truth_ic(cfg)
    st_o = ocycle.State(fine=fields.model_ic(cfg), members=fields.member_ics(cfg))
    F64 = torch.float64
    fine_d, mem_d = to_dev(st_o.fine, F64), to_dev(st_o.members, F64)
    prev_d = torch.empty_like(fine_d)
    xs_d = torch.empty((cfg.nfields,) + tuple(cfg.coarse_shape[1:]), dtype=F64, device="cuda")
    dc_d = torch.empty_like(xs_d)
    mt = Model(cfg, "fine")
    seed = cfg.seed + 5
    for c in range(1, cfg.n_cycles + 1):
        truth, _ = mt.forecast(truth, cfg.n_obs)
        y = ocycle.observe_truth(cfg, truth, idx, comp) + fields.obs_noise(cfg, c)
        say(f"C1 feedback cycle {c}")
        st_o = ocycle.cycle(cfg, st_o, y, idx, comp, n_sweeps=1, seed=seed, feedback=True)
        ctx.cycle(fine_d, prev_d, mem_d, xs_d, dc_d, to_dev(y, F64), seed, c, cfg.n_obs, n_sweeps=1, alpha=0.5,
                  feedback=True)
        assert rel_l2(to_np(fine_d), st_o.fine) < 1e-10, c
        assert rel_l2(to_np(mem_d), st_o.members) < 1e-10, c
    assert ctx.get_status() == 0
