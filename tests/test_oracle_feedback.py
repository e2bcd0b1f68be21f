"""Pins of the oracle's fine-to-coarse feedback (members recentred on the
restricted fine analysis): the mean becomes the injected fine state, the
anomalies are kept, and with r_C = 1 and no sweeps the ensemble mean after
a cycle is the fine analysis itself."""

import numpy as np

from oracle import cycle
from synthetic import configs, fields


def test_recentred_mean_is_the_injected_fine_state_and_anomalies_are_kept():
    cfg = configs.tiny_2d(precision="f64")
    rng = np.random.default_rng(21)
    members = fields.ns_member_ics(cfg) + 0.01 * rng.standard_normal((cfg.n_members, 4, cfg.nyc, cfg.nxc))
    fine = fields.ns_truth_ic(cfg) + 0.01 * rng.standard_normal((4, cfg.ny, cfg.nx))
    out = cycle.recentre(members, fine, cfg)
    # injection written as slicing of every r-th node
    np.testing.assert_allclose(out.mean(axis=0), fine[:, ::cfg.ratio, ::cfg.ratio], atol=1e-14, rtol=0)
    np.testing.assert_allclose(out - out.mean(axis=0), members - members.mean(axis=0), atol=1e-14, rtol=0)


def test_recentring_in_1d_uses_every_ratio_th_node():
    cfg = configs.tiny_1d(precision="f64")
    rng = np.random.default_rng(5)
    members = rng.standard_normal((cfg.n_members, 1, cfg.nxc))
    fine = rng.standard_normal((1, cfg.nx))
    out = cycle.recentre(members, fine, cfg)
    np.testing.assert_allclose(out.mean(axis=0)[0], fine[0, ::cfg.ratio], atol=1e-14, rtol=0)


def test_feedback_with_unit_ratio_makes_the_mean_the_fine_analysis():
    """r_C = 1, n_s = 0: members and fine state live on one grid and the
    recentred ensemble mean equals x^F_a to roundoff, while the members keep
    the analysed anomalies of the same cycle without feedback."""
    cfg = configs.tiny_1d(ratio=1, nx=64, n_probes=8, n_members=10)
    idx, comp = fields.probes_for(cfg)
    rng = np.random.default_rng(4)
    fine = fields.burgers_model_ic(cfg)
    members = fine[None] + 0.05 * rng.standard_normal((cfg.n_members, 1, cfg.nx))
    y = rng.standard_normal(cfg.n_probes) * 0.1
    st = cycle.State(fine=fine, members=members)
    with_fb = cycle.cycle(cfg, st, y, idx, comp, n_sweeps=0, feedback=True)
    without = cycle.cycle(cfg, st, y, idx, comp, n_sweeps=0, feedback=False)
    np.testing.assert_allclose(with_fb.members.mean(axis=0), with_fb.fine, atol=1e-12, rtol=0)
    np.testing.assert_allclose(with_fb.fine, without.fine, atol=0, rtol=0)
    a = with_fb.members - with_fb.members.mean(axis=0)
    b = without.members - without.members.mean(axis=0)
    np.testing.assert_allclose(a, b, atol=1e-12, rtol=0)
