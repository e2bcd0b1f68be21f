"""What the trained network gains over the method without it, on held-out
seeds of the 512^2 / 128^2, N = 32 workload with the committed weights:
equal RMSE to the plain MEnKF (Pi_F + 3 relaxed sweeps), and the
regularisation that the sweeps provide (conservativity residual Gamma of
Sec. 6 well below that of the bare prolongation) from one fused kernel."""

import os

import pytest

pytestmark = pytest.mark.gpu


def test_trained_network_regularises_like_the_sweeps():
    from paper_2012_10091_amd import learned
    from synthetic import configs
    from tests.gpu_helpers import say
    cfg = configs.CONFIGS["C4"]
    path = learned.weights_for(cfg.name)
    assert os.path.exists(path), path
    net = learned.load(path)
    say("held-out evaluation of the committed 512^2 network")
    r = learned.evaluate(cfg, net, n_cycles=12, seed_offset=7777, log=say)
    assert r["learned_rmse"] <= 1.05 * r["plain_rmse"], r
    assert r["gamma_learned"] < 0.5 * r["gamma_pif"], r
    assert r["net_vs_plain_correction"] < 0.5 * r["pif_vs_plain_correction"], r
