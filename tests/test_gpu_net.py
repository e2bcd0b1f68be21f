"""GPU parity of the learned prolongation (inference kernel, fallback guard,
training forward/backward and Adam) against the FP64 oracle network."""

import dataclasses

import numpy as np
import pytest
import torch

from oracle import grids, net as onet
from synthetic import configs, fields
from tests.gpu_helpers import bf16_round, make_ctx, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu
F32 = torch.float32


def _bf16(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _params(cfg, seed=5, zero_last=False, last_gain=1.0):
    p = onet.init_params(cfg, seed=seed, zero_last=zero_last)
    p.w3 = p.w3 * last_gain
    p.b1 = 0.05 * np.random.default_rng(seed).standard_normal(32)
    p.b2 = 0.05 * np.random.default_rng(seed + 1).standard_normal(32)
    p.b3 = 0.0 * p.b3 if zero_last else 0.01 * np.random.default_rng(seed + 2).standard_normal(4)
    for name in ("w1", "b1", "w2", "b2", "w3", "b3"):
        setattr(p, name, _bf16(getattr(p, name)))
    return p


def _gpu_net(p, guard=10.0):
    import paper_2012_10091_amd as m
    flat = m.pack_params([p.w1, p.b1, p.w2, p.b2, p.w3, p.b3])
    return m.Net(flat, p.in_scale, p.in_offset, p.out_scale, guard=guard)


def _inputs(cfg, amp=0.01, seed=9):
    r = np.random.default_rng(seed)
    dc = (amp * r.standard_normal((4, cfg.nyc, cfg.nxc))).astype(np.float32).astype(np.float64)
    xf = fields.truth_ic(cfg).astype(np.float32).astype(np.float64)
    return dc, xf


@pytest.mark.parametrize("cfg", [configs.tiny_2d(), configs.ragged_2d()], ids=["tiny", "ragged"])
def test_learned_prolongation_matches_oracle(cfg):
    import paper_2012_10091_amd as m
    ctx, _, _ = make_ctx(cfg)
    p = _params(cfg)
    gnet = _gpu_net(p)
    dc, xf = _inputs(cfg)
    xf_d = to_dev(xf, F32)
    say("learned prolongation", cfg.name)
    ctx.prolong_smooth(to_dev(dc, F32), xf_d, None, n_sweeps=0, mode=m.MENKF_PROLONG_LEARNED, net=gnet)
    dproj = grids.prolong(dc, cfg.ratio, 2)
    corr = onet.learned_correction(p, dproj, xf)
    got = to_np(xf_d) - xf
    nn_o = corr - dproj
    assert np.linalg.norm(nn_o) > 0.1 * np.linalg.norm(dproj)      # the network contributes
    assert rel_l2(got, corr) < 2e-2, rel_l2(got, corr)
    assert rel_l2(got - dproj, nn_o) < 2e-2, rel_l2(got - dproj, nn_o)   # measured 3.9e-3 (BF16 storage)


@pytest.mark.parametrize("cfg", [configs.tiny_2d(), configs.ragged_2d()], ids=["tiny", "ragged"])
def test_learned_prolongation_matches_oracle_steps_at_bf16_storage(cfg):
    """The inference kernel against the oracle's steps with its BF16 storage
    (input and hidden activations; the test weights are BF16 already): the
    network's part of the correction agrees to the FP32 rounding of the
    corrected state, well inside what the BF16 storage itself costs."""
    import paper_2012_10091_amd as m
    ctx, _, _ = make_ctx(cfg)
    p = _params(cfg)
    gnet = _gpu_net(p)
    dc, xf = _inputs(cfg)
    xf_d = to_dev(xf, F32)
    say("learned prolongation at BF16 storage", cfg.name)
    ctx.prolong_smooth(to_dev(dc, F32), xf_d, None, n_sweeps=0, mode=m.MENKF_PROLONG_LEARNED, net=gnet)
    dproj = grids.prolong(dc, cfg.ratio, 2)
    inp = bf16_round(onet.make_input(p, dproj.astype(np.float32), xf.astype(np.float32)))
    a1 = bf16_round(np.maximum(onet.conv(inp, p.w1, p.b1), 0.0))
    a2 = bf16_round(np.maximum(onet.conv(a1, p.w2, p.b2), 0.0))
    nn_o = onet.conv(a2, p.w3, p.b3) / p.out_scale[:, None, None]
    got = to_np(xf_d) - xf - dproj
    assert rel_l2(got, nn_o) < 2e-3, rel_l2(got, nn_o)          # measured 2.4e-4 - 3.7e-4


def test_zero_last_layer_equals_plain_bitwise():
    import paper_2012_10091_amd as m
    cfg = configs.ragged_2d()
    ctx, _, _ = make_ctx(cfg)
    gnet = _gpu_net(_params(cfg, zero_last=True))
    dc, xf = _inputs(cfg)
    a, b = to_dev(xf, F32), to_dev(xf, F32)
    dcd = to_dev(dc, F32)
    say("zero last layer == plain")
    ctx.prolong_smooth(dcd, a, None, n_sweeps=0, mode=m.MENKF_PROLONG_LEARNED, net=gnet)
    ctx.prolong_smooth(dcd, b, None, n_sweeps=0, mode=m.MENKF_PROLONG_PLAIN)
    np.testing.assert_array_equal(to_np(a), to_np(b))


def test_fallback_guard_restores_plain_path():
    import paper_2012_10091_amd as m
    cfg = configs.tiny_2d()
    ctx, _, _ = make_ctx(cfg)
    gnet = _gpu_net(_params(cfg), guard=1e-20)
    dc, xf = _inputs(cfg)
    xprev = fields.truth_ic(cfg).astype(np.float32)
    a, b = to_dev(xf, F32), to_dev(xf, F32)
    dcd, xp = to_dev(dc, F32), to_dev(xprev, F32)
    say("fallback on every tile")
    ctx.prolong_smooth(dcd, a, xp, n_sweeps=1, mode=m.MENKF_PROLONG_LEARNED_FALLBACK, net=gnet)
    ctx.prolong_smooth(dcd, b, xp, n_sweeps=1, mode=m.MENKF_PROLONG_PLAIN)
    np.testing.assert_array_equal(to_np(a), to_np(b))
    assert int(gnet.fallback_count.item()) == (cfg.nx // 16) * (cfg.ny // 16)
    # a generous guard keeps the network everywhere
    gnet2 = _gpu_net(_params(cfg), guard=1e6)
    c = to_dev(xf, F32)
    ctx.prolong_smooth(dcd, c, xp, n_sweeps=0, mode=m.MENKF_PROLONG_LEARNED_FALLBACK, net=gnet2)
    assert int(gnet2.fallback_count.item()) == 0
    d = to_dev(xf, F32)
    ctx.prolong_smooth(dcd, d, None, n_sweeps=0, mode=m.MENKF_PROLONG_LEARNED, net=gnet2)
    np.testing.assert_array_equal(to_np(c), to_np(d))


def test_judge_distance_decision_and_stickiness():
    """LEARNED_FALLBACK with the judge: the device's distance
    |x_net - x_plain| / |x_plain - x^F_f| against the oracle's network and
    plain corrections (BF16 network tolerance), the network kept below the
    tolerance (bitwise = LEARNED), the plain correction above it (bitwise =
    PLAIN) and kept on the unjudged calls that follow, until a judged call
    accepts the network again."""
    import paper_2012_10091_amd as m
    from oracle import smooth
    from oracle.models import Model
    cfg = configs.tiny_2d()
    p = _params(cfg)
    dc, xf = _inputs(cfg)
    xprev = fields.truth_ic(cfg.with_(seed=cfg.seed + 3)).astype(np.float32).astype(np.float64)
    ns = 2
    dproj = grids.prolong(dc, cfg.ratio, 2)
    x_net = xf + onet.learned_correction(p, dproj, xf)
    x_pl = smooth.smooth(xf + dproj, xprev, Model(cfg, "fine"), ns, 0.5)
    d_o = np.linalg.norm(x_net - x_pl) / np.linalg.norm(x_pl - xf)
    dcd, xp = to_dev(dc, F32), to_dev(xprev, F32)
    ctx, _, _ = make_ctx(cfg)
    gnet = _gpu_net(p)
    gnet.judge_every, gnet.judge_tol = 1, 1e30
    say(f"judge: oracle distance {d_o:.4f}")
    a = to_dev(xf, F32)
    ctx.prolong_smooth(dcd, a, xp, n_sweeps=ns, mode=m.MENKF_PROLONG_LEARNED_FALLBACK, net=gnet)
    st = to_np(gnet.judge_stats)
    assert abs(st[0] - d_o) < 5e-2 * d_o, (st[0], d_o)
    assert list(st[1:]) == [1, 0, 0]
    b = to_dev(xf, F32)
    ctx.prolong_smooth(dcd, b, None, n_sweeps=0, mode=m.MENKF_PROLONG_LEARNED, net=gnet)
    np.testing.assert_array_equal(to_np(a), to_np(b))
    plain = to_dev(xf, F32)
    ctx.prolong_smooth(dcd, plain, xp, n_sweeps=ns, mode=m.MENKF_PROLONG_PLAIN)
    # a fresh context (judge state reset): judged every second call, tolerance below the distance
    ctx2, _, _ = make_ctx(cfg)
    g2 = _gpu_net(p)
    g2.judge_every, g2.judge_tol = 2, 0.5 * float(st[0])
    outs = []
    for k in range(3):
        if k == 2:
            g2.judge_tol = 1e30                  # the third call (judged) accepts the network
        c = to_dev(xf, F32)
        ctx2.prolong_smooth(dcd, c, xp, n_sweeps=ns, mode=m.MENKF_PROLONG_LEARNED_FALLBACK, net=g2)
        outs.append(to_np(c))
    np.testing.assert_array_equal(outs[0], to_np(plain))      # judged, rejected
    np.testing.assert_array_equal(outs[1], to_np(plain))      # not judged, plain kept
    np.testing.assert_array_equal(outs[2], to_np(b))          # judged, accepted
    st2 = to_np(g2.judge_stats)
    assert list(st2[1:]) == [2, 2, 0]
    assert ctx2.get_status() == 0


def _train_case(seed=3):
    cfg = configs.tiny_2d(nx=32, ny=32)
    r = np.random.default_rng(seed)
    npairs, H = 2, 32
    dproj = (0.01 * r.standard_normal((npairs, 4, H, H))).astype(np.float32)
    xf = np.stack([fields.truth_ic(cfg.with_(seed=cfg.seed + k)) for k in range(npairs)]).astype(np.float32)
    target = (dproj * 1.3 + 0.0005 * r.standard_normal(dproj.shape)).astype(np.float32)
    crops = np.array([[0, 0, 0], [1, 27, 5], [0, 13, 29]], dtype=np.int32)
    return cfg, dproj, xf, target, crops


def _oracle_loss_grad(p, dproj, xf, target, crops, C):
    dproj, xf, target = (np.asarray(a, dtype=np.float64) for a in (dproj, xf, target))
    n = crops.shape[0] * 4 * C * C
    grads = [np.zeros_like(t) for t in p.tensors()]
    loss = 0.0
    H, W = dproj.shape[-2:]
    for pr, y0, x0 in crops:
        inp = onet.make_input(p, dproj[pr], xf[pr])
        out, cache = onet.forward(p, inp)
        t = (target[pr] - dproj[pr]) * p.out_scale[:, None, None]
        ys = (y0 + np.arange(C)) % H
        xs = (x0 + np.arange(C)) % W
        mask = np.zeros((H, W), dtype=bool)
        mask[np.ix_(ys, xs)] = True
        diff = np.where(mask[None], out - t, 0.0)
        loss += float(np.sum(diff * diff))
        g, _ = onet.backward(p, cache, 2.0 * diff / n)
        for a, b in zip(grads, g):
            a += b
    return loss / n, grads


def test_training_gradient_matches_oracle():
    import paper_2012_10091_amd as m
    cfg, dproj, xf, target, crops = _train_case()
    p = _params(cfg, last_gain=3.0)
    gnet = _gpu_net(p)
    C = 10
    tr = m.Trainer(gnet, batch=crops.shape[0], crop=C)
    say("training gradient parity")
    loss = tr.step(to_dev(dproj, F32), to_dev(xf, F32), to_dev(target, F32),
                   torch.as_tensor(crops, device="cuda"), apply_adam=False)
    lo, go = _oracle_loss_grad(p, dproj, xf, target, crops, C)
    assert abs(float(loss.item()) - lo) < 2e-2 * lo, (float(loss.item()), lo)
    gg = m.unpack_params(tr.grad.cpu())
    for name, a, b in zip(("w1", "b1", "w2", "b2", "w3", "b3"), gg, go):
        assert rel_l2(a.double().numpy(), b) < 5e-2, (name, rel_l2(a.double().numpy(), b))


def _bf16_storage_loss_grad(p, dproj, xf, target, crops, C):
    """The oracle's forward and backward steps (oracle.net.conv and
    conv_backward, FP64) with the storage of the GPU training path: the
    input, the weights and the hidden activations rounded to BF16, the
    biases and every gradient kept wide."""
    q = dataclasses.replace(p, w1=bf16_round(p.w1), w2=bf16_round(p.w2), w3=bf16_round(p.w3))
    dproj, xf, target = (np.asarray(a, dtype=np.float64) for a in (dproj, xf, target))
    n = crops.shape[0] * 4 * C * C
    grads = [np.zeros_like(t) for t in p.tensors()]
    loss = 0.0
    H, W = dproj.shape[-2:]
    for pr, y0, x0 in crops:
        inp = bf16_round(onet.make_input(p, dproj[pr].astype(np.float32), xf[pr].astype(np.float32)))
        z1 = onet.conv(inp, q.w1, q.b1)
        a1 = bf16_round(np.maximum(z1, 0.0))
        z2 = onet.conv(a1, q.w2, q.b2)
        a2 = bf16_round(np.maximum(z2, 0.0))
        out = onet.conv(a2, q.w3, q.b3)
        t = (target[pr] - dproj[pr]) * p.out_scale[:, None, None]
        mask = np.zeros((H, W), dtype=bool)
        mask[np.ix_((y0 + np.arange(C)) % H, (x0 + np.arange(C)) % W)] = True
        diff = np.where(mask[None], out - t, 0.0)
        loss += float(np.sum(diff * diff))
        da2, dw3, db3 = onet.conv_backward(a2, q.w3, 2.0 * diff / n)
        da1, dw2, db2 = onet.conv_backward(a1, q.w2, da2 * (a2 > 0))
        _, dw1, db1 = onet.conv_backward(inp, q.w1, da1 * (a1 > 0))
        for a, b in zip(grads, (dw1, db1, dw2, db2, dw3, db3)):
            a += b
    return loss / n, grads


@pytest.mark.parametrize("seed,gain", [(3, 3.0), (7, 0.3)])
def test_training_gradient_matches_oracle_steps_at_bf16_storage(seed, gain):
    """Against the oracle's own steps taken with the path's BF16 storage the
    gradient of the MFMA training kernels agrees to FP32 accumulation error
    (the 5e-2 above is the BF16 storage itself: 0.4-2.3 % measured)."""
    import paper_2012_10091_amd as m
    cfg, dproj, xf, target, crops = _train_case(seed)
    p = _params(cfg, last_gain=gain)
    gnet = _gpu_net(p)
    C = 10
    tr = m.Trainer(gnet, batch=crops.shape[0], crop=C)
    say(f"training gradient vs the oracle's steps at BF16 storage, seed {seed}")
    loss = tr.step(to_dev(dproj, F32), to_dev(xf, F32), to_dev(target, F32),
                   torch.as_tensor(crops, device="cuda"), apply_adam=False)
    lo, go = _bf16_storage_loss_grad(p, dproj, xf, target, crops, C)
    assert abs(float(loss.item()) - lo) < 1e-6 * lo, (float(loss.item()), lo)
    gg = m.unpack_params(tr.grad.cpu())
    for name, a, b in zip(("w1", "b1", "w2", "b2", "w3", "b3"), gg, go):
        assert rel_l2(a.double().numpy(), b) < 2e-5, (name, rel_l2(a.double().numpy(), b))


def test_training_reduces_loss():
    import paper_2012_10091_amd as m
    cfg, dproj, xf, target, crops = _train_case(seed=4)
    p = _params(cfg, zero_last=True)
    gnet = _gpu_net(p)
    tr = m.Trainer(gnet, batch=3, crop=10, lr=3e-3)
    args = (to_dev(dproj, F32), to_dev(xf, F32), to_dev(target, F32), torch.as_tensor(crops, device="cuda"))
    say("training 60 Adam steps")
    first = float(tr.step(*args).item())
    for _ in range(59):
        tr.step(*args)
    last = float(tr.step(*args, apply_adam=False).item())
    assert last < 0.5 * first, (first, last)
    # the repacked BF16 weights follow the master copy
    w3 = m.unpack_params(gnet.params.cpu())[4]
    assert float(w3.abs().max()) > 0


def test_training_phases_equal_the_fused_step():
    """menkf_net_forward, menkf_net_backward and menkf_net_adam in that order
    give bitwise the loss, gradient, parameters, Adam moments and packed
    weights of menkf_net_train_step, over several steps."""
    import paper_2012_10091_amd as m
    cfg, dproj, xf, target, crops = _train_case(seed=5)
    p = _params(cfg, last_gain=1.0)
    fused, split = _gpu_net(p), _gpu_net(p)
    ta = m.Trainer(fused, batch=3, crop=10, lr=2e-3)
    tb = m.Trainer(split, batch=3, crop=10, lr=2e-3)
    args = (to_dev(dproj, F32), to_dev(xf, F32), to_dev(target, F32), torch.as_tensor(crops, device="cuda"))
    say("training phases vs the fused step, 4 steps")
    for k in range(4):
        la = float(ta.step(*args).item())
        lb = float(tb.forward(*args).item())
        tb.backward(*args)
        tb.adam(*args)
        torch.cuda.synchronize()
        assert la == lb, (k, la, lb)
        assert torch.equal(ta.grad, tb.grad), k
        assert torch.equal(fused.params, split.params), k
        assert torch.equal(ta.m, tb.m) and torch.equal(ta.v, tb.v), k
        assert torch.equal(fused.wpacked, split.wpacked), k
