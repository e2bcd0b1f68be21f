"""GPU checks of the whole-cycle entry point and of the batch of uneven
independent instances: menkf_cycle equals the sequence of calls it stands
for; a batch spread over several streams equals the same cycles issued one
after another on one stream; its captured graph replays equal eager batches;
and at the full uneven-batch workload (48 instances, fine 256^2 to 768^2,
N 16 to 128, 256 to 2048 probes) one instance is followed through the oracle,
three more (learned prolongation) have their analysis checked against the
oracle's, and the batch is checked against sequential cycles."""

import numpy as np
import pytest
import torch

from oracle import cycle as ocycle
from oracle import enkf, grids, rng, smooth
from oracle.models import Model
from synthetic import configs, fields
from tests.gpu_helpers import make_ctx, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu

F32 = torch.float32
F64 = torch.float64


def _instance(cfg, with_y=True):
    ctx, idx, comp = make_ctx(cfg)
    fine = to_dev(fields.model_ic(cfg), F32)
    mem = to_dev(fields.member_ics(cfg), F32)
    inst = {"cfg": cfg, "ctx": ctx, "fine": fine, "prev": torch.empty_like(fine), "members": mem,
            "xs": torch.empty((4, cfg.nyc, cfg.nxc), dtype=F32, device="cuda"),
            "dc": torch.empty((4, cfg.nyc, cfg.nxc), dtype=F32, device="cuda"),
            "idx": idx, "comp": comp}
    if with_y:
        y = ocycle.observe_truth(cfg, fields.truth_ic(cfg), idx, comp) + fields.obs_noise(cfg, 1)
        inst["y"] = to_dev(y, F64)
    return inst


def _args(inst, cycle, n_sweeps=3, mode=0, net=None):
    c = inst["cfg"]
    return inst["ctx"].cycle_args(inst["fine"], inst["prev"], inst["members"], inst["xs"], inst["dc"], inst["y"],
                                  c.seed + 5, cycle, c.n_obs, n_sweeps=n_sweeps, alpha=0.5, mode=mode, net=net)


def _clone_state(inst):
    return {"fine": inst["fine"].clone(), "members": inst["members"].clone()}


def _set_state(inst, st):
    inst["fine"].copy_(st["fine"])
    inst["members"].copy_(st["members"])


def _small_uneven():
    return [configs.tiny_2d(),
            configs.ragged_2d(),
            configs.tiny_2d(nx=96, ny=96, n_members=16, n_probes=50, seed=2012 + 31),
            configs.tiny_2d(nx=128, ny=64, n_members=12, n_probes=30, seed=2012 + 32),
            configs.tiny_2d(nx=64, ny=128, n_members=5, n_probes=70, seed=2012 + 33)]


def _net():
    import paper_2012_10091_amd as m
    from paper_2012_10091_amd import learned
    s, o, sc = learned.default_scaling()
    return m.Net(learned.init_params(seed=7, last_gain=0.3), s, o, sc, guard=10.0)


@pytest.mark.parametrize("aux", [False, True], ids=["one-stream", "aux-stream"])
def test_cycle_equals_the_calls_it_stands_for(aux):
    cfg = configs.tiny_2d()
    a, b = _instance(cfg), _instance(cfg)
    side = torch.cuda.Stream() if aux else None
    say(f"menkf_cycle vs separate calls, tiny_2d, aux stream {aux}")
    for c in (1, 2):
        a["ctx"].cycle(a["fine"], a["prev"], a["members"], a["xs"], a["dc"], a["y"], cfg.seed + 5, c, cfg.n_obs,
                       n_sweeps=3, aux_stream=side)
        ctx = b["ctx"]
        ctx.forecast(0, b["fine"], cfg.n_obs, prev=b["prev"])
        ctx.forecast(1, b["members"], cfg.n_obs)
        ctx.restrict(b["fine"], b["xs"])
        ctx.gain(b["members"], b["xs"], b["y"], cfg.seed + 5, c)
        ctx.update(b["members"], b["dc"])
        ctx.prolong_smooth(b["dc"], b["fine"], b["prev"], n_sweeps=3, alpha=0.5)
    torch.cuda.synchronize()
    # with a second stream the x* column comes from (s^2 I + Y^T Y)^-1 Y^T d*
    # instead of the N_y x N_y factorisation: the member columns are the
    # same arithmetic, delta^C (and so the fine state) agree to FP64 roundoff
    # carried into FP32
    assert torch.equal(a["members"], b["members"])
    if aux:
        assert rel_l2(to_np(a["fine"]), to_np(b["fine"])) < 1e-6
    else:
        assert torch.equal(a["fine"], b["fine"])
    assert a["ctx"].get_status() == 0


def _mid_fork_cfg():
    # 4096 probes: 64 block steps whose first trailing updates have more
    # tiles than three per compute unit, so the second stream's fine
    # forecast is forked from inside the factorisation (and the x* system
    # right after the gain's front end)
    return configs.tiny_2d(nx=256, ny=256, n_members=16, n_probes=4096, seed=2012 + 41)


@pytest.mark.parametrize("cfg,ztol", [(configs.tiny_2d(), 1e-9), (configs.ragged_2d(), 1e-9),
                                      (configs.CONFIGS["C1"], 1e-9),
                                      (configs.tiny_2d(n_members=2, n_probes=3), 1e-9),
                                      (configs.tiny_1d(precision="f64", n_members=2, n_probes=1), 1e-9),
                                      (_mid_fork_cfg(), 1e-9)],
                         ids=["tiny2d", "ragged2d", "C1-f64", "tiny2d-N2-Ny3", "tiny1d-f64-N2-Ny1",
                              "256sq-Ny4096-mid-fork"])
def test_deferred_xstar_column_matches_the_factorisation(cfg, ztol):
    """The x* column of Z from the deferred path (second stream) equals the
    one of the N_y x N_y factorisation to FP64 roundoff; the member columns
    are bitwise equal."""
    dt = F64 if cfg.precision == "f64" else F32
    ctx_a, idx, comp = make_ctx(cfg)
    ctx_b, _, _ = make_ctx(cfg)
    fine = to_dev(fields.model_ic(cfg), dt)
    mem = to_dev(fields.member_ics(cfg), dt)
    y = to_dev(ocycle.observe_truth(cfg, fields.truth_ic(cfg), idx, comp) + fields.obs_noise(cfg, 1), F64)
    xs = torch.empty(cfg.coarse_shape, dtype=dt, device="cuda")
    a = [fine.clone(), torch.empty_like(fine), mem.clone(), xs.clone(), xs.clone()]
    b = [fine.clone(), torch.empty_like(fine), mem.clone(), xs.clone(), xs.clone()]
    side = torch.cuda.Stream()
    say(f"deferred x* column vs factorisation, {cfg.name}")
    ctx_a.cycle(*a, y, cfg.seed + 5, 1, cfg.n_obs, n_sweeps=1, aux_stream=side)
    ctx_b.cycle(*b, y, cfg.seed + 5, 1, cfg.n_obs, n_sweeps=1)
    za, zb = to_np(ctx_a.get_gain()), to_np(ctx_b.get_gain())
    N = cfg.n_members
    np.testing.assert_array_equal(za[:N], zb[:N])
    assert rel_l2(za[N], zb[N]) < ztol, rel_l2(za[N], zb[N])
    assert rel_l2(to_np(a[4]), to_np(b[4])) < (1e-9 if cfg.precision == "f64" else 1e-6)
    assert ctx_a.get_status() == 0


def test_two_stream_cycle_graph_replays_match_eager_at_a_mid_fork_size():
    """menkf_cycle with a second stream, captured once and replayed three
    times with eager cycles and synchronisations in between: every replay
    is bitwise the eager cycle (both forks of the second stream, the one
    inside the factorisation included)."""
    import paper_2012_10091_amd as m
    cfg = _mid_fork_cfg()
    g_i, e_i = _instance(cfg), _instance(cfg)
    side_g, side_e = torch.cuda.Stream(), torch.cuda.Stream()
    stream = torch.cuda.Stream()
    say("graph of a two-stream cycle at 4096 probes, 3 replays against eager cycles")
    with torch.cuda.stream(stream):
        m.Graph.begin(stream)
        g_i["ctx"].cycle(g_i["fine"], g_i["prev"], g_i["members"], g_i["xs"], g_i["dc"], g_i["y"], cfg.seed + 5,
                         1, cfg.n_obs, n_sweeps=1, aux_stream=side_g)
        graph = m.Graph.end(stream)
    torch.cuda.synchronize()
    for rep in range(3):
        e_i["ctx"].cycle(e_i["fine"], e_i["prev"], e_i["members"], e_i["xs"], e_i["dc"], e_i["y"], cfg.seed + 5,
                         1, cfg.n_obs, n_sweeps=1, aux_stream=side_e)
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        assert torch.equal(g_i["members"], e_i["members"]), rep
        assert torch.equal(g_i["fine"], e_i["fine"]), rep
    assert g_i["ctx"].get_status() == 0 and e_i["ctx"].get_status() == 0


def test_c1_cycles_fp64_with_the_deferred_column_match_oracle():
    cfg = configs.CONFIGS["C1"]
    ctx, idx, comp = make_ctx(cfg)
    truth = fields.truth_ic(cfg)
    st_o = ocycle.State(fine=fields.model_ic(cfg), members=fields.member_ics(cfg))
    fine_d, mem_d = to_dev(st_o.fine, F64), to_dev(st_o.members, F64)
    prev_d = torch.empty_like(fine_d)
    xs_d = torch.empty(cfg.coarse_shape, dtype=F64, device="cuda")
    dc_d = torch.empty_like(xs_d)
    mt = Model(cfg, "fine")
    side = torch.cuda.Stream()
    for c in range(1, cfg.n_cycles + 1):
        truth, _ = mt.forecast(truth, cfg.n_obs)
        y = ocycle.observe_truth(cfg, truth, idx, comp) + fields.obs_noise(cfg, c)
        say(f"C1 cycle {c} with the deferred x* column")
        st_o = ocycle.cycle(cfg, st_o, y, idx, comp, n_sweeps=1, seed=cfg.seed + 5)
        ctx.cycle(fine_d, prev_d, mem_d, xs_d, dc_d, to_dev(y, F64), cfg.seed + 5, c, cfg.n_obs, n_sweeps=1,
                  alpha=0.5, aux_stream=side)
        assert rel_l2(to_np(fine_d), st_o.fine) < 1e-10, c
        assert rel_l2(to_np(mem_d), st_o.members) < 1e-10, c


def test_batch_on_lanes_equals_sequential_cycles():
    import paper_2012_10091_amd as m
    insts = [_instance(c) for c in _small_uneven()]
    net = _net()
    modes = [0, 2, 0, 2, 0]
    init = [_clone_state(i) for i in insts]
    batch = m.Batch(n_lanes=3)
    stream = torch.cuda.Stream()
    say("batch of 5 uneven instances on 3 lanes, 2 cycles")
    for c in (1, 2):
        args = [_args(i, c, mode=mo, net=net if mo else None) for i, mo in zip(insts, modes)]
        batch.cycle(args, stream=stream)
    stream.synchronize()
    lanes = batch.lanes()
    assert sorted(set(lanes)) == [0, 1, 2]
    got = [_clone_state(i) for i in insts]
    for i, st in zip(insts, init):
        _set_state(i, st)
    say("same cycles one after another on one stream")
    for c in (1, 2):
        for i, mo in zip(insts, modes):
            i["ctx"].cycle(i["fine"], i["prev"], i["members"], i["xs"], i["dc"], i["y"], i["cfg"].seed + 5, c,
                           i["cfg"].n_obs, n_sweeps=3, alpha=0.5, mode=mo, net=net if mo else None)
    torch.cuda.synchronize()
    for i, g in zip(insts, got):
        assert i["ctx"].get_status() == 0
        assert torch.equal(i["fine"], g["fine"]), i["cfg"].name
        assert torch.equal(i["members"], g["members"]), i["cfg"].name


def test_batch_graph_replays_equal_eager_batches():
    import paper_2012_10091_amd as m
    insts = [_instance(c) for c in _small_uneven()[:4]]
    init = [_clone_state(i) for i in insts]
    batch = m.Batch(n_lanes=2)
    stream = torch.cuda.Stream()
    args = [_args(i, m.MENKF_CYCLE_DEVICE) for i in insts]
    say("capture the batch cycle of 4 instances")
    with torch.cuda.stream(stream):
        m.Graph.begin(stream)
        batch.cycle(args, stream=stream)
        g = m.Graph.end(stream)
    for i in insts:
        i["ctx"].set_cycle(1, stream=stream)
    stream.synchronize()
    replays = []
    for rep in range(3):
        say(f"replay {rep}")
        g.launch(stream)
        stream.synchronize()
        # eager work of the program between replays
        torch.cuda.synchronize()
        replays.append([_clone_state(i) for i in insts])
    for i, st in zip(insts, init):
        _set_state(i, st)
        i["ctx"].set_cycle(1)
    say("eager batches")
    for rep in range(3):
        batch.cycle([_args(i, m.MENKF_CYCLE_DEVICE) for i in insts], stream=stream)
        stream.synchronize()
        for i, r in zip(insts, replays[rep]):
            assert torch.equal(i["fine"], r["fine"]), (rep, i["cfg"].name)
            assert torch.equal(i["members"], r["members"]), (rep, i["cfg"].name)


def test_uneven_batch_full_size():
    import paper_2012_10091_amd as m
    from paper_2012_10091_amd import learned
    cfgs = configs.uneven_batch()
    say(f"uneven batch: {len(cfgs)} instances, building states")
    insts = [_instance(c) for c in cfgs]
    net = learned.load(learned.weights_for("ns2d_512_128_n32"), guard=10.0)
    small = min(range(len(cfgs)), key=lambda k: cfgs[k].nx * cfgs[k].n_members * cfgs[k].n_probes)
    big = max(range(len(cfgs)), key=lambda k: cfgs[k].nx * cfgs[k].n_members)
    # the oracle follows the smallest instance with plain prolongation; the
    # others use the learned prolongation with its per-tile fallback
    modes = [0 if k == small else m.MENKF_PROLONG_LEARNED_FALLBACK for k in range(len(cfgs))]
    init = [_clone_state(i) for i in insts]
    batch = m.Batch(n_lanes=4)
    stream = torch.cuda.Stream()
    say("one batch cycle")
    batch.cycle([_args(i, 1, mode=mo, net=net if mo else None) for i, mo in zip(insts, modes)], stream=stream)
    stream.synchronize()
    for i in insts:
        assert i["ctx"].get_status() == 0, i["cfg"].name
        assert torch.isfinite(i["fine"]).all() and torch.isfinite(i["members"]).all(), i["cfg"].name
    got = {k: _clone_state(insts[k]) for k in range(len(cfgs))}

    # every instance: the batch equals its own cycle issued alone
    for k in sorted({small, big, 0, len(cfgs) - 1}):
        i = insts[k]
        _set_state(i, init[k])
        say(f"sequential cycle of {i['cfg'].name}")
        a = _args(i, 1, mode=modes[k], net=net if modes[k] else None)
        i["ctx"].cycle(i["fine"], i["prev"], i["members"], i["xs"], i["dc"], i["y"], i["cfg"].seed + 5, 1,
                       i["cfg"].n_obs, n_sweeps=3, alpha=0.5, mode=modes[k], net=net if modes[k] else None)
        torch.cuda.synchronize()
        assert torch.equal(i["fine"], got[k]["fine"]), i["cfg"].name
        assert torch.equal(i["members"], got[k]["members"]), i["cfg"].name
        del a

    # the smallest instance through the oracle: forecast parity, then the
    # analysis and fine correction from the device forecast
    i, cfg = insts[small], cfgs[small]
    say(f"oracle check of {cfg.name}: fine {cfg.nx}^2, N {cfg.n_members}, {cfg.n_probes} probes")
    fine0 = to_np(init[small]["fine"])
    mem0 = to_np(init[small]["members"])
    xf_d, mem_d = init[small]["fine"].clone(), init[small]["members"].clone()
    prev_d = torch.empty_like(xf_d)
    i["ctx"].forecast(0, xf_d, cfg.n_obs, prev=prev_d)
    i["ctx"].forecast(1, mem_d, cfg.n_obs)
    o_f, o_prev = Model(cfg, "fine").forecast(fine0, cfg.n_obs)
    o_m, _ = Model(cfg, "coarse").forecast(mem0, cfg.n_obs)
    assert rel_l2(to_np(xf_d), o_f) < 1e-5
    assert rel_l2(to_np(mem_d), o_m) < 1e-5
    xf, xprev, memf = to_np(xf_d), to_np(prev_d), to_np(mem_d)
    xstar = grids.restrict(xf, cfg.ratio, 2)
    eps = rng.perturbations(cfg.seed + 5, 1, cfg.n_members, cfg.n_probes, cfg.obs_sigma)
    res = enkf.analysis(memf, xstar, to_np(i["y"]), eps, ocycle.make_H(cfg, i["idx"], i["comp"]), cfg.obs_sigma)
    x = xf + grids.prolong(res["delta"], cfg.ratio, 2)
    x = smooth.smooth(x, xprev, Model(cfg, "fine"), 3, 0.5)
    # analysed states to the FP32 forecast bound, increments to the BF16x3
    # analysis bound (members) and the FP32 sweep bound (fine)
    assert rel_l2(to_np(got[small]["members"]), res["members"]) < 1e-5
    assert rel_l2(to_np(got[small]["members"]) - memf, res["members"] - memf) < 1e-3
    assert rel_l2(to_np(got[small]["fine"]), x) < 1e-5
    assert rel_l2(to_np(got[small]["fine"]) - xf, x - xf) < 1e-2

    # three more instances (learned prolongation, the largest ensemble and
    # the most probes among them): the members after the batch cycle against
    # the oracle's analysis of the device forecast (the prolongation does not
    # enter the members)
    most_probes = max(range(len(cfgs)), key=lambda k: cfgs[k].n_probes)
    for k in sorted({big, most_probes, len(cfgs) // 2} - {small}):
        i, cfg = insts[k], cfgs[k]
        say(f"oracle analysis of {cfg.name}: fine {cfg.nx}^2, N {cfg.n_members}, {cfg.n_probes} probes")
        xf_d, mem_d = init[k]["fine"].clone(), init[k]["members"].clone()
        i["ctx"].forecast(0, xf_d, cfg.n_obs)
        i["ctx"].forecast(1, mem_d, cfg.n_obs)
        memf = to_np(mem_d)
        xstar = grids.restrict(to_np(xf_d), cfg.ratio, 2)
        eps = rng.perturbations(cfg.seed + 5, 1, cfg.n_members, cfg.n_probes, cfg.obs_sigma)
        res = enkf.analysis(memf, xstar, to_np(i["y"]), eps, ocycle.make_H(cfg, i["idx"], i["comp"]), cfg.obs_sigma)
        assert rel_l2(to_np(got[k]["members"]), res["members"]) < 1e-5, cfg.name
        assert rel_l2(to_np(got[k]["members"]) - memf, res["members"] - memf) < 1e-3, cfg.name
