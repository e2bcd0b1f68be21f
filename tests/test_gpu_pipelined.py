"""GPU checks of the pipelined cycle (menkf_cycle with pipelined = 1 and
menkf_cycle_flush): the fine-grid correction of Algo. 4 steps 5-6 deferred
to the next call changes no arithmetic, so K pipelined calls and a flush are
bitwise K ordinary calls, eager and as a replayed graph, with the plain and
the judged learned correction, on one stream and with a second stream, for
the exact-R gain (second stream forked inside the factorisation) and the
ensemble-space gain (second stream beside the member forecast)."""

import dataclasses

import pytest
import torch

from oracle import cycle as ocycle
from synthetic import configs, fields
from tests.gpu_helpers import make_ctx, say, to_dev

pytestmark = pytest.mark.gpu

F32 = torch.float32
F64 = torch.float64


def _instance(cfg):
    ctx, idx, comp = make_ctx(cfg)
    fine = to_dev(fields.model_ic(cfg), F32)
    y = ocycle.observe_truth(cfg, fields.truth_ic(cfg), idx, comp) + fields.obs_noise(cfg, 1)
    return {"ctx": ctx, "fine": fine, "prev": torch.empty_like(fine),
            "members": to_dev(fields.member_ics(cfg), F32),
            "xs": torch.empty(cfg.coarse_shape, dtype=F32, device="cuda"),
            "dc": torch.zeros(cfg.coarse_shape, dtype=F32, device="cuda"), "y": to_dev(y, F64)}


def _net(judge_every):
    import paper_2012_10091_amd as m
    from paper_2012_10091_amd import learned
    s, o, sc = learned.default_scaling()
    return m.Net(learned.init_params(seed=7, last_gain=0.3), s, o, sc, guard=10.0, judge_every=judge_every,
                 judge_tol=1.0)


def _cycle(inst, cfg, c, mode, net, aux, pipelined, stream=None):
    inst["ctx"].cycle(inst["fine"], inst["prev"], inst["members"], inst["xs"], inst["dc"], inst["y"], cfg.seed + 5,
                      c, cfg.n_obs, n_sweeps=3, alpha=0.5, mode=mode, net=net, stream=stream, aux_stream=aux,
                      pipelined=pipelined)


def _flush(inst, mode, net, stream=None):
    inst["ctx"].cycle_flush(inst["fine"], inst["prev"], inst["dc"], n_sweeps=3, alpha=0.5, mode=mode, net=net,
                            stream=stream)


def _ensemble_space(cfg):
    # the ensemble-space gain: with a second stream the fine forecast runs
    # beside the member forecast (no deferred x* column)
    @dataclasses.dataclass(frozen=True)
    class C(type(cfg)):
        gain_mode: int = 2
    return C(**dataclasses.asdict(cfg))


@pytest.mark.parametrize("ens", [False, True], ids=["exact-R", "ensemble-space"])
@pytest.mark.parametrize("aux", [False, True], ids=["one-stream", "aux-stream"])
@pytest.mark.parametrize("mode", [0, 2], ids=["plain", "learned-judged"])
def test_pipelined_cycles_and_flush_equal_ordinary_cycles(aux, mode, ens):
    cfg = _ensemble_space(configs.tiny_2d()) if ens else configs.tiny_2d()
    a, b = _instance(cfg), _instance(cfg)
    na, nb = (_net(2), _net(2)) if mode else (None, None)
    sa = torch.cuda.Stream() if aux else None
    sb = torch.cuda.Stream() if aux else None
    say(f"pipelined vs ordinary cycles, tiny_2d, mode {mode}, aux stream {aux}, ensemble-space gain {ens}")
    for c in (1, 2, 3):
        _cycle(a, cfg, c, mode, na, sa, True)
        _cycle(b, cfg, c, mode, nb, sb, False)
        torch.cuda.synchronize()
        # the members do not wait for the correction
        assert torch.equal(a["members"], b["members"]), c
    _flush(a, mode, na)
    # a second flush has nothing pending
    _flush(a, mode, na)
    torch.cuda.synchronize()
    for k in ("fine", "prev", "members", "dc"):
        assert torch.equal(a[k], b[k]), k
    if mode:
        assert torch.equal(na.judge_stats, nb.judge_stats)
    assert a["ctx"].get_status() == 0 and b["ctx"].get_status() == 0


def test_pipelined_graph_replays_equal_ordinary_cycles_at_a_mid_fork_size():
    """A pipelined two-stream cycle at 4096 probes (the second stream forked
    from inside the factorisation), captured once and replayed three times
    with synchronisations in between, then flushed: bitwise three ordinary
    eager cycles."""
    import paper_2012_10091_amd as m
    cfg = configs.tiny_2d(nx=256, ny=256, n_members=16, n_probes=4096, seed=2012 + 41)
    g, e = _instance(cfg), _instance(cfg)
    side_g, side_e = torch.cuda.Stream(), torch.cuda.Stream()
    stream = torch.cuda.Stream()
    say("graph of a pipelined two-stream cycle at 4096 probes, 3 replays against ordinary eager cycles")
    with torch.cuda.stream(stream):
        m.Graph.begin(stream)
        _cycle(g, cfg, 1, 0, None, side_g, True, stream=stream)
        graph = m.Graph.end(stream)
    torch.cuda.synchronize()
    for rep in range(3):
        _cycle(e, cfg, 1, 0, None, side_e, False)
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        assert torch.equal(g["members"], e["members"]), rep
    with torch.cuda.stream(stream):
        _flush(g, 0, None, stream=stream)
    stream.synchronize()
    assert torch.equal(g["fine"], e["fine"])
    assert torch.equal(g["prev"], e["prev"])
    assert g["ctx"].get_status() == 0 and e["ctx"].get_status() == 0


def test_pipelined_cycle_rejects_feedback():
    import paper_2012_10091_amd as m
    cfg = configs.tiny_2d()
    a = _instance(cfg)
    with pytest.raises(m.MenkfError):
        a["ctx"].cycle(a["fine"], a["prev"], a["members"], a["xs"], a["dc"], a["y"], cfg.seed + 5, 1, cfg.n_obs,
                       n_sweeps=3, feedback=True, pipelined=True)
