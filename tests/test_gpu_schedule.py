"""GPU checks of the forecast schedules and their autotuner: every stencil
tile shape and member chunking must give forecasts bitwise equal to the
default schedule (the per-point arithmetic does not depend on the tiling),
and the default schedule itself is checked against the oracle in the
forecast parity tests."""

import numpy as np
import pytest
import torch

from synthetic import configs, fields
from tests.gpu_helpers import make_ctx, say, to_dev

pytestmark = pytest.mark.gpu

TILES = {"f32": [(32, 16), (64, 8), (32, 8), (16, 16), (64, 4), (0, 16), (0, 32)],
         "f64": [(32, 8), (16, 8), (16, 16), (64, 4)]}


def _forecast(ctx, cfg, dt, nsteps):
    xf = to_dev(fields.truth_ic(cfg), dt)
    mem = to_dev(fields.member_ics(cfg), dt)
    prev = torch.empty_like(xf)
    ctx.forecast(0, xf, nsteps, prev=prev)
    ctx.forecast(1, mem, nsteps)
    torch.cuda.synchronize()
    return xf.cpu(), prev.cpu(), mem.cpu()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_every_schedule_is_bitwise_equal(prec):
    cfg = configs.ragged_2d(precision=prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    ctx, _, _ = make_ctx(cfg)
    say(f"schedule sweep ragged_2d {prec}: default")
    ref = _forecast(ctx, cfg, dt, 2)
    for tile in TILES[prec]:
        for chunk in (0, 5, 1):
            say(f"schedule sweep ragged_2d {prec}: tile {tile} chunk {chunk}")
            ctx.set_schedule(0, tile, 0)
            ctx.set_schedule(1, tile, chunk)
            assert ctx.get_schedule(1) == {"tile": tile, "member_chunk": chunk}
            got = _forecast(ctx, cfg, dt, 2)
            for a, b in zip(got, ref):
                assert torch.equal(a, b), (tile, chunk)


def test_sweep_and_residual_do_not_depend_on_the_fine_tile():
    cfg = configs.ragged_2d(precision="f32")
    ctx, _, _ = make_ctx(cfg)
    rs = np.random.default_rng(3)
    x = to_dev(fields.truth_ic(cfg), torch.float32)
    xp = to_dev(fields.truth_ic(cfg) + 1e-3 * rs.standard_normal((4, cfg.ny, cfg.nx)), torch.float32)
    dc = torch.zeros((4, cfg.nyc, cfg.nxc), dtype=torch.float32, device="cuda")
    outs = []
    for tile in ((32, 16), (16, 16), (64, 4)):
        say(f"sweep/residual with fine tile {tile}")
        ctx.set_schedule(0, tile, 0)
        y = x.clone()
        ctx.prolong_smooth(dc, y, xp, n_sweeps=3, alpha=0.5)
        r = ctx.residual(y, xp)
        torch.cuda.synchronize()
        outs.append((y.cpu(), r.cpu()))
    for y, r in outs[1:]:
        assert torch.equal(y, outs[0][0])
        assert torch.equal(r, outs[0][1])


def test_autotune_picks_a_listed_schedule_and_keeps_results():
    cfg = configs.tiny_2d(precision="f32")
    ctx, _, _ = make_ctx(cfg)
    ref = _forecast(ctx, cfg, torch.float32, 2)
    scratch = to_dev(fields.member_ics(cfg), torch.float32)
    say("autotune tiny_2d coarse")
    best = ctx.autotune(1, scratch, 2, reps=1)
    say("autotune result", best)
    assert best["tile"] in TILES["f32"]
    assert 0 <= best["member_chunk"] <= cfg.n_members
    assert best["ms"] > 0
    assert ctx.get_schedule(1) == {"tile": best["tile"], "member_chunk": best["member_chunk"]}
    say("autotune tiny_2d fine")
    ctx.autotune(0, to_dev(fields.truth_ic(cfg), torch.float32), 2, reps=1)
    got = _forecast(ctx, cfg, torch.float32, 2)
    for a, b in zip(got, ref):
        assert torch.equal(a, b)


@pytest.mark.parametrize("side", [(256, 256), (512, 256), (768, 768)], ids=["coarse64x64", "coarse128x64",
                                                                            "coarse192x192"])
def test_row_march_is_bitwise_equal_to_the_tile_kernel(side):
    """Grids whose coarse rows the row-march schedules take whole (0 x 16:
    one RK stage per launch; 0 x 32: two stages per launch, the state
    alternating with a second array, so odd step counts end with a copy):
    forecasts of every member and x_{k-1}, with and without member chunks,
    bitwise equal to the default tile's."""
    nx, ny = side
    cfg = configs.tiny_2d(nx=nx, ny=ny, n_members=5, precision="f32", dt=5e-4 * 256 / nx)
    ctx, _, _ = make_ctx(cfg)
    mem0 = to_dev(fields.member_ics(cfg), torch.float32)
    outs = []
    for tile, chunk in (((32, 16), 0), ((0, 16), 0), ((0, 16), 2), ((0, 32), 0), ((0, 32), 2)):
        say(f"row march {nx}x{ny}: coarse tile {tile} chunk {chunk}")
        ctx.set_schedule(1, tile, chunk)
        m = mem0.clone()
        ctx.forecast(1, m, 3)
        p = mem0[:1].clone()
        pv = torch.empty_like(p)
        ctx.forecast(1, p, 2, prev=pv)
        torch.cuda.synchronize()
        outs.append((m.cpu(), p.cpu(), pv.cpu()))
    for got in outs[1:]:
        for a, b in zip(got, outs[0]):
            assert torch.equal(a, b)
