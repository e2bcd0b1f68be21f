"""menkf_diagnostics_noalloc: the diagnostics with their reduction partials in
the library's static device array, on a context with no workspace, against
menkf_diagnostics (workspace partials) on the same states.  Two calls in a
row on one GPU, the second on a smaller state, so the second reuses the
array the first left behind."""

import ctypes

import numpy as np
import pytest
import torch

import paper_2012_10091_amd as m
from synthetic import configs, fields
from tests.gpu_helpers import say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _states(cfg, seed):
    r = np.random.default_rng(seed)
    xt = fields.model_ic(cfg)
    xa = xt + 0.01 * r.standard_normal(xt.shape)
    xa[(3,) + (2,) * (xa.ndim - 1)] = np.nan          # one non-finite entry to count
    dt = torch.float64 if cfg.precision == "f64" else torch.float32
    return to_dev(xa, dt), to_dev(xt, dt)


def _noalloc(lib, ctx, xa, xt):
    out = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
    st = lib.menkf_diagnostics_noalloc(ctx.handle, ctypes.c_void_p(xa.data_ptr()), ctypes.c_void_p(xt.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, m.binding.last_error(ctx.handle)
    return to_np(out)


def test_noalloc_diagnostics_match_the_workspace_variant():
    lib = m.load_library()
    cases = [("C3-fine-f32", configs.CONFIGS["C3"]), ("tiny2d-f64", configs.tiny_2d(precision="f64"))]
    for k, (name, cfg) in enumerate(cases):
        say(f"noalloc diagnostics call {k + 1}: {name} {cfg.ny}x{cfg.nx}")
        bare = m.Context(cfg, allocate=False)
        ref = m.Context(cfg)
        xa, xt = _states(cfg, 10 + k)
        got = _noalloc(lib, bare, xa, xt)
        want = to_np(ref.diagnostics(xa, xt))
        # the same kernels in the same reduction order: bitwise equal
        np.testing.assert_array_equal(got, want)
        assert got[2] == 1 and got[1] > 0
        # the workspace variant refuses a context without workspace
        with pytest.raises(m.MenkfError):
            bare.diagnostics(xa, xt)
