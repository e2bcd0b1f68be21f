"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, validates configurations on the host and plans its
workspace.  No device computation is requested here."""

import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "menkf.h")


def _lib():
    import paper_2012_10091_amd as m
    return m.load_library()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(menkf_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_entry_point():
    lib = _lib()
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_declares_the_same_names():
    from paper_2012_10091_amd import _lib as L
    assert sorted(L.SIGNATURES) == declared_symbols()


def test_ram_ratio_matches_paper(golden_dir):
    from paper_2012_10091_amd import ram_ratio
    with open(os.path.join(golden_dir, "ram_ratio.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for dim, r, n, printed in rows:
        v = ram_ratio(int(dim), int(r), int(n))
        # the paper prints three significant digits
        assert abs(v - float(printed)) <= 0.5 * 10 ** (-(len(printed.split(".")[1]))) + 1e-12, (v, printed)


def _create(**kw):
    import paper_2012_10091_amd as m
    from paper_2012_10091_amd import binding as b
    base = dict(model=m.MENKF_NS2D, nx=64, ny=64, ratio=4, n_members=8, n_probes=16, dt=1e-3)
    base.update(kw)
    cfg = b.make_config(**base)
    lib = _lib()
    h = ctypes.c_void_p()
    st = lib.menkf_create(ctypes.byref(cfg), ctypes.byref(h))
    return st, h, lib


@pytest.mark.parametrize("kw,code", [
    (dict(ratio=3), -2),                       # 64 not a multiple of 3
    (dict(model=7), -1),
    (dict(precision=5), -1),
    (dict(n_members=1), -1),                   # anomalies need N >= 2
    (dict(n_members=257), -1),
    (dict(n_probes=0), -1),
    (dict(nx=12, ratio=4), -2),                # coarse grid of 3 nodes
    (dict(dt=0.0), -1),
    (dict(obs_sigma=0.0), -1),
    (dict(obs_sigma=0.0, gain_mode=2), -1),    # ensemble space needs R = s^2 I, s > 0
    (dict(gain_mode=3), -1),
    (dict(gain_mode=1, n_probes=20, n_members=8), -1),   # Y Y^T + E E^T singular
    (dict(model=1, ny=4), -2),                 # 1D needs ny = 1
])
def test_create_rejects_bad_configurations(kw, code):
    st, h, lib = _create(**kw)
    assert st == code
    assert not h.value
    assert lib.menkf_last_error(None)


def test_create_and_workspace_plan():
    st, h, lib = _create(n_members=64, n_probes=4096, nx=1024, ny=1024)
    assert st == 0
    n = ctypes.c_size_t()
    assert lib.menkf_workspace_size(h, ctypes.byref(n)) == 0
    fine = 1024 * 1024 * 4 * 4
    coarse = 64 * 256 * 256 * 4 * 4
    chol = (4096 + 192) ** 2 * 8
    assert n.value >= 3 * fine + 3 * coarse + chol
    assert n.value < 3 * fine + 3 * coarse + chol + 64 * 2 ** 20
    # calls that need a workspace refuse to run without one
    assert lib.menkf_forecast(h, 0, ctypes.c_void_p(1), 1, 1, None, None) == -7
    lib.menkf_destroy(h)


def test_ensemble_space_mode_plans_its_small_system():
    st, h, lib = _create(gain_mode=2, n_members=64, n_probes=4096, nx=1024, ny=1024)
    assert st == 0
    lib.menkf_destroy(h)


def test_sample_mode_accepts_small_observation_count():
    st, h, lib = _create(gain_mode=1, n_probes=14, n_members=8)
    assert st == 0
    lib.menkf_destroy(h)


def test_schedule_defaults_and_validation():
    import paper_2012_10091_amd as m
    from paper_2012_10091_amd import _lib as L
    for prec, default in ((m.MENKF_F32, (32, 16)), (m.MENKF_F64, (32, 8))):
        st, h, lib = _create(precision=prec)
        assert st == 0
        sc = L.MenkfSchedule()
        for level in (0, 1):
            assert lib.menkf_get_schedule(h, level, ctypes.byref(sc)) == 0
            assert (sc.tile_x, sc.tile_y, sc.member_chunk) == (*default, 0)
        assert lib.menkf_set_schedule(h, 1, ctypes.byref(L.MenkfSchedule(16, 16, 3, 0))) == 0
        assert lib.menkf_get_schedule(h, 1, ctypes.byref(sc)) == 0
        assert (sc.tile_x, sc.tile_y, sc.member_chunk) == (16, 16, 3)
        # zero tile = default of the precision; unknown shapes and negative chunks are refused
        assert lib.menkf_set_schedule(h, 0, ctypes.byref(L.MenkfSchedule(0, 0, 0, 0))) == 0
        assert lib.menkf_get_schedule(h, 0, ctypes.byref(sc)) == 0
        assert (sc.tile_x, sc.tile_y) == default
        assert lib.menkf_set_schedule(h, 1, ctypes.byref(L.MenkfSchedule(48, 16, 0, 0))) == -1
        assert lib.menkf_set_schedule(h, 1, ctypes.byref(L.MenkfSchedule(32, 8, -1, 0))) == -1
        assert lib.menkf_set_schedule(h, 2, ctypes.byref(L.MenkfSchedule(32, 8, 0, 0))) == -1
        assert lib.menkf_get_schedule(h, 1, ctypes.byref(sc)) == 0
        assert (sc.tile_x, sc.tile_y, sc.member_chunk) == (16, 16, 3)
        # the 64x8 FP32 tile exceeds nothing but is FP32-only
        assert lib.menkf_set_schedule(h, 1, ctypes.byref(L.MenkfSchedule(64, 8, 0, 0))) == (0 if prec == 0 else -1)
        # the autotuner needs a workspace
        assert lib.menkf_autotune(h, 1, ctypes.c_void_p(1), 8, 1, 1, None, None, None) == -7
        lib.menkf_destroy(h)


def _inlet(**kw):
    base = dict(model=3, nx=800, ny=1, ratio=4, n_members=100, n_probes=80, dt=2e-4, length=10.0,
                nu=0.005, obs_sigma=0.05, u0=1.0, omega=6.283185307179586, theta_sigma=(0.005, 0.005),
                precision=1)
    base.update(kw)
    return _create(**base)


def test_inlet_model_plans_the_parameter_filter():
    st, h, lib = _inlet()
    assert st == 0, lib.menkf_last_error(None)
    n3 = ctypes.c_size_t()
    assert lib.menkf_workspace_size(h, ctypes.byref(n3)) == 0
    lib.menkf_destroy(h)
    st, h, lib = _create(model=1, nx=800, ny=1, ratio=4, n_members=100, n_probes=80, dt=2e-4, length=10.0,
                         nu=0.005, obs_sigma=0.05, precision=1)
    assert st == 0
    n1 = ctypes.c_size_t()
    assert lib.menkf_workspace_size(h, ctypes.byref(n1)) == 0
    lib.menkf_destroy(h)
    # the trial member copy (100 x 200 doubles) and theta^f (100 x 2 doubles)
    assert n3.value - n1.value >= 100 * 200 * 8 + 100 * 2 * 8
    assert n3.value - n1.value < 100 * 200 * 8 + 100 * 2 * 8 + 1024


@pytest.mark.parametrize("kw,code", [
    (dict(nx=5296, ratio=4), -6),                # F64 row beyond the LDS window
    (dict(nx=8196, ratio=4, precision=0), -6),   # F32 row beyond 8 points x 1024 threads
    (dict(theta_sigma=(-1.0, 0.0)), -1),
    (dict(u0=float("nan")), -1),
    (dict(omega=float("inf")), -1),
])
def test_inlet_model_rejects(kw, code):
    st, h, lib = _inlet(**kw)
    assert st == code
    assert not h.value


def test_inlet_model_limits_are_accepted():
    for kw in (dict(nx=5288, ratio=4), dict(nx=8192, ratio=4, precision=0)):
        st, h, lib = _inlet(**kw)
        assert st == 0, (kw, lib.menkf_last_error(None))
        lib.menkf_destroy(h)


def test_dual_calls_need_a_workspace():
    st, h, lib = _inlet()
    assert st == 0
    one = ctypes.c_void_p(8)
    assert lib.menkf_forecast_inlet(h, 1, one, 1, 1, None, one, one, None) == -7
    assert lib.menkf_param_perturb(h, one, one, 1, 1, None) == -7
    assert lib.menkf_param_update(h, one, one, one, None) == -7
    lib.menkf_destroy(h)


def _euler(**kw):
    base = dict(model=4, nx=800, ny=1, ratio=4, n_members=100, n_probes=80, dt=6e-4, length=10.0,
                obs_sigma=5e-4, gamma=1.4, mach=0.4, omega=6.283185307179586, theta_sigma=(1e-5, 0.0),
                filter_sigma=1.0, precision=1)
    base.update(kw)
    return _create(**base)


def test_euler_model_plans_three_fields():
    st, h, lib = _euler()
    assert st == 0, lib.menkf_last_error(None)
    n4 = ctypes.c_size_t()
    assert lib.menkf_workspace_size(h, ctypes.byref(n4)) == 0
    lib.menkf_destroy(h)
    st, h, lib = _inlet()
    n3 = ctypes.c_size_t()
    assert lib.menkf_workspace_size(h, ctypes.byref(n3)) == 0
    lib.menkf_destroy(h)
    # three fields instead of one: the fine and coarse buffers triple
    assert n4.value > n3.value + 2 * (3 * 800 * 8 + 3 * 100 * 200 * 8)


@pytest.mark.parametrize("kw,code", [
    (dict(nx=1800, ratio=4), -6),                # F64 state beyond the LDS window
    (dict(nx=3616, ratio=4, precision=0), -6),
    (dict(mach=1.2), -1),                        # supersonic inlet
    (dict(mach=0.0), -1),
    (dict(gamma=1.0), -1),
    (dict(filter_sigma=1.5), -1),
    (dict(filter_sigma=-0.1), -1),
    (dict(nx=28, ratio=4, n_probes=8), -2),      # 7 coarse nodes: no room for the filter stencils
])
def test_euler_model_rejects(kw, code):
    st, h, lib = _euler(**kw)
    assert st == code, lib.menkf_last_error(None)
    assert not h.value


def test_euler_model_limits_are_accepted():
    for kw in (dict(nx=1792, ratio=4), dict(nx=3612, ratio=4, precision=0), dict(nx=32, ratio=4, n_probes=8)):
        st, h, lib = _euler(**kw)
        assert st == 0, (kw, lib.menkf_last_error(None))
        lib.menkf_destroy(h)


E_ARG, E_WORKSPACE = -1, -7   # menkf_status codes of the header


def test_training_phases_validate_on_the_host():
    """menkf_net_forward / _backward / _adam reject bad descriptors before
    any device work, like menkf_net_train_step (status codes only, no GPU)."""
    from paper_2012_10091_amd import _lib as L
    lib = _lib()
    for name in ("menkf_net_train_step", "menkf_net_forward", "menkf_net_backward", "menkf_net_adam"):
        fn = getattr(lib, name)
        assert fn(None, None) == E_ARG, name
        d = L.MenkfNetTrain()           # all pointers NULL
        assert fn(ctypes.byref(d), None) == E_ARG, name
    # a complete descriptor (dummy, never dereferenced: validation fails
    # first) without Adam moments: only the Adam phase refuses it
    d = L.MenkfNetTrain()
    for f in ("params", "grad", "dproj", "xf", "target", "crops_dev", "loss_dev", "workspace_dev"):
        setattr(d, f, 256)
    d.npairs, d.H, d.W, d.batch, d.crop, d.step = 1, 32, 32, 1, 8, 1
    d.workspace_bytes = 0
    assert lib.menkf_net_adam(ctypes.byref(d), None) == E_ARG
    # with moments but no workspace: every phase reports the workspace
    d.adam_m, d.adam_v = 256, 256
    for name in ("menkf_net_forward", "menkf_net_backward", "menkf_net_adam"):
        assert getattr(lib, name)(ctypes.byref(d), None) == E_WORKSPACE, name


def test_set_observations_is_set_probes():
    lib = _lib()
    assert lib.menkf_set_observations(None, None, None) == E_ARG
    st, h, lib = _create()
    assert st == 0
    try:
        assert lib.menkf_set_observations(h, None, None) == E_ARG
        assert lib.menkf_set_probes(h, None, None) == E_ARG
    finally:
        lib.menkf_destroy(h)
