"""ctypes loader for libmenkf.so.

The library is the product: if it is missing this module raises, it never
falls back to anything else.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmenkf.so")

c_int32 = ctypes.c_int32
c_uint64 = ctypes.c_uint64
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
c_char_p = ctypes.c_char_p


class MenkfConfig(ctypes.Structure):
    _fields_ = [
        ("model", c_int32), ("precision", c_int32), ("gain_mode", c_int32),
        ("nx", c_int32), ("ny", c_int32), ("ratio", c_int32),
        ("n_members", c_int32), ("n_probes", c_int32),
        ("length", c_double), ("dt", c_double), ("nu", c_double),
        ("gamma", c_double), ("mach", c_double), ("reynolds", c_double), ("prandtl", c_double),
        ("obs_sigma", c_double),
        ("anomaly_terms", c_int32),
        ("u0", c_double), ("omega", c_double),
        ("theta_sigma", c_double * 2),
        ("filter_sigma", c_double),
        ("time_scheme", c_int32),
    ]


class MenkfNet(ctypes.Structure):
    _fields_ = [
        ("wpacked", c_void_p), ("params", c_void_p),
        ("in_scale", ctypes.c_float * 8), ("in_offset", ctypes.c_float * 8),
        ("out_scale", ctypes.c_float * 4),
        ("guard", ctypes.c_float),
        ("fallback_count_dev", c_void_p),
        ("judge_every", c_int32), ("judge_tol", ctypes.c_float),
        ("judge_dev", c_void_p),
    ]


class MenkfNetTrain(ctypes.Structure):
    _fields_ = [
        ("params", c_void_p), ("grad", c_void_p), ("adam_m", c_void_p), ("adam_v", c_void_p),
        ("wpacked", c_void_p),
        ("dproj", c_void_p), ("xf", c_void_p), ("target", c_void_p),
        ("npairs", c_int32), ("H", c_int32), ("W", c_int32),
        ("crops_dev", c_void_p),
        ("batch", c_int32), ("crop", c_int32),
        ("in_scale", ctypes.c_float * 8), ("in_offset", ctypes.c_float * 8),
        ("out_scale", ctypes.c_float * 4),
        ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
        ("step", c_int32), ("apply_adam", c_int32),
        ("loss_dev", c_void_p),
        ("workspace_dev", c_void_p),
        ("workspace_bytes", c_size_t),
    ]


class MenkfSchedule(ctypes.Structure):
    _fields_ = [("tile_x", c_int32), ("tile_y", c_int32), ("member_chunk", c_int32), ("reserved", c_int32)]


class MenkfCycleArgs(ctypes.Structure):
    _fields_ = [
        ("ctx", c_void_p),
        ("fine", c_void_p), ("fine_prev", c_void_p), ("members", c_void_p),
        ("xstar", c_void_p), ("deltac", c_void_p),
        ("yobs", c_void_p),
        ("seed", c_uint64), ("cycle", c_uint64),
        ("nsteps", c_int32), ("n_sweeps", c_int32),
        ("alpha", c_double),
        ("prolong_mode", c_int32),
        ("net", ctypes.POINTER(MenkfNet)),
        ("aux_stream", c_void_p),
        ("feedback", c_int32),
        ("pipelined", c_int32),
    ]


class MenkfDualArgs(ctypes.Structure):
    _fields_ = [
        ("ctx", c_void_p),
        ("fine", c_void_p), ("fine_prev", c_void_p), ("members", c_void_p),
        ("xstar", c_void_p), ("deltac", c_void_p),
        ("yobs", c_void_p),
        ("theta", c_void_p), ("theta_mean", c_void_p), ("clock", c_void_p),
        ("seed", c_uint64), ("cycle", c_uint64),
        ("nsteps", c_int32), ("n_sweeps", c_int32),
        ("alpha", c_double),
        ("aux_stream", c_void_p),
    ]


NET_NPARAM = 12740
NET_NPACKED = 20736


# name -> (restype, argtypes)
SIGNATURES = {
    "menkf_create": (c_int32, [ctypes.POINTER(MenkfConfig), ctypes.POINTER(c_void_p)]),
    "menkf_destroy": (None, [c_void_p]),
    "menkf_last_error": (c_char_p, [c_void_p]),
    "menkf_workspace_size": (c_int32, [c_void_p, ctypes.POINTER(c_size_t)]),
    "menkf_set_workspace": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "menkf_set_probes": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "menkf_set_observations": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "menkf_forecast": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "menkf_set_schedule": (c_int32, [c_void_p, c_int32, ctypes.POINTER(MenkfSchedule)]),
    "menkf_get_schedule": (c_int32, [c_void_p, c_int32, ctypes.POINTER(MenkfSchedule)]),
    "menkf_autotune": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_int32, c_int32,
                                 ctypes.POINTER(MenkfSchedule), ctypes.POINTER(ctypes.c_float), c_void_p]),
    "menkf_restrict": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "menkf_gain": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_uint64, c_uint64, c_void_p, c_void_p]),
    "menkf_get_gain": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "menkf_set_cycle": (c_int32, [c_void_p, c_uint64, c_void_p]),
    "menkf_update": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "menkf_prolong_smooth": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_double, c_int32,
                                       ctypes.POINTER(MenkfNet), c_void_p]),
    "menkf_get_status": (c_int32, [c_void_p, ctypes.POINTER(c_int32), c_int32, c_void_p]),
    "menkf_recentre": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "menkf_net_pack": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "menkf_net_train_workspace_size": (c_int32, [c_int32, c_int32, ctypes.POINTER(c_size_t)]),
    "menkf_net_train_step": (c_int32, [ctypes.POINTER(MenkfNetTrain), c_void_p]),
    "menkf_net_forward": (c_int32, [ctypes.POINTER(MenkfNetTrain), c_void_p]),
    "menkf_net_backward": (c_int32, [ctypes.POINTER(MenkfNetTrain), c_void_p]),
    "menkf_net_adam": (c_int32, [ctypes.POINTER(MenkfNetTrain), c_void_p]),
    "menkf_observe": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_void_p]),
    "menkf_diagnostics": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "menkf_residual": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "menkf_spread": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "menkf_diagnostics_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "menkf_ram_ratio": (c_double, [c_int32, c_int32, c_int32]),
    "menkf_cycle": (c_int32, [ctypes.POINTER(MenkfCycleArgs), c_void_p]),
    "menkf_cycle_flush": (c_int32, [ctypes.POINTER(MenkfCycleArgs), c_void_p]),
    "menkf_batch_create": (c_int32, [c_int32, ctypes.POINTER(c_void_p)]),
    "menkf_batch_destroy": (None, [c_void_p]),
    "menkf_batch_cycle": (c_int32, [c_void_p, ctypes.POINTER(MenkfCycleArgs), c_int32, c_void_p]),
    "menkf_batch_lanes": (c_int32, [c_void_p, ctypes.POINTER(c_int32), c_int32]),
    "menkf_forecast_inlet": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                       c_void_p]),
    "menkf_param_perturb": (c_int32, [c_void_p, c_void_p, c_void_p, c_uint64, c_uint64, c_void_p]),
    "menkf_param_update": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "menkf_dual_cycle": (c_int32, [ctypes.POINTER(MenkfDualArgs), c_void_p]),
    "menkf_graph_begin": (c_int32, [c_void_p]),
    "menkf_graph_end": (c_int32, [c_void_p, ctypes.POINTER(c_void_p)]),
    "menkf_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "menkf_graph_destroy": (None, [c_void_p]),
}

TEST_HOOKS = {
    "menkf_test_philox": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p]),
    "menkf_test_mfma": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "menkf_test_chol_diag": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
}

_LIB = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmenkf.so and declare every entry point; raises if it is not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(
            f"libmenkf.so not found at {path}: build it with `python -m paper_2012_10091_amd.build` "
            "(hipcc, gfx950). There is no fallback implementation.")
    lib = ctypes.CDLL(path)
    for name, (res, args) in {**SIGNATURES, **TEST_HOOKS}.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
