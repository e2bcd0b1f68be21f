"""Thin Python binding of libmenkf (argument marshalling only).

Every method maps one-to-one onto a ``menkf_*`` C entry point of
include/menkf.h; torch tensors supply device memory and the current HIP
stream.  No computation of the method happens here.
"""

from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib

MENKF_BURGERS1D = 1
MENKF_NS2D = 2
MENKF_BURGERS1D_INLET = 3
MENKF_EULER1D_INLET = 4
MENKF_F32 = 0
MENKF_F64 = 1
MENKF_GAIN_EXACT_R = 0
MENKF_GAIN_SAMPLE_EE = 1
MENKF_GAIN_ENSEMBLE_SPACE = 2
MENKF_FINE = 0
MENKF_COARSE = 1
MENKF_PROLONG_PLAIN = 0
MENKF_PROLONG_LEARNED = 1
MENKF_PROLONG_LEARNED_FALLBACK = 2
MENKF_TIME_SSPRK3 = 0
MENKF_TIME_FIRST_ORDER = 1
MENKF_CYCLE_DEVICE = (1 << 64) - 1

STATUS = {0: "MENKF_OK", -1: "MENKF_E_ARG", -2: "MENKF_E_SHAPE", -3: "MENKF_E_NOT_SPD",
          -4: "MENKF_E_NONFINITE", -5: "MENKF_E_HIP", -6: "MENKF_E_UNSUPPORTED", -7: "MENKF_E_WORKSPACE"}


class MenkfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_config(model, nx, ny, ratio, n_members, n_probes, dt, precision=MENKF_F32,
                gain_mode=MENKF_GAIN_EXACT_R, length=6.283185307179586, nu=0.0, gamma=1.4,
                mach=0.3, reynolds=1000.0, prandtl=0.71, obs_sigma=0.01, anomaly_terms=0, u0=1.0, omega=0.0,
                theta_sigma=(0.0, 0.0), filter_sigma=0.0, time_scheme=0) -> _lib.MenkfConfig:
    return _lib.MenkfConfig(model, precision, gain_mode, nx, ny, ratio, n_members, n_probes,
                            length, dt, nu, gamma, mach, reynolds, prandtl, obs_sigma, anomaly_terms,
                            u0, omega, (ctypes.c_double * 2)(*theta_sigma), filter_sigma, time_scheme)


def config_from(cfg) -> _lib.MenkfConfig:
    """menkf_config from any object with the workload attributes (dim, nx, ny, ...)."""
    if cfg.dim == 2:
        model = MENKF_NS2D
    else:
        if getattr(cfg, "bc", "periodic") != "inlet":
            model = MENKF_BURGERS1D
        else:
            model = MENKF_EULER1D_INLET if getattr(cfg, "eq", "burgers") == "euler" else MENKF_BURGERS1D_INLET
    return make_config(
        model, cfg.nx, cfg.ny, cfg.ratio, cfg.n_members,
        cfg.n_probes, cfg.dt, precision=MENKF_F64 if cfg.precision == "f64" else MENKF_F32,
        gain_mode=getattr(cfg, "gain_mode", MENKF_GAIN_EXACT_R), length=cfg.length, nu=cfg.nu,
        gamma=cfg.gamma, mach=cfg.mach, reynolds=cfg.reynolds, prandtl=cfg.prandtl,
        obs_sigma=cfg.obs_sigma, anomaly_terms=getattr(cfg, "anomaly_terms", 0),
        u0=getattr(cfg, "u0", 1.0), omega=getattr(cfg, "omega", 0.0),
        theta_sigma=tuple(getattr(cfg, "theta_walk", (0.0, 0.0))), filter_sigma=getattr(cfg, "filter_sigma", 0.0),
        time_scheme=MENKF_TIME_FIRST_ORDER if getattr(cfg, "time_scheme", "ssprk3") == "first_order"
        else MENKF_TIME_SSPRK3)


def ram_ratio(dim: int, ratio: int, n_members: int) -> float:
    return _lib.load().menkf_ram_ratio(dim, ratio, n_members)


def last_error(ctx=None) -> str:
    s = _lib.load().menkf_last_error(ctx)
    return s.decode() if s else ""


class Context:
    """One assimilation instance: a menkf_ctx plus its torch-owned workspace."""

    def __init__(self, cfg, device: str = "cuda", allocate: bool = True):
        self.lib = _lib.load()
        self.c_cfg = cfg if isinstance(cfg, _lib.MenkfConfig) else config_from(cfg)
        h = ctypes.c_void_p()
        st = self.lib.menkf_create(ctypes.byref(self.c_cfg), ctypes.byref(h))
        if st != 0:
            raise MenkfError(st, last_error(None))
        self.handle = h
        c = self.c_cfg
        self.dim = 2 if c.model == MENKF_NS2D else 1
        self.F = 4 if self.dim == 2 else (3 if c.model == MENKF_EULER1D_INLET else 1)
        self.dtype = torch.float64 if c.precision == MENKF_F64 else torch.float32
        self.nx, self.ny, self.ratio = c.nx, c.ny, c.ratio
        self.nxc = c.nx // c.ratio
        self.nyc = c.ny // c.ratio if self.dim == 2 else 1
        self.N, self.Ny = c.n_members, c.n_probes
        self.device = device
        self.workspace = None
        self._probes = None
        if allocate:
            self.allocate()

    # ------------------------------------------------------------ helpers
    def _check(self, st):
        if st != 0:
            raise MenkfError(st, last_error(self.handle))

    @property
    def fine_shape(self):
        return (self.F, self.nx) if self.dim == 1 else (self.F, self.ny, self.nx)

    @property
    def coarse_shape(self):
        return (self.F, self.nxc) if self.dim == 1 else (self.F, self.nyc, self.nxc)

    def _state(self, t, shape, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA tensor")
        if t.dtype != self.dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous {self.dtype}")
        if tuple(t.shape[-len(shape):]) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected (..., {shape})")
        return t

    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        self._check(self.lib.menkf_workspace_size(self.handle, ctypes.byref(n)))
        return n.value

    def allocate(self):
        nbytes = self.workspace_size()
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._check(self.lib.menkf_set_workspace(self.handle, _ptr(self.workspace), nbytes))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.menkf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ entry points
    def set_probes(self, idx: torch.Tensor, comp: torch.Tensor):
        for t in (idx, comp):
            if t.dtype != torch.int32 or not t.is_cuda or t.numel() != self.Ny:
                raise ValueError("probe tables must be CUDA int32 tensors of n_probes entries")
        self._probes = (idx.contiguous(), comp.contiguous())
        self._check(self.lib.menkf_set_probes(self.handle, _ptr(self._probes[0]), _ptr(self._probes[1])))

    def set_observations(self, idx: torch.Tensor, comp: torch.Tensor):
        """menkf_set_observations: the same call as set_probes."""
        for t in (idx, comp):
            if t.dtype != torch.int32 or not t.is_cuda or t.numel() != self.Ny:
                raise ValueError("probe tables must be CUDA int32 tensors of n_probes entries")
        self._probes = (idx.contiguous(), comp.contiguous())
        self._check(self.lib.menkf_set_observations(self.handle, _ptr(self._probes[0]), _ptr(self._probes[1])))

    def forecast(self, level: int, state: torch.Tensor, nsteps: int, prev: Optional[torch.Tensor] = None,
                 stream=None):
        shape = self.fine_shape if level == MENKF_FINE else self.coarse_shape
        self._state(state, shape, "state")
        nb = 1 if state.dim() == len(shape) else state.shape[0]
        if prev is not None:
            self._state(prev, shape, "prev")
            if prev.numel() != state.numel():
                raise ValueError("prev must match state")
        self._check(self.lib.menkf_forecast(self.handle, level, _ptr(state), nb, nsteps, _ptr(prev),
                                            _stream(stream)))

    # ------------------------------------------------------------ dual filter (inlet-forced model)
    def _theta(self, t, rows, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA float64 tensor")
        if t.numel() != 2 * rows:
            raise ValueError(f"{name} must hold {rows} x 2 doubles")
        return t

    def forecast_inlet(self, level: int, state: torch.Tensor, nsteps: int, theta: torch.Tensor, t0: torch.Tensor,
                       prev: Optional[torch.Tensor] = None, stream=None):
        shape = self.fine_shape if level == MENKF_FINE else self.coarse_shape
        self._state(state, shape, "state")
        nb = 1 if state.dim() == len(shape) else state.shape[0]
        self._theta(theta, nb, "theta")
        if t0.dtype != torch.float64 or t0.numel() != 1 or not t0.is_cuda:
            raise ValueError("t0 must be one CUDA float64")
        if prev is not None:
            self._state(prev, shape, "prev")
            if prev.numel() != state.numel():
                raise ValueError("prev must match state")
        self._check(self.lib.menkf_forecast_inlet(self.handle, level, _ptr(state), nb, nsteps, _ptr(prev),
                                                  _ptr(theta), _ptr(t0), _stream(stream)))

    def param_perturb(self, theta: torch.Tensor, theta_f: torch.Tensor, seed: int, cycle: int, stream=None):
        self._theta(theta, self.N, "theta")
        self._theta(theta_f, self.N, "theta_f")
        self._check(self.lib.menkf_param_perturb(self.handle, _ptr(theta), _ptr(theta_f), seed, cycle,
                                                 _stream(stream)))

    def param_update(self, theta_f: torch.Tensor, theta_a: torch.Tensor, theta_mean: torch.Tensor, stream=None):
        self._theta(theta_f, self.N, "theta_f")
        self._theta(theta_a, self.N, "theta_a")
        self._theta(theta_mean, 1, "theta_mean")
        self._check(self.lib.menkf_param_update(self.handle, _ptr(theta_f), _ptr(theta_a), _ptr(theta_mean),
                                                _stream(stream)))

    def dual_args(self, fine, fine_prev, members, xstar, deltac, yobs, theta, theta_mean, clock, seed: int,
                  cycle: int, nsteps: int, n_sweeps: int = 1, alpha: float = 0.5, aux_stream=None):
        """The menkf_dual_args of one dual cycle of this instance (buffers checked here)."""
        self._state(fine, self.fine_shape, "fine")
        self._state(fine_prev, self.fine_shape, "fine_prev")
        self._state(members, self.coarse_shape, "members")
        if members.shape[0] != self.N:
            raise ValueError("members must hold n_members states")
        self._state(xstar, self.coarse_shape, "xstar")
        self._state(deltac, self.coarse_shape, "deltac")
        if yobs.dtype != torch.float64 or yobs.numel() != self.Ny or not yobs.is_cuda:
            raise ValueError("yobs must be a CUDA float64 tensor of n_probes entries")
        self._theta(theta, self.N, "theta")
        self._theta(theta_mean, 1, "theta_mean")
        if clock.dtype != torch.float64 or clock.numel() != 1 or not clock.is_cuda:
            raise ValueError("clock must be one CUDA float64")
        a = _lib.MenkfDualArgs()
        a.ctx = self.handle
        a.fine, a.fine_prev, a.members = _ptr(fine), _ptr(fine_prev), _ptr(members)
        a.xstar, a.deltac, a.yobs = _ptr(xstar), _ptr(deltac), _ptr(yobs)
        a.theta, a.theta_mean, a.clock = _ptr(theta), _ptr(theta_mean), _ptr(clock)
        a.seed, a.cycle = seed, cycle
        a.nsteps, a.n_sweeps, a.alpha = nsteps, n_sweeps, alpha
        if aux_stream is not None:
            a.aux_stream = aux_stream.cuda_stream
        return a

    def dual_cycle(self, fine, fine_prev, members, xstar, deltac, yobs, theta, theta_mean, clock, seed: int,
                   cycle: int, nsteps: int, n_sweeps: int = 1, alpha: float = 0.5, stream=None, aux_stream=None):
        a = self.dual_args(fine, fine_prev, members, xstar, deltac, yobs, theta, theta_mean, clock, seed, cycle,
                           nsteps, n_sweeps, alpha, aux_stream)
        self._check(self.lib.menkf_dual_cycle(ctypes.byref(a), _stream(stream)))

    def set_schedule(self, level: int, tile=(0, 0), member_chunk: int = 0):
        sc = _lib.MenkfSchedule(int(tile[0]), int(tile[1]), int(member_chunk), 0)
        self._check(self.lib.menkf_set_schedule(self.handle, level, ctypes.byref(sc)))

    def get_schedule(self, level: int) -> dict:
        sc = _lib.MenkfSchedule()
        self._check(self.lib.menkf_get_schedule(self.handle, level, ctypes.byref(sc)))
        return {"tile": (sc.tile_x, sc.tile_y), "member_chunk": sc.member_chunk}

    def autotune(self, level: int, scratch: torch.Tensor, nsteps: int, reps: int = 2, stream=None) -> dict:
        """Time every forecast schedule of `level` on `scratch` (overwritten) and keep the fastest."""
        shape = self.fine_shape if level == MENKF_FINE else self.coarse_shape
        self._state(scratch, shape, "scratch")
        nb = 1 if scratch.dim() == len(shape) else scratch.shape[0]
        sc = _lib.MenkfSchedule()
        ms = ctypes.c_float()
        self._check(self.lib.menkf_autotune(self.handle, level, _ptr(scratch), nb, nsteps, reps, ctypes.byref(sc),
                                            ctypes.byref(ms), _stream(stream)))
        return {"tile": (sc.tile_x, sc.tile_y), "member_chunk": sc.member_chunk, "ms": ms.value}

    def restrict(self, xf: torch.Tensor, xc: torch.Tensor, stream=None):
        self._state(xf, self.fine_shape, "xf")
        self._state(xc, self.coarse_shape, "xc")
        self._check(self.lib.menkf_restrict(self.handle, _ptr(xf), _ptr(xc), _stream(stream)))

    def gain(self, members: torch.Tensor, xstar: torch.Tensor, yobs: torch.Tensor, seed: int, cycle: int,
             eps: Optional[torch.Tensor] = None, stream=None):
        self._state(members, self.coarse_shape, "members")
        if members.shape[0] != self.N:
            raise ValueError("members must hold n_members states")
        self._state(xstar, self.coarse_shape, "xstar")
        if yobs.dtype != torch.float64 or yobs.numel() != self.Ny or not yobs.is_cuda:
            raise ValueError("yobs must be a CUDA float64 tensor of n_probes entries")
        if eps is not None and (eps.dtype != torch.float64 or eps.numel() != self.N * self.Ny
                                or not eps.is_contiguous()):
            raise ValueError("eps must be contiguous float64 (n_members, n_probes)")
        self._check(self.lib.menkf_gain(self.handle, _ptr(members), _ptr(xstar), _ptr(yobs), seed, cycle,
                                        _ptr(eps), _stream(stream)))

    def set_cycle(self, cycle: int, stream=None):
        self._check(self.lib.menkf_set_cycle(self.handle, cycle, _stream(stream)))

    def get_gain(self, stream=None) -> torch.Tensor:
        z = torch.empty((self.N + 1, self.N), dtype=torch.float64, device=self.device)
        self._check(self.lib.menkf_get_gain(self.handle, _ptr(z), _stream(stream)))
        return z

    def update(self, members: torch.Tensor, deltac: torch.Tensor, stream=None):
        self._state(members, self.coarse_shape, "members")
        self._state(deltac, self.coarse_shape, "deltac")
        self._check(self.lib.menkf_update(self.handle, _ptr(members), _ptr(deltac), _stream(stream)))

    def prolong_smooth(self, deltac: torch.Tensor, xf: torch.Tensor, xprev: Optional[torch.Tensor],
                       n_sweeps: int = 1, alpha: float = 0.5, mode: int = MENKF_PROLONG_PLAIN,
                       net=None, stream=None):
        self._state(deltac, self.coarse_shape, "deltac")
        self._state(xf, self.fine_shape, "xf")
        if xprev is not None:
            self._state(xprev, self.fine_shape, "xprev")
        if net is None:
            netp = None
        elif isinstance(net, _lib.MenkfNet):
            netp = ctypes.byref(net)
        else:
            netp = ctypes.byref(net.c_struct())
        self._check(self.lib.menkf_prolong_smooth(self.handle, _ptr(deltac), _ptr(xf), _ptr(xprev), n_sweeps,
                                                  alpha, mode, netp, _stream(stream)))

    def cycle_args(self, fine, fine_prev, members, xstar, deltac, yobs, seed: int, cycle: int, nsteps: int,
                   n_sweeps: int = 1, alpha: float = 0.5, mode: int = MENKF_PROLONG_PLAIN, net=None,
                   aux_stream=None, feedback: bool = False, pipelined: bool = False):
        """The menkf_cycle_args of one cycle of this instance (buffers checked here)."""
        self._state(fine, self.fine_shape, "fine")
        self._state(fine_prev, self.fine_shape, "fine_prev")
        self._state(members, self.coarse_shape, "members")
        if members.shape[0] != self.N:
            raise ValueError("members must hold n_members states")
        self._state(xstar, self.coarse_shape, "xstar")
        self._state(deltac, self.coarse_shape, "deltac")
        if yobs.dtype != torch.float64 or yobs.numel() != self.Ny or not yobs.is_cuda:
            raise ValueError("yobs must be a CUDA float64 tensor of n_probes entries")
        a = _lib.MenkfCycleArgs()
        a.ctx = self.handle
        a.fine, a.fine_prev, a.members = _ptr(fine), _ptr(fine_prev), _ptr(members)
        a.xstar, a.deltac, a.yobs = _ptr(xstar), _ptr(deltac), _ptr(yobs)
        a.seed, a.cycle = seed, cycle
        a.nsteps, a.n_sweeps, a.alpha, a.prolong_mode = nsteps, n_sweeps, alpha, mode
        if net is not None:
            ns = net if isinstance(net, _lib.MenkfNet) else net.c_struct()
            a.net = ctypes.pointer(ns)
            a._keep = ns
        if aux_stream is not None:
            a.aux_stream = aux_stream.cuda_stream
        a.feedback = 1 if feedback else 0
        a.pipelined = 1 if pipelined else 0
        return a

    def cycle(self, fine, fine_prev, members, xstar, deltac, yobs, seed: int, cycle: int, nsteps: int,
              n_sweeps: int = 1, alpha: float = 0.5, mode: int = MENKF_PROLONG_PLAIN, net=None, stream=None,
              aux_stream=None, feedback: bool = False, pipelined: bool = False):
        a = self.cycle_args(fine, fine_prev, members, xstar, deltac, yobs, seed, cycle, nsteps, n_sweeps, alpha,
                            mode, net, aux_stream, feedback, pipelined)
        self._check(self.lib.menkf_cycle(ctypes.byref(a), _stream(stream)))

    def cycle_flush(self, fine, fine_prev, deltac, n_sweeps: int = 1, alpha: float = 0.5,
                    mode: int = MENKF_PROLONG_PLAIN, net=None, stream=None):
        """menkf_cycle_flush: the correction a pipelined cycle left pending."""
        self._state(fine, self.fine_shape, "fine")
        self._state(fine_prev, self.fine_shape, "fine_prev")
        self._state(deltac, self.coarse_shape, "deltac")
        a = _lib.MenkfCycleArgs()
        a.ctx = self.handle
        a.fine, a.fine_prev, a.deltac = _ptr(fine), _ptr(fine_prev), _ptr(deltac)
        a.n_sweeps, a.alpha, a.prolong_mode = n_sweeps, alpha, mode
        if net is not None:
            ns = net if isinstance(net, _lib.MenkfNet) else net.c_struct()
            a.net = ctypes.pointer(ns)
            a._keep = ns
        self._check(self.lib.menkf_cycle_flush(ctypes.byref(a), _stream(stream)))

    def recentre(self, members: torch.Tensor, xf: torch.Tensor, stream=None):
        self._state(members, self.coarse_shape, "members")
        if members.shape[0] != self.N:
            raise ValueError("members must hold n_members states")
        self._state(xf, self.fine_shape, "xf")
        self._check(self.lib.menkf_recentre(self.handle, _ptr(members), _ptr(xf), _stream(stream)))

    def get_status(self, clear: bool = True, stream=None) -> int:
        info = ctypes.c_int32()
        st = self.lib.menkf_get_status(self.handle, ctypes.byref(info), int(clear), _stream(stream))
        if st not in (0, -3):
            self._check(st)
        return info.value

    def observe(self, level: int, state: torch.Tensor, stream=None) -> torch.Tensor:
        shape = self.fine_shape if level == MENKF_FINE else self.coarse_shape
        self._state(state, shape, "state")
        nb = 1 if state.dim() == len(shape) else state.shape[0]
        y = torch.empty((nb, self.Ny), dtype=torch.float64, device=self.device)
        self._check(self.lib.menkf_observe(self.handle, level, _ptr(state), nb, _ptr(y), _stream(stream)))
        return y

    def residual(self, x: torch.Tensor, xprev: torch.Tensor, out: Optional[torch.Tensor] = None,
                 stream=None) -> torch.Tensor:
        self._state(x, self.fine_shape, "x")
        self._state(xprev, self.fine_shape, "xprev")
        if out is None:
            out = torch.empty_like(x)
        self._check(self.lib.menkf_residual(self.handle, _ptr(x), _ptr(xprev), _ptr(out), _stream(stream)))
        return out

    def diagnostics(self, xa: torch.Tensor, xt: torch.Tensor, out: Optional[torch.Tensor] = None,
                    stream=None) -> torch.Tensor:
        self._state(xa, self.fine_shape, "xa")
        self._state(xt, self.fine_shape, "xt")
        if out is None:
            out = torch.empty(3, dtype=torch.float64, device=self.device)
        self._check(self.lib.menkf_diagnostics(self.handle, _ptr(xa), _ptr(xt), _ptr(out), _stream(stream)))
        return out

    def spread(self, members: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """menkf_spread: (trace of the ensemble covariance, sum of the squared
        mean, non-finite count) of the observed quantity of nb coarse states."""
        self._state(members, self.coarse_shape, "members")
        if members.dim() != len(self.coarse_shape) + 1:
            raise ValueError("members must be a batch of coarse states")
        if out is None:
            out = torch.empty(3, dtype=torch.float64, device=self.device)
        self._check(self.lib.menkf_spread(self.handle, _ptr(members), members.shape[0], _ptr(out), _stream(stream)))
        return out


class Graph:
    """A captured sequence of menkf_* calls (menkf_graph_* entry points)."""

    def __init__(self, handle):
        self.lib = _lib.load()
        self.handle = handle

    @staticmethod
    def begin(stream):
        lib = _lib.load()
        st = lib.menkf_graph_begin(_stream(stream))
        if st != 0:
            raise MenkfError(st, last_error(None))

    @staticmethod
    def end(stream) -> "Graph":
        lib = _lib.load()
        h = ctypes.c_void_p()
        st = lib.menkf_graph_end(_stream(stream), ctypes.byref(h))
        if st != 0:
            raise MenkfError(st, last_error(None))
        return Graph(h)

    def launch(self, stream=None):
        st = self.lib.menkf_graph_launch(self.handle, _stream(stream))
        if st != 0:
            raise MenkfError(st, last_error(None))

    def __del__(self):
        try:
            if self.handle:
                self.lib.menkf_graph_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


class Batch:
    """Independent instances advanced together on n_lanes streams (menkf_batch_*)."""

    def __init__(self, n_lanes: int = 4):
        self.lib = _lib.load()
        h = ctypes.c_void_p()
        st = self.lib.menkf_batch_create(n_lanes, ctypes.byref(h))
        if st != 0:
            raise MenkfError(st, last_error(None))
        self.handle = h
        self.n_lanes = n_lanes
        self._n = 0

    def cycle(self, args, stream=None):
        """Issue one cycle of every instance; args is a list of Context.cycle_args()."""
        arr = (_lib.MenkfCycleArgs * len(args))(*args)
        self._arr = (arr, list(args))
        st = self.lib.menkf_batch_cycle(self.handle, arr, len(args), _stream(stream))
        if st != 0:
            raise MenkfError(st, last_error(None))
        self._n = len(args)

    def lanes(self):
        out = (ctypes.c_int32 * self._n)()
        st = self.lib.menkf_batch_lanes(self.handle, out, self._n)
        if st != 0:
            raise MenkfError(st, last_error(None))
        return list(out)

    def __del__(self):
        try:
            if self.handle:
                self.lib.menkf_batch_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


# ------------------------------------------------------------------ learned prolongation
P_OFFSETS = {"w1": (0, (32, 8, 3, 3)), "b1": (2304, (32,)), "w2": (2336, (32, 32, 3, 3)),
             "b2": (11552, (32,)), "w3": (11584, (4, 32, 3, 3)), "b3": (12736, (4,))}


def pack_params(tensors) -> "torch.Tensor":
    """Flat FP32 parameter vector from (w1, b1, w2, b2, w3, b3) in PyTorch conv order."""
    flat = torch.cat([torch.as_tensor(t, dtype=torch.float32).reshape(-1) for t in tensors])
    if flat.numel() != _lib.NET_NPARAM:
        raise ValueError(f"expected {_lib.NET_NPARAM} parameters, got {flat.numel()}")
    return flat


def unpack_params(flat):
    flat = torch.as_tensor(flat).reshape(-1)
    return [flat[o:o + int(torch.tensor(sh).prod())].reshape(sh) for o, sh in P_OFFSETS.values()]


class Net:
    """Device parameters of the learned prolongation (menkf_net / menkf_net_pack)."""

    def __init__(self, params, in_scale, in_offset, out_scale, guard=10.0, device="cuda", judge_every=0,
                 judge_tol=1.0):
        self.lib = _lib.load()
        self.params = torch.as_tensor(params, dtype=torch.float32).reshape(-1).to(device).contiguous()
        if self.params.numel() != _lib.NET_NPARAM:
            raise ValueError("bad parameter count")
        self.wpacked = torch.empty(_lib.NET_NPACKED, dtype=torch.bfloat16, device=device)
        self.in_scale = [float(v) for v in in_scale]
        self.in_offset = [float(v) for v in in_offset]
        self.out_scale = [float(v) for v in out_scale]
        self.guard = float(guard)
        self.fallback_count = torch.zeros(1, dtype=torch.int32, device=device)
        self.judge_every = int(judge_every)
        self.judge_tol = float(judge_tol)
        # [last judged distance, judged calls, calls on the plain correction, calls with a guarded tile]
        self.judge_stats = torch.zeros(4, dtype=torch.float64, device=device)
        self.repack()

    def repack(self, stream=None):
        st = self.lib.menkf_net_pack(_ptr(self.params), _ptr(self.wpacked), _stream(stream))
        if st != 0:
            raise MenkfError(st, last_error(None))

    def c_struct(self) -> _lib.MenkfNet:
        n = _lib.MenkfNet()
        n.wpacked = self.wpacked.data_ptr()
        n.params = self.params.data_ptr()
        for i in range(8):
            n.in_scale[i] = self.in_scale[i]
            n.in_offset[i] = self.in_offset[i]
        for i in range(4):
            n.out_scale[i] = self.out_scale[i]
        n.guard = self.guard
        n.fallback_count_dev = self.fallback_count.data_ptr()
        n.judge_every = self.judge_every
        n.judge_tol = self.judge_tol
        n.judge_dev = self.judge_stats.data_ptr()
        self._c = n
        return n


class Trainer:
    """Adam training of a Net on periodic crops (menkf_net_train_step)."""

    def __init__(self, net: Net, batch: int, crop: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lib = _lib.load()
        self.net = net
        dev = net.params.device
        self.grad = torch.zeros_like(net.params)
        self.m = torch.zeros_like(net.params)
        self.v = torch.zeros_like(net.params)
        self.batch, self.crop = batch, crop
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        self.step_count = 0
        n = ctypes.c_size_t()
        st = self.lib.menkf_net_train_workspace_size(batch, crop, ctypes.byref(n))
        if st != 0:
            raise MenkfError(st, last_error(None))
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)

    def _desc(self, dproj, xf, target, crops, apply_adam):
        for t in (dproj, xf, target):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 4:
                raise ValueError("fields must be contiguous float32 CUDA (npairs, 4, H, W)")
        if crops.dtype != torch.int32 or tuple(crops.shape) != (self.batch, 3) or not crops.is_cuda:
            raise ValueError("crops must be int32 CUDA (batch, 3)")
        d = _lib.MenkfNetTrain()
        d.params, d.grad = self.net.params.data_ptr(), self.grad.data_ptr()
        d.adam_m, d.adam_v = self.m.data_ptr(), self.v.data_ptr()
        d.wpacked = self.net.wpacked.data_ptr()
        d.dproj, d.xf, d.target = dproj.data_ptr(), xf.data_ptr(), target.data_ptr()
        d.npairs, d.H, d.W = dproj.shape[0], dproj.shape[2], dproj.shape[3]
        d.crops_dev = crops.data_ptr()
        d.batch, d.crop = self.batch, self.crop
        for i in range(8):
            d.in_scale[i] = self.net.in_scale[i]
            d.in_offset[i] = self.net.in_offset[i]
        for i in range(4):
            d.out_scale[i] = self.net.out_scale[i]
        d.lr, d.beta1, d.beta2, d.eps = self.lr, self.beta1, self.beta2, self.eps
        d.step, d.apply_adam = max(self.step_count, 1), int(apply_adam)
        d.loss_dev = self.loss.data_ptr()
        d.workspace_dev = self.workspace.data_ptr()
        d.workspace_bytes = self.workspace.numel()
        return d

    def _call(self, fn, d, stream):
        st = fn(ctypes.byref(d), _stream(stream))
        if st != 0:
            raise MenkfError(st, last_error(None))

    def step(self, dproj, xf, target, crops, apply_adam=True, stream=None):
        """dproj, xf, target: (npairs, 4, H, W) float32 CUDA; crops: (batch, 3) int32 CUDA."""
        if apply_adam:
            self.step_count += 1
        d = self._desc(dproj, xf, target, crops, apply_adam)
        self._call(self.lib.menkf_net_train_step, d, stream)
        return self.loss

    def forward(self, dproj, xf, target, crops, stream=None):
        """menkf_net_forward: activations and the batch loss (returned tensor)."""
        self._call(self.lib.menkf_net_forward, self._desc(dproj, xf, target, crops, False), stream)
        return self.loss

    def backward(self, dproj, xf, target, crops, stream=None):
        """menkf_net_backward: the parameter gradient (self.grad) from the last forward."""
        self._call(self.lib.menkf_net_backward, self._desc(dproj, xf, target, crops, False), stream)
        return self.grad

    def adam(self, dproj, xf, target, crops, stream=None):
        """menkf_net_adam: one Adam update of the parameters from self.grad."""
        self.step_count += 1
        self._call(self.lib.menkf_net_adam, self._desc(dproj, xf, target, crops, True), stream)

