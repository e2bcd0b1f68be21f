#!/usr/bin/env python3
"""Throughput of the MEnKF hot path on one MI355X.

Workload: 2D compressible Navier-Stokes, fine 1024^2, coarse 256^2, 64
members, 4096 velocity probes, an analysis every 20 RK4 steps (dt 5e-4).
One step of this bench = one assimilation cycle: fine forecast (20 steps),
ensemble forecast (64 members x 20 steps), restriction, gain (FP64
innovation covariance + Cholesky), member update, prolongation + 3 relaxed
sweeps (plain) or the learned prolongation.  The cycle is captured once as
a HIP graph and replayed; observations for every cycle are generated
beforehand (a truth run on the GPU) and sit in HBM.

Prints one JSON line (metric, value in cycles/s, roofline of the dominant
kernel measured with HIP events on its own stream, oracle CPU baseline).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "assimilation cycles/s, 2D 1024²/256² N=64, learned vs plain at equal RMSE"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--sweeps", type=int, default=3)
    ap.add_argument("--rmse-cycles", type=int, default=100)
    ap.add_argument("--judge-every", type=int, default=10,
                    help="the learned prolongation's judge: every n-th cycle the plain correction is formed and "
                         "compared (and replaces the network's above the tolerance)")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--weights", default=None)
    ap.add_argument("--small", action="store_true", help="tiny workload (functional check only)")
    ap.add_argument("--autotune", type=int, default=1, help="autotune the forecast schedules first")
    ap.add_argument("--pipelined", type=int, default=1,
                    help="time pipelined cycles (each cycle's fine-grid correction applied at the start of the next, "
                         "beside its factorisation); the ordinary cycles are timed beside them")
    ap.add_argument("--workload", default="ns2d_1024_256_n64",
                    choices=["ns2d_1024_256_n64", "ns2d_512_128_n32", "burgers1d_16384_4096_n256", "uneven48",
                             "inlet_dual", "euler_dual", "learned_train"],
                    help="ns2d_512_128_n32: the learned-prolongation workload (2D 512^2/128^2, N = 32); "
                         "burgers1d_16384_4096_n256: 1D Burgers at scale (plain MEnKF only); uneven48: the batch "
                         "of 48 uneven instances in one graph; inlet_dual: the dual (parameter + state) filter of "
                         "the inlet-forced Burgers case (none of these is the headline)")
    ap.add_argument("--dual-precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--time-scheme", default="ssprk3", choices=["ssprk3", "first_order"],
                    help="inlet_dual: SSP-RK3, or the paper's first-order scheme (forward Euler, one Jacobi "
                         "iteration of the implicit step at each analysis step)")
    ap.add_argument("--theta-walk", type=float, default=None,
                    help="standard deviation of the parameter random walk per analysis (default: the workload's)")
    ap.add_argument("--dual-study", action="store_true",
                    help="with --workload inlet_dual: the parameter estimate over the whole assimilation window "
                         "for coarsening ratios 1, 2, 4, 8, 16 instead of the timing")
    ap.add_argument("--lanes", type=int, default=4, help="streams of the uneven batch")
    ap.add_argument("--schedule", default=None,
                    help="fixed forecast schedules instead of autotuning, e.g. fine=64x8:0,coarse=32x8:32")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for hardware-counter runs: a 1 GiB device copy (calibration) and one eager cycle")
    return ap.parse_args()


def make_cfg(args):
    from synthetic import configs
    if args.small:
        return configs.tiny_2d(precision="f32")
    by_name = {c.name: c for c in configs.CONFIGS.values()}
    return by_name[args.workload]


def metric_for(cfg):
    if cfg.name == "ns2d_1024_256_n64":
        return METRIC
    if cfg.dim == 2:
        return f"assimilation cycles/s, 2D {cfg.nx}²/{cfg.nxc}² N={cfg.n_members}, learned vs plain at equal RMSE"
    return f"assimilation cycles/s, 1D Burgers {cfg.nx}/{cfg.nxc} N={cfg.n_members}, plain MEnKF"


class Cycle:
    """Device state of one assimilation instance and its captured cycle."""

    def __init__(self, cfg, n_sweeps, mode=0, net=None, pipelined=False):
        import torch

        import paper_2012_10091_amd as m
        from synthetic import fields
        self.m = m
        self.cfg = cfg
        self.ctx = m.Context(cfg)
        idx, comp = fields.probes_for(cfg)
        self.ctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.as_tensor(comp, device="cuda"))
        f32 = torch.float32
        self.fine = torch.as_tensor(fields.model_ic(cfg), dtype=f32, device="cuda").contiguous()
        self.members = torch.as_tensor(fields.member_ics(cfg), dtype=f32, device="cuda").contiguous()
        self.prev = torch.empty_like(self.fine)
        self.xs = torch.empty(cfg.coarse_shape, dtype=f32, device="cuda")
        self.dc = torch.empty_like(self.xs)
        self.y = torch.zeros(cfg.n_probes, dtype=torch.float64, device="cuda")
        self.n_sweeps = n_sweeps
        self.mode = mode
        self.net = net
        self.seed = cfg.seed + 5
        self.graph = None
        self.aux = torch.cuda.Stream()
        self.overlap = True
        self.pipelined = pipelined

    def autotune(self):
        """Pick the forecast schedules of both levels with the library's autotuner."""
        import torch
        self.tuned = {
            "fine": self.ctx.autotune(self.m.MENKF_FINE, self.fine.clone(), self.cfg.n_obs, reps=3),
            "coarse": self.ctx.autotune(self.m.MENKF_COARSE, self.members.clone(), self.cfg.n_obs, reps=3),
        }
        torch.cuda.synchronize()
        return self.tuned

    def issue(self, stream):
        """One cycle (menkf_cycle).  With overlap the fine forecast runs on a
        second stream beside the late block steps of the factorisation;
        pipelined cycles apply the previous cycle's fine-grid correction
        there too, ahead of the fine forecast (each replay still does one
        whole cycle of work)."""
        self.ctx.cycle(self.fine, self.prev, self.members, self.xs, self.dc, self.y, self.seed,
                       self.m.MENKF_CYCLE_DEVICE, self.cfg.n_obs, n_sweeps=self.n_sweeps, alpha=0.5, mode=self.mode,
                       net=self.net, stream=stream, aux_stream=self.aux if self.overlap else None,
                       pipelined=self.pipelined)

    def set_state(self, fine, members):
        self.fine.copy_(fine)
        self.members.copy_(members)

    def capture(self, stream):
        import torch
        with torch.cuda.stream(stream):
            self.m.Graph.begin(stream)
            self.issue(stream)
            self.graph = self.m.Graph.end(stream)
        self.ctx.set_cycle(1, stream=stream)


def truth_observations(cfg, n_cycles):
    """Truth run on the GPU (same fine model) and noisy probe observations."""
    import numpy as np
    import torch

    import paper_2012_10091_amd as m
    from synthetic import fields
    ctx = m.Context(cfg.with_(n_members=2))
    idx, comp = fields.probes_for(cfg)
    ctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.as_tensor(comp, device="cuda"))
    truth = torch.as_tensor(fields.truth_ic(cfg), dtype=torch.float32, device="cuda").contiguous()
    Y = torch.empty((n_cycles, cfg.n_probes), dtype=torch.float64, device="cuda")
    states = []
    for c in range(n_cycles):
        ctx.forecast(m.MENKF_FINE, truth, cfg.n_obs)
        Y[c] = ctx.observe(m.MENKF_FINE, truth)[0] + torch.as_tensor(fields.obs_noise(cfg, c + 1), device="cuda")
        states.append(truth.clone() if c % 10 == 9 else None)
    torch.cuda.synchronize()
    del np
    return Y, states


def time_cycles(cyc, Y, warmup, steps):
    import torch
    stream = torch.cuda.Stream()
    cyc.capture(stream)
    torch.cuda.synchronize()
    for c in range(warmup):
        with torch.cuda.stream(stream):
            cyc.y.copy_(Y[c])
        cyc.graph.launch(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for c in range(warmup, warmup + steps):
        with torch.cuda.stream(stream):
            cyc.y.copy_(Y[c])
        cyc.graph.launch(stream)
    ev1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / 1e3, wall


def rmse_comparison(cfg, net, n_cycles, n_sweeps, judge_every):
    """Plain (Pi_F + sweeps) and learned MEnKF runs from the same seeds
    against one truth.  The learned run is the timed path: the network with
    its per-tile guard in every cycle.  Every judge_every cycles the plain
    correction of the learned run's own analysis is formed on a scratch copy
    and the relative L2 distance of the two corrected states recorded (for
    information: the run is not switched).  A third run adds the
    fine-to-coarse feedback (members recentred on the fine analysis after
    every cycle) to the plain path."""
    import numpy as np
    import torch
    import paper_2012_10091_amd as m
    from synthetic import fields
    runs = {k: Cycle(cfg, n_sweeps,
                     mode=m.MENKF_PROLONG_LEARNED_FALLBACK if k == "learned" else m.MENKF_PROLONG_PLAIN,
                     net=net if k == "learned" else None)
            for k in ("plain", "learned", "plain_feedback")}
    net.judge_stats.zero_()
    ctx = runs["plain"].ctx
    truth = torch.as_tensor(fields.truth_ic(cfg), dtype=torch.float32, device="cuda").contiguous()
    free = runs["plain"].fine.clone()          # the same fine model and initial state, no analysis
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    rm = {"plain": [], "learned": [], "plain_feedback": [], "free": []}
    spread = []
    judge = []
    scratch = torch.empty_like(runs["plain"].fine)
    for c in range(1, n_cycles + 1):
        ctx.forecast(m.MENKF_FINE, truth, cfg.n_obs)
        y = ctx.observe(m.MENKF_FINE, truth)[0] + torch.as_tensor(fields.obs_noise(cfg, c), device="cuda")
        for k, r in runs.items():
            r.y.copy_(y)
            cc = r.ctx
            cc.forecast(m.MENKF_FINE, r.fine, cfg.n_obs, prev=r.prev)
            cc.forecast(m.MENKF_COARSE, r.members, cfg.n_obs)
            cc.restrict(r.fine, r.xs)
            cc.gain(r.members, r.xs, r.y, r.seed, c)
            cc.update(r.members, r.dc)
            if k == "learned" and c % 10 == 0:
                # the network's own correction (no judge) against the plain
                # correction of the same analysis, on scratch copies
                scratch.copy_(r.fine)
                cc.prolong_smooth(r.dc, scratch, r.prev, n_sweeps=n_sweeps, alpha=0.5)
                nn = r.fine.clone()
                cc.prolong_smooth(r.dc, nn, None, n_sweeps=0, mode=m.MENKF_PROLONG_LEARNED, net=r.net)
                d = float(torch.linalg.vector_norm(nn - scratch) / torch.linalg.vector_norm(scratch - r.fine))
                judge.append((c, d))
                del nn
            cc.prolong_smooth(r.dc, r.fine, r.prev, n_sweeps=r.n_sweeps, alpha=0.5, mode=r.mode, net=r.net)
            if k == "plain_feedback":
                cc.recentre(r.members, r.fine)
            cc.diagnostics(r.fine, truth, out=out)
            o = out.cpu().numpy()
            rm[k].append(float(np.sqrt(o[0] / o[1])))
        ctx.forecast(m.MENKF_FINE, free, cfg.n_obs)
        ctx.diagnostics(free, truth, out=out)
        o = out.cpu().numpy()
        rm["free"].append(float(np.sqrt(o[0] / o[1])))
        if c == 1 or c == n_cycles:
            o = ctx.spread(runs["plain"].members).cpu().numpy()
            spread.append(float(np.sqrt(o[0] / o[1])))
    for r in runs.values():
        if r.ctx.get_status() != 0:
            raise RuntimeError("analysis failed in the RMSE comparison")
    js = net.judge_stats.cpu().numpy()
    half = n_cycles // 2
    res = {k: float(np.mean(v[half:])) for k, v in rm.items()}
    return {
        "plain_rmse": res["plain"], "learned_rmse": res["learned"],
        "ratio": res["learned"] / res["plain"], "equal_rmse": res["learned"] <= 1.05 * res["plain"],
        "free_run_rmse": res["free"], "plain_below_free_run": 1.0 - res["plain"] / res["free"],
        "learned_below_free_run": 1.0 - res["learned"] / res["free"],
        "plain_member_spread_first_last": spread,
        "feedback_rmse": res["plain_feedback"], "feedback_ratio": res["plain_feedback"] / res["plain"],
        "cycles": n_cycles,
        "judge": {"every": net.judge_every, "tol": net.judge_tol, "judged": int(js[1]),
                  "plain_corrected_cycles": int(js[2]), "guarded_cycles": int(js[3]),
                  "last_judged_distance": float(js[0])},
        "guarded_tiles": int(net.fallback_count.item()),
        "network_distance_to_plain_correction": judge,
        "rmse_first_last": {k: [v[0], v[-1]] for k, v in rm.items()},
    }


def stage_kernel_roofline(cfg, cyc, reps=2):
    """Average duration of the ensemble RK4 stage kernel launches, timed with
    HIP events on the stream they are launched on, and their bytes per
    launch: the algorithmic minimum (one read and one write of the state per
    time step, shared by the launches of the step) and the kernel's own
    contract (13 state passes per step over four single-stage launches, 7
    over the two launches of the paired row march)."""
    import torch
    import paper_2012_10091_amd as m
    stream = torch.cuda.Stream()
    scratch = cyc.members.clone()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        cyc.ctx.forecast(m.MENKF_COARSE, scratch, cfg.n_obs, stream=stream)     # warm
        ev0.record(stream)
        for _ in range(reps):
            cyc.ctx.forecast(m.MENKF_COARSE, scratch, cfg.n_obs, stream=stream)
        ev1.record(stream)
    stream.synchronize()
    sc = cyc.ctx.get_schedule(m.MENKF_COARSE)
    chunk = sc["member_chunk"] or cfg.n_members
    n_chunks = -(-cfg.n_members // chunk)
    paired = tuple(sc["tile"]) == (0, 32)
    per_step = 2 if paired else 4
    launches = reps * cfg.n_obs * per_step * n_chunks
    avg_s = ev0.elapsed_time(ev1) / 1e3 / launches
    pts = cfg.n_members * cfg.nxc * cfg.nyc / n_chunks      # points per launch (equal chunks)
    state_bytes = pts * 4 * 4
    # kernel contract per step: single-stage launches 13 passes (stage 1: 1R 1W,
    # 2: 2R 2W, 3: 2R 1W, 4: 3R 1W); paired launches 7 (stages 1+2: 1R 2W,
    # stages 3+4: 3R 1W)
    contract = (7.0 if paired else 13.0) / per_step * state_bytes
    minimum = 2.0 * state_bytes / per_step      # one read + one write of the state per step
    if paired:
        shape = f"ns_march_pair<float,{cfg.nxc},0|1> (row march, two RK stages per launch, 32 rows per workgroup"
    elif sc["tile"][0] == 0:
        shape = f"ns_march<float,{cfg.nxc},*> (row march, one RK stage per launch, 16 rows per workgroup"
    else:
        shape = f"ns_stage<float,{sc['tile'][0]},{sc['tile'][1]},*> (tile, one RK stage per launch"
    return {
        "kernel": f"{shape}; ensemble RK4, {cfg.n_members} x 4 x {cfg.nyc}x{cfg.nxc}, member chunk "
                  f"{sc['member_chunk'] or cfg.n_members})",
        "avg_launch_us": avg_s * 1e6,
        "launches_per_step": per_step,
        "contract_bytes": contract,
        "traffic": measured_traffic(sc, cfg),
        "min_bytes": minimum,
        "achieved_contract": contract / avg_s / 1e9,
        "achieved": minimum / avg_s / 1e9,
    }


# FP32 operations per point and time step of the 1D Burgers forecast (three
# SSP-RK3 stages): per stage 7 for L(u) (difference, product, scaling;
# second difference, scaling, sum) and 2, 4, 4 for the stage combinations.
BURGERS_FLOPS_PER_POINT_STEP = 3 * 7 + 2 + 4 + 4
FP32_NONPACKED_PEAK_TFLOPS = 78.6   # 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz (packed FP32 off)


def window_kernel_roofline(cfg, cyc, reps=5):
    """The 1D member forecast (one launch per observation window, every
    member's row held in LDS for the window) timed with HIP events on its
    own stream, against the vector ALU peak: the state crosses HBM once per
    window, so the launch is bound by its arithmetic and latency, not by
    memory."""
    import torch
    import paper_2012_10091_amd as m
    stream = torch.cuda.Stream()
    scratch = cyc.members.clone()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        cyc.ctx.forecast(m.MENKF_COARSE, scratch, cfg.n_obs, stream=stream)
        ev0.record(stream)
        for _ in range(reps):
            cyc.ctx.forecast(m.MENKF_COARSE, scratch, cfg.n_obs, stream=stream)
        ev1.record(stream)
    stream.synchronize()
    avg_s = ev0.elapsed_time(ev1) / 1e3 / reps
    pts = cfg.n_members * cfg.nxc
    flops = BURGERS_FLOPS_PER_POINT_STEP * pts * cfg.n_obs
    return {
        "bound": "alu", "unit": "TFLOP/s", "peak": FP32_NONPACKED_PEAK_TFLOPS,
        "kernel": f"burgers_window_lds<float,*> (one workgroup per member, the row in LDS for the "
                  f"{cfg.n_obs}-step window; {cfg.n_members} x {cfg.nxc})",
        "avg_launch_us": avg_s * 1e6, "flops_per_launch": flops,
        "flops_per_point_step": BURGERS_FLOPS_PER_POINT_STEP,
        "achieved": flops / avg_s / 1e12, "hbm_bytes_per_launch": 2.0 * pts * 4,
        "hbm_gbs": 2.0 * pts * 4 / avg_s / 1e9,
    }


BF16_MFMA_PEAK_TFLOPS = 2500.0


def update_gemm_utilisation(cfg, cyc, reps=20):
    """The member update X Z (the anomaly GEMM of the analysis) timed alone:
    menkf_update on a scratch copy of the members with the gain factors of
    the last cycle, HIP events on its own stream.  MFMA work counts the
    BF16x3 products (3 x 2 N (N + 1) points); HBM bytes are one read and
    one write of the members (the minimum for an in-place update)."""
    import torch
    stream = torch.cuda.Stream()
    scratch = cyc.members.clone()
    dc = torch.empty_like(cyc.dc)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        cyc.ctx.update(scratch, dc, stream=stream)
        e0.record(stream)
        for _ in range(reps):
            cyc.ctx.update(scratch, dc, stream=stream)
        e1.record(stream)
    stream.synchronize()
    avg = e0.elapsed_time(e1) / 1e3 / reps
    N = cfg.n_members
    npts = cfg.n_coarse * cfg.nfields
    terms = 3
    flops = terms * 2.0 * N * (N + 1) * npts
    nbytes = 2.0 * N * npts * 4
    name = "update_wave" if N <= 128 else "update_bf16"
    return {"kernel": f"{name} (X Z, BF16x3 on MFMA, FP32 accumulation)", "avg_launch_us": avg * 1e6,
            "mfma_tflops": flops / avg / 1e12, "mfma_frac_of_bf16_peak": flops / avg / 1e12 / BF16_MFMA_PEAK_TFLOPS,
            "hbm_gbs": nbytes / avg / 1e9, "hbm_frac": nbytes / avg / 1e9 / HBM_PEAK_GBS}


FP64_PEAK_TFLOPS_MATRIX = 78.6
MALL_NOTE = ("not split: FETCH_SIZE / WRITE_SIZE count the L2 <-> data-fabric traffic, which includes "
             "Infinity Cache (MALL) hits; the counter list of rocprofv3 on this GPU exposes no MALL hit counter")


def gain_fp64_utilisation(cfg, cyc, reps=5):
    """The analysis (menkf_gain: observation of the members, anomalies, FP64
    S = Y Y^T + R on FP64 MFMA, blocked FP64 Cholesky with the solves folded
    in, Z = Y^T S^-1 [D | d*]) timed alone with HIP events on its own stream,
    against its algorithmic FP64 work 2 N_y^2 N (S) + N_y^3 / 3 (Cholesky)
    + 2 N_y^2 (N + 1) (solves) + 2 N_y N (N + 1) (Z)."""
    import torch
    stream = torch.cuda.Stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        cyc.ctx.gain(cyc.members, cyc.xs, cyc.y, 1, 1, stream=stream)
        e0.record(stream)
        for r in range(reps):
            cyc.ctx.gain(cyc.members, cyc.xs, cyc.y, 1, 2 + r, stream=stream)
        e1.record(stream)
    stream.synchronize()
    avg = e0.elapsed_time(e1) / 1e3 / reps
    ny, n = float(cfg.n_probes), float(cfg.n_members)
    parts = {"S": 2 * ny * ny * n, "cholesky": ny ** 3 / 3, "solves": 2 * ny * ny * (n + 1),
             "Z": 2 * ny * n * (n + 1)}
    flops = sum(parts.values())
    return {"call": "menkf_gain (exact R, N_y x N_y FP64)", "avg_us": avg * 1e6, "flops": flops,
            "flops_parts": parts, "tflops": flops / avg / 1e12,
            "frac_of_fp64_peak": flops / avg / 1e12 / FP64_PEAK_TFLOPS_MATRIX}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ns_march_pair_64x4x256sq_traffic.md")


def measured_traffic(schedule, cfg):
    """HBM bytes per launch of the stage kernel from the committed counter
    summary, or None when the kernel source, the ensemble's shape or the
    schedule differs from the one the counters were taken on
    (64 x 4 x 256^2)."""
    if (cfg.n_members, cfg.nyc, cfg.nxc) != (64, 256, 256):
        return None
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and " " not in line.split(": ")[0])
    src = os.path.join(ROOT, "paper_2012_10091_amd", "csrc", "ns2d.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    tag = f"{schedule['tile'][0]}x{schedule['tile'][1]}:{schedule['member_chunk']}"
    if vals.get("kernel_source_sha256") != h or vals.get("profiled_coarse_schedule") != tag:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_model():
    """The host CPU's model name (lscpu), for the baseline's record."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        f = {k.strip(): v.strip() for k, v in (ln.split(":", 1) for ln in out.splitlines() if ":" in ln)}
        if "Model name" in f:
            return (f"{f['Model name']} (family {f.get('CPU family', '?')}, model {f.get('Model', '?')}, "
                    f"{f.get('Socket(s)', '?')} socket(s), {f.get('CPU(s)', '?')} CPUs on the host)")
    except (OSError, subprocess.SubprocessError):
        pass
    return None


def cpu_baseline(cfg, budget_s=12.0):
    """The FP64 oracle on the host: the fine forecast and the forecast of all
    members (one batch, as in a cycle) step by step until the cycle's n_obs
    steps are done or the forecasts have taken about budget_s, then the
    analysis, Pi_F and three sweeps; the forecasts scaled to the cycle's
    n_obs steps when fewer were timed."""
    import numpy as np
    from oracle import cycle as ocycle
    from oracle import enkf, grids, rng, smooth
    from oracle.models import Model
    from synthetic import fields
    cores = len(os.sched_getaffinity(0))
    mf, mc = Model(cfg, "fine"), Model(cfg, "coarse")
    idx, comp = fields.probes_for(cfg)
    y = ocycle.observe_truth(cfg, fields.truth_ic(cfg), idx, comp)
    eps = rng.perturbations(cfg.seed + 5, 1, cfg.n_members, cfg.n_probes, cfg.obs_sigma)
    xf = np.asarray(fields.model_ic(cfg), dtype=np.float64)
    mem = np.asarray(fields.member_ics(cfg), dtype=np.float64)
    t_fine = t_mem = 0.0
    k = 0
    while k < cfg.n_obs and (k == 0 or t_fine + t_mem < budget_s):
        t = time.perf_counter()
        xf, xf_prev = mf.forecast(xf, 1)
        t_fine += time.perf_counter() - t
        t = time.perf_counter()
        mem, _ = mc.forecast(mem, 1)
        t_mem += time.perf_counter() - t
        k += 1
    t = time.perf_counter()
    res = enkf.analysis(mem, grids.restrict(xf, cfg.ratio, cfg.dim), y, eps, ocycle.make_H(cfg, idx, comp),
                        cfg.obs_sigma)
    t_an = time.perf_counter() - t
    t = time.perf_counter()
    smooth.smooth(xf + grids.prolong(res["delta"], cfg.ratio, cfg.dim), xf_prev, mf, 3, 0.5)
    t_pro = time.perf_counter() - t
    per_cycle = cfg.n_obs / k * (t_fine + t_mem) + t_an + t_pro
    scaled = f"forecasts scaled by {cfg.n_obs}/{k}" if k < cfg.n_obs else "a whole cycle, not scaled"
    return {
        "value": 1.0 / per_cycle,
        "unit": "cycles/s",
        "cores": cores,
        "cpu": cpu_model(),
        "kind": "oracle",
        "sample": (f"{k} of a cycle's {cfg.n_obs} time steps of the fine state ({t_fine:.1f}s) and of all "
                   f"{cfg.n_members} members in one batch ({t_mem:.1f}s), one analysis ({t_an:.1f}s), "
                   f"Pi_F + 3 sweeps ({t_pro:.1f}s); {scaled}"),
    }


def load_net(cfg, path, judge_every):
    from paper_2012_10091_amd import learned
    path = path or learned.weights_for(cfg.name)
    if not os.path.exists(path):
        return None, path
    return learned.load(path, guard=10.0, judge_every=judge_every), path


def bench_train(args):
    """Training throughput of the learned prolongation's network: Adam steps of
    menkf_net_train_step (forward, backward, Adam; BF16 storage, FP32
    arithmetic) on random periodic 128^2 crops, 16 per step, of synthetic
    pairs shaped like the 512^2 workload's, timed with HIP events on the
    stream they run on.  Beside it the oracle's FP64 forward and backward of
    one crop on the host."""
    import numpy as np
    import torch

    import paper_2012_10091_amd as m
    from oracle import net as onet
    from paper_2012_10091_amd import learned
    from synthetic import configs, fields
    cfg = configs.CONFIGS["C4"]
    batch, crop, npairs = 16, 128, 64
    net = learned.load(learned.weights_for("ns2d_512_128_n32"))
    rs = np.random.default_rng(cfg.seed + 71)
    xf0 = fields.model_ic(cfg).astype(np.float32)
    shape = (npairs, 4, cfg.ny, cfg.nx)
    xf = torch.as_tensor(np.broadcast_to(xf0, shape) + 1e-2 * rs.standard_normal(shape).astype(np.float32),
                         device="cuda").contiguous()
    dproj = torch.as_tensor(1e-3 * rs.standard_normal(shape).astype(np.float32), device="cuda").contiguous()
    target = torch.as_tensor(1e-3 * rs.standard_normal(shape).astype(np.float32), device="cuda").contiguous()
    n_sets = args.warmup + args.steps
    crops = torch.as_tensor(np.stack([rs.integers(0, npairs, (n_sets, batch)), rs.integers(0, cfg.ny, (n_sets, batch)),
                                      rs.integers(0, cfg.nx, (n_sets, batch))], axis=2).astype(np.int32),
                            device="cuda").contiguous()
    tr = m.Trainer(net, batch=batch, crop=crop)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            tr.step(dproj, xf, target, crops[i], stream=stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(args.warmup, n_sets):
            tr.step(dproj, xf, target, crops[i], stream=stream)
        e1.record(stream)
    stream.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    steps_s = args.steps / sec
    fl = learned.train_flops_per_crop(crop) * batch
    tflops = fl * steps_s / 1e12
    log(f"bench: training {steps_s:.1f} Adam steps/s ({steps_s * batch:.0f} crops/s), {tflops:.2f} TFLOP/s")
    out = {
        "metric": "learned-prolongation training Adam steps/s (batch 16 periodic 128^2 crops, 512^2 pairs)",
        "value": steps_s, "unit": "Adam steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 / steps_s, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "learned_train_512_crop128_b16", "pairs": npairs, "crops_per_s": steps_s * batch,
                   "flops_per_step": fl,
                   "kernels": "menkf_net_train_step: every convolution on BF16 MFMA 32x32x16 with FP32 "
                              "accumulation (forward of the three layers, data gradients with the FP32 output "
                              "gradient as BF16 hi + lo terms, weight gradients as 32 x 32 products over the "
                              "pixels, one per tap, gradient hi + lo), BF16 activations, Adam in FP32"},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / BF16_MFMA_PEAK_TFLOPS, "traffic": None,
                     "peak_note": "dense BF16 MFMA peak; achieved counts each convolution MAC of the forward and "
                                  "both gradients once (not the hi + lo products, nor the zero rows that pad "
                                  "4 or 8 channels to the 32-wide MFMA tile)"},
    }
    if args.cpu_baseline:
        log("bench: timing the oracle's forward + backward of one crop on the host")
        cores = len(os.sched_getaffinity(0))
        params = onet.init_params(cfg, zero_last=False)
        x = onet.make_input(params, rs.standard_normal((4, crop, crop)) * 1e-3, xf0[:, :crop, :crop])
        t = time.perf_counter()
        n = 0
        while time.perf_counter() - t < 10.0:
            o, cache = onet.forward(params, x)
            _, g = onet.mse(o, np.zeros_like(o))
            onet.backward(params, cache, g)
            n += 1
        dt = (time.perf_counter() - t) / n
        out["cpu_baseline"] = {"value": 1.0 / (dt * batch), "unit": "Adam steps/s", "cores": cores, "cpu": cpu_model(),
                               "kind": "oracle",
                               "sample": f"{n} FP64 forward + backward passes of one periodic {crop}^2 crop "
                                         f"({dt:.2f}s each), scaled to {batch} crops per step (Adam itself not timed)"}
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """48 independent instances of uneven sizes, one batch cycle per graph replay."""
    import torch

    import paper_2012_10091_amd as m
    from paper_2012_10091_amd import learned
    from synthetic import configs, fields
    cfgs = configs.uneven_batch()
    net = learned.load(learned.weights_for("ns2d_512_128_n32"), guard=10.0, judge_every=args.judge_every)
    f32 = torch.float32
    insts = []
    t0 = time.perf_counter()
    for cfg in cfgs:
        ctx = m.Context(cfg)
        idx, comp = fields.probes_for(cfg)
        ctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.as_tensor(comp, device="cuda"))
        fine = torch.as_tensor(fields.model_ic(cfg), dtype=f32, device="cuda").contiguous()
        mem = torch.as_tensor(fields.member_ics(cfg), dtype=f32, device="cuda").contiguous()
        truth = torch.as_tensor(fields.truth_ic(cfg), dtype=f32, device="cuda").contiguous()
        y = ctx.observe(m.MENKF_FINE, truth)[0] + torch.as_tensor(fields.obs_noise(cfg, 1), device="cuda")
        xs = torch.empty((4, cfg.nyc, cfg.nxc), dtype=f32, device="cuda")
        it = {"cfg": cfg, "ctx": ctx, "fine": fine, "prev": torch.empty_like(fine), "members": mem, "xs": xs,
              "dc": torch.empty_like(xs), "y": y.contiguous()}
        if args.autotune:
            ctx.autotune(m.MENKF_FINE, fine.clone(), cfg.n_obs, reps=2)
            ctx.autotune(m.MENKF_COARSE, mem.clone(), cfg.n_obs, reps=2)
        insts.append(it)
    torch.cuda.synchronize()
    log(f"bench: {len(insts)} instances ready in {time.perf_counter() - t0:.1f}s (autotune {bool(args.autotune)})")
    init = [(i["fine"].clone(), i["members"].clone()) for i in insts]

    def run(lanes):
        for i, (f, mm) in zip(insts, init):
            i["fine"].copy_(f)
            i["members"].copy_(mm)
        batch = m.Batch(n_lanes=lanes)
        stream = torch.cuda.Stream()
        a = [i["ctx"].cycle_args(i["fine"], i["prev"], i["members"], i["xs"], i["dc"], i["y"], i["cfg"].seed + 5,
                                 m.MENKF_CYCLE_DEVICE, i["cfg"].n_obs, n_sweeps=args.sweeps, alpha=0.5,
                                 mode=m.MENKF_PROLONG_LEARNED_FALLBACK, net=net) for i in insts]
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            m.Graph.begin(stream)
            batch.cycle(a, stream=stream)
            g = m.Graph.end(stream)
        for i in insts:
            i["ctx"].set_cycle(1, stream=stream)
        for _ in range(args.warmup):
            g.launch(stream)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            g.launch(stream)
        e1.record(stream)
        stream.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        bad = [i["cfg"].name for i in insts if i["ctx"].get_status() != 0]
        return args.steps / sec, bad, batch.lanes()

    cps, bad, lanes = run(args.lanes)
    log(f"bench: batch on {args.lanes} lanes: {cps:.2f} batch cycles/s, failed instances {bad}")
    cps1, bad1, _ = run(1)
    log(f"bench: batch on 1 lane: {cps1:.2f} batch cycles/s")
    # the dominant kernel: the coarse stage kernel of the instance with the
    # largest ensemble, timed alone on its own stream
    big = max(insts, key=lambda i: i["cfg"].n_members * i["cfg"].nxc * i["cfg"].nyc)
    rl = stage_kernel_roofline(big["cfg"], type("C", (), {"ctx": big["ctx"], "members": big["members"]})())
    log(f"bench: stage kernel of {big['cfg'].name}: {rl['avg_launch_us']:.1f} us per launch, algorithmic "
        f"{rl['achieved']:.0f} GB/s")
    out = {
        "metric": "uneven-batch assimilation cycles/s (48 independent 2D instances in one graph)",
        "value": cps, "unit": "batch cycles/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 / cps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uneven48", "instances": len(insts),
                   "fine_sides": sorted({c.nx for c in cfgs}), "members": sorted({c.n_members for c in cfgs}),
                   "probes_range": [min(c.n_probes for c in cfgs), max(c.n_probes for c in cfgs)],
                   "lanes": args.lanes, "lane_of": lanes, "instance_cycles_per_s": cps * len(insts),
                   "one_lane_batch_cycles_per_s": cps1, "autotuned": bool(args.autotune),
                   "prolongation": f"learned, judged every {net.judge_every} cycles against Pi_F + {args.sweeps} "
                                   f"sweeps (its fallback)", "failed_instances": bad + bad1},
        "roofline": {
            "bound": "hbm", "achieved": rl["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": rl["achieved"] / HBM_PEAK_GBS, "traffic": None,
            "kernel": rl["kernel"] + f" of the largest ensemble ({big['cfg'].name}), timed alone",
            "avg_launch_us": rl["avg_launch_us"], "algorithmic_bytes_per_launch": rl["min_bytes"],
            "algorithmic_bytes": "one read and one write of the state per time step, shared by the launches of a step",
        },
    }
    if args.cpu_baseline:
        # the oracle's cycle of one instance per fine side (its forecasts
        # timed for about 4 s, the rest scaled), and the batch as 16 times those three
        sample = []
        for side in sorted({c.nx for c in cfgs}):
            c = next(c for c in cfgs if c.nx == side)
            log(f"bench: timing the oracle on {c.name} (bounded sample)")
            sample.append((c.name, 1.0 / cpu_baseline(c, budget_s=4.0)["value"]))
        per_batch = len(cfgs) / len(sample) * sum(t for _, t in sample)
        out["cpu_baseline"] = {"value": 1.0 / per_batch, "unit": "batch cycles/s", "cores": len(os.sched_getaffinity(0)),
                               "cpu": cpu_model(), "kind": "oracle",
                               "sample": "cycles (forecast steps timed for ~4 s each, scaled to 20) of " + ", ".join(f"{n} ({t:.1f}s)" for n, t in sample)
                                         + f"; the batch of {len(cfgs)} taken as {len(cfgs) // len(sample)} times these"}
    print(json.dumps(out), flush=True)


FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
# FP64/FP32 operations per grid point and time step of the inlet forecast
# kernel: per Runge-Kutta stage 8 for the right-hand side (centred
# difference, product, second difference, scaling, sum) and 2 for
# x + dt L; 3 each for the stage combinations of stages 2 and 3.
INLET_FLOPS_PER_POINT_STEP = 3 * 10 + 2 * 3
# the first-order scheme: one right-hand side (8) and x + dt L (2) per step
FIRST_ORDER_FLOPS_PER_POINT_STEP = 10


def dual_cpu_baseline(cfg, n_cycles=20):
    """The FP64 oracle's dual cycle on a bounded sample of cycles (Sec. 4 size)."""
    import numpy as np
    from oracle import dual
    from synthetic import fields
    cores = len(os.sched_getaffinity(0))
    idx, _ = fields.probes_for(cfg)
    st = dual.DualState(fine=fields.inlet_uniform(cfg), members=fields.inlet_uniform(cfg, "coarse", cfg.n_members),
                        theta=fields.inlet_theta_ics(cfg), t=0.0)
    y = np.full(cfg.n_probes, cfg.u0)
    t = time.perf_counter()
    for _ in range(n_cycles):
        st, _ = dual.dual_cycle(cfg, st, y, idx, n_sweeps=1)
    sec = time.perf_counter() - t
    return {"value": n_cycles / sec, "unit": "dual cycles/s", "cores": cores, "cpu": cpu_model(), "kind": "oracle",
            "sample": f"{n_cycles} dual cycles of the oracle at the full size ({sec:.1f}s)"}


def bench_dual(args):
    """Dual (parameter + state) MEnKF of the inlet-forced Burgers case at the
    Sec. 4 size: fine 800 nodes, coarse 200, 100 members, 80 sensors every 30
    steps.  One step = one dual cycle (two member forecasts, fine forecast,
    two gains, parameter and member updates, correction + sweep), captured as
    one graph with the device cycle counter and clock.  Truth, spin-up and
    observations are produced by the library on the GPU beforehand."""
    import numpy as np
    import torch

    import paper_2012_10091_amd as m
    from synthetic import configs, fields
    cfg = configs.inlet_burgers(n_members=100, precision=args.dual_precision, time_scheme=args.time_scheme)
    F64 = torch.float64
    dt = F64 if cfg.precision == "f64" else torch.float32
    ctx = m.Context(cfg)
    idx, comp = fields.probes_for(cfg)
    ctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.as_tensor(comp, device="cuda"))
    dev = lambda a, ty=dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", ty).contiguous()
    truth = dev(fields.inlet_uniform(cfg))
    fine = dev(fields.inlet_uniform(cfg))
    prev = torch.empty_like(fine)
    mem = dev(fields.inlet_uniform(cfg, "coarse", cfg.n_members))
    theta = dev(fields.inlet_theta_ics(cfg), F64)
    th_true = dev(np.array([cfg.theta_true]), F64)
    tmean = dev(fields.inlet_theta_ics(cfg).mean(axis=0), F64)
    spin = int(round(cfg.t_spinup / cfg.dt))
    t0 = torch.zeros(1, dtype=F64, device="cuda")
    ctx.forecast_inlet(m.MENKF_FINE, truth, spin, th_true, t0)
    ctx.forecast_inlet(m.MENKF_FINE, fine, spin, tmean, t0)
    ctx.forecast_inlet(m.MENKF_COARSE, mem, spin, theta, t0)
    n_cyc = args.warmup + args.steps
    t_obs = torch.empty(1, dtype=F64, device="cuda")
    Y = torch.empty((n_cyc, cfg.n_probes), dtype=F64, device="cuda")
    for c in range(n_cyc):
        t_obs.fill_(spin * cfg.dt + c * cfg.n_obs * cfg.dt)
        ctx.forecast_inlet(m.MENKF_FINE, truth, cfg.n_obs, th_true, t_obs)
        Y[c] = ctx.observe(m.MENKF_FINE, truth)[0] + dev(fields.obs_noise(cfg, c + 1), F64)
    clock = torch.full((1,), spin * cfg.dt, dtype=F64, device="cuda")
    xs = torch.empty((1, cfg.nxc), dtype=dt, device="cuda")
    dc = torch.empty_like(xs)
    y = torch.empty(cfg.n_probes, dtype=F64, device="cuda")
    torch.cuda.synchronize()
    log(f"bench: dual workload {cfg.name} {cfg.precision} ready (spin-up {spin} steps)")
    stream = torch.cuda.Stream()
    aux = torch.cuda.Stream()     # the fine forecast runs beside the member forecast
    with torch.cuda.stream(stream):
        ctx.set_cycle(1, stream=stream)
        m.Graph.begin(stream)
        ctx.dual_cycle(fine, prev, mem, xs, dc, y, theta, tmean, clock, cfg.seed + 5, m.MENKF_CYCLE_DEVICE,
                       cfg.n_obs, n_sweeps=1, alpha=0.5, stream=stream, aux_stream=aux)
        g = m.Graph.end(stream)
    for c in range(args.warmup):
        with torch.cuda.stream(stream):
            y.copy_(Y[c])
        g.launch(stream)
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for c in range(args.warmup, n_cyc):
        with torch.cuda.stream(stream):
            y.copy_(Y[c])
        g.launch(stream)
    e1.record(stream)
    stream.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    cps = args.steps / sec
    status = ctx.get_status()
    th = tmean.cpu().numpy().tolist()
    log(f"bench: dual {cps:.1f} cycles/s, theta mean after {n_cyc} cycles {th}, status {status}")
    # dominant kernel: the member forecast (burgers_inlet_window), timed on its own stream
    scratch = mem.clone()
    reps = 20
    with torch.cuda.stream(stream):
        ctx.forecast_inlet(m.MENKF_COARSE, scratch, cfg.n_obs, theta, clock, stream=stream)
        e0.record(stream)
        for _ in range(reps):
            ctx.forecast_inlet(m.MENKF_COARSE, scratch, cfg.n_obs, theta, clock, stream=stream)
        e1.record(stream)
    stream.synchronize()
    avg_s = e0.elapsed_time(e1) / 1e3 / reps
    per_point = INLET_FLOPS_PER_POINT_STEP if cfg.time_scheme == "ssprk3" else FIRST_ORDER_FLOPS_PER_POINT_STEP
    flops = per_point * cfg.n_members * cfg.nxc * cfg.n_obs
    peak = FP64_VECTOR_PEAK_TFLOPS if cfg.precision == "f64" else FP32_VECTOR_PEAK_TFLOPS
    achieved = flops / avg_s / 1e12
    log(f"bench: member forecast {avg_s * 1e6:.1f} us per launch, {achieved:.3f} TFLOP/s")
    scheme = "SSP-RK3" if cfg.time_scheme == "ssprk3" else "first-order (forward Euler, Jacobi analysis step)"
    out = {
        "metric": f"dual assimilation cycles/s, inlet-forced Burgers 800/200 N=100 (parameters + state), {scheme}",
        "value": cps, "unit": "dual cycles/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 / cps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": cfg.precision, "data": "synthetic",
        "config": {"workload": cfg.name, "fine": cfg.nx, "coarse": cfg.nxc, "members": cfg.n_members,
                   "probes": cfg.n_probes, "steps_per_cycle": cfg.n_obs, "spinup_steps": spin,
                   "theta_true": list(cfg.theta_true), "theta_prior": list(cfg.theta_prior),
                   "theta_mean_after": th, "cycles_run": n_cyc, "status_word": status},
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": None,
            "kernel": f"burgers_inlet_window<{'double' if cfg.precision == 'f64' else 'float'}> "
                      f"({cfg.n_members} members x {cfg.nxc} nodes x {cfg.n_obs} steps, LDS-resident)",
            "avg_launch_us": avg_s * 1e6, "flops_per_launch": flops,
        },
    }
    if args.cpu_baseline:
        log("bench: timing the oracle's dual cycle on the host (bounded sample)")
        out["cpu_baseline"] = dual_cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


def dual_study(args):
    """Parameter estimation of the inlet-forced case for r_C = 1, 2, 4, 8, 16
    as in Sec. 4: everything starts from u0 at t = 0, runs freely to t = 10,
    then one analysis every 30 steps up to t = 29 (3166 dual cycles).  The
    truth (theta = (0.2, 0)) is a fine run of the library's own model; all
    ratios see the same observations.  Prints one JSON line with theta-mean
    traces and summary figures per ratio."""
    import numpy as np
    import torch

    import paper_2012_10091_amd as m
    from synthetic import configs, fields
    F64 = torch.float64
    ratios = (1, 2, 4, 8, 16)
    base = configs.inlet_burgers(n_members=100, precision=args.dual_precision)
    if args.theta_walk is not None:
        base = base.with_(theta_walk=(args.theta_walk, args.theta_walk))
    dt = F64 if base.precision == "f64" else torch.float32
    dev = lambda a, ty=dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", ty).contiguous()
    spin = int(round(base.t_spinup / base.dt))
    n_cyc = base.n_cycles
    # truth and observations (same for every ratio)
    tctx = m.Context(base)
    idx, comp = fields.probes_for(base)
    tctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.as_tensor(comp, device="cuda"))
    truth = dev(fields.inlet_uniform(base))
    th_true = dev(np.array([base.theta_true]), F64)
    t_obs = torch.zeros(1, dtype=F64, device="cuda")
    tctx.forecast_inlet(m.MENKF_FINE, truth, spin, th_true, t_obs)
    Y = torch.empty((n_cyc, base.n_probes), dtype=F64, device="cuda")
    for c in range(n_cyc):
        t_obs.fill_(spin * base.dt + c * base.n_obs * base.dt)
        tctx.forecast_inlet(m.MENKF_FINE, truth, base.n_obs, th_true, t_obs)
        Y[c] = tctx.observe(m.MENKF_FINE, truth)[0] + dev(fields.obs_noise(base, c + 1), F64)
    truth_end = truth.clone()
    torch.cuda.synchronize()
    log(f"bench: dual study, {n_cyc} observation times ready")
    out = {"study": "inlet_dual_theta", "precision": base.precision, "members": base.n_members,
           "probes": base.n_probes, "window": [spin * base.dt, (spin + n_cyc * base.n_obs) * base.dt],
           "theta_true": list(base.theta_true), "theta_prior": list(base.theta_prior),
           "theta_walk": list(base.theta_walk), "ratios": {}}
    every = 50
    for r in ratios:
        cfg = base.with_(ratio=r, name=f"burgers1d_inlet_800_r{r}_n100")
        ctx = m.Context(cfg)
        ctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.as_tensor(comp, device="cuda"))
        theta = dev(fields.inlet_theta_ics(cfg), F64)
        tmean = dev(fields.inlet_theta_ics(cfg).mean(axis=0), F64)
        fine = dev(fields.inlet_uniform(cfg))
        prev = torch.empty_like(fine)
        mem = dev(fields.inlet_uniform(cfg, "coarse", cfg.n_members))
        t0 = torch.zeros(1, dtype=F64, device="cuda")
        ctx.forecast_inlet(m.MENKF_FINE, fine, spin, tmean, t0)
        ctx.forecast_inlet(m.MENKF_COARSE, mem, spin, theta, t0)
        clock = torch.full((1,), spin * cfg.dt, dtype=F64, device="cuda")
        xs = torch.empty((1, cfg.nxc), dtype=dt, device="cuda")
        dc = torch.empty_like(xs)
        y = torch.empty(cfg.n_probes, dtype=F64, device="cuda")
        hist = torch.empty((n_cyc, 2), dtype=F64, device="cuda")
        stream = torch.cuda.Stream()
        aux = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            ctx.set_cycle(1, stream=stream)
            m.Graph.begin(stream)
            ctx.dual_cycle(fine, prev, mem, xs, dc, y, theta, tmean, clock, cfg.seed + 5, m.MENKF_CYCLE_DEVICE,
                           cfg.n_obs, n_sweeps=1, alpha=0.5, stream=stream, aux_stream=aux)
            g = m.Graph.end(stream)
        t = time.perf_counter()
        for c in range(n_cyc):
            with torch.cuda.stream(stream):
                y.copy_(Y[c])
            g.launch(stream)
            with torch.cuda.stream(stream):
                hist[c].copy_(tmean)
        stream.synchronize()
        wall = time.perf_counter() - t
        h = hist.cpu().numpy()
        status = ctx.get_status()
        tc = cfg.n_obs * cfg.dt                      # time units per cycle (t_c = 1)
        # converged: the running mean over one t_c stays within 0.01 (5 %) of the truth
        w = int(round(1.0 / tc))
        run = np.convolve(h[:, 0], np.ones(w) / w, mode="valid")     # run[k] = mean of cycles k..k+w-1
        bad = np.nonzero(np.abs(run - cfg.theta_true[0]) >= 0.01)[0]
        conv = (int(bad[-1]) + 1 if len(bad) else 0) + w              # end of the first good window
        last = h[-int(round(5.0 / tc)):]             # the last 5 t_c
        fe = float(torch.linalg.vector_norm(fine - truth_end) / torch.linalg.vector_norm(truth_end))
        rec = {"coarse": cfg.nxc, "status": status, "wall_s": wall,
               "t_converged_1tc_mean_within_0p01": None if conv > n_cyc else conv * tc,
               "theta_mean_last5tc": last.mean(axis=0).tolist(), "theta_std_last5tc": last.std(axis=0).tolist(),
               "theta_end": h[-1].tolist(), "fine_rel_err_end": fe,
               "theta_after_cycles_1_10_50": [h[0].tolist(), h[9].tolist(), h[49].tolist()],
               "trace_every_50_cycles": h[::every].round(5).tolist()}
        out["ratios"][str(r)] = rec
        log(f"bench: r={r}: theta end {h[-1]}, last-5tc mean {rec['theta_mean_last5tc']} "
            f"std {rec['theta_std_last5tc']}, converged after {rec['t_converged_1tc_mean_within_0p01']} t_c, "
            f"fine rel err {fe:.4f}, {wall:.1f}s")
    print(json.dumps(out), flush=True)


# FP64/FP32 operations per node and step of the Euler forecast kernel:
# flux 9 (u = m / rho, p from 4 operations, two products with their sums),
# update 4 per field, filter 10 per field.
EULER_FLOPS_PER_POINT_STEP = 9 + 3 * 4 + 3 * 10


class EulerTruth:
    """Reference run of the acoustic case on the GPU: the library's fine
    forecast advanced one step per call, its inlet amplitude the truth
    theta(t) = theta0 (1 + sin(omega t / b)) at the end of each step (the
    per-step parameters and start times are tabulated on the device)."""

    def __init__(self, ctx, cfg):
        import torch

        from synthetic import fields
        self.ctx, self.cfg = ctx, cfg
        self.x = torch.as_tensor(fields.inlet_uniform(cfg)) \
            .to("cuda", torch.float64 if cfg.precision == "f64" else torch.float32).contiguous()

    def advance(self, nsteps, t_start):
        """nsteps single steps from time t_start."""
        import numpy as np
        import torch
        cfg = self.cfg
        ts = t_start + np.arange(nsteps) * cfg.dt
        th = np.zeros((nsteps, 2))
        th[:, 0] = cfg.theta_true[0] * (1.0 + np.sin(cfg.omega / cfg.theta_b * (ts + cfg.dt)))
        th_d = torch.as_tensor(th, dtype=torch.float64, device="cuda")
        ts_d = torch.as_tensor(ts, dtype=torch.float64, device="cuda")
        for k in range(nsteps):
            self.ctx.forecast_inlet(0, self.x, 1, th_d[k], ts_d[k:k + 1])


def euler_observations(m, cfg, ctx, n_obs_list, t_end=110.0):
    """Spin-up of the truth (restarted at t = 0, as the paper does), then the
    noise-free momentum at the sensors every n_obs steps for each n_obs of
    the list, plus the momentum field at those times, over [0, t_end]."""
    import torch
    spin = int(round(cfg.t_spinup / cfg.dt))
    tr = EulerTruth(ctx, cfg)
    tr.advance(spin, 0.0)
    total = int(round(t_end / cfg.dt))
    obs = {n: [] for n in n_obs_list}
    fields_at = {n: [] for n in n_obs_list}
    step = 0
    marks = sorted({k * n for n in n_obs_list for k in range(1, total // n + 1)})
    mi = 0
    while step < total:
        nxt = marks[mi] if mi < len(marks) else total
        tr.advance(nxt - step, step * cfg.dt)
        step = nxt
        if mi < len(marks) and step == marks[mi]:
            y = ctx.observe(m.MENKF_FINE, tr.x)[0].clone()
            for n in n_obs_list:
                if step % n == 0:
                    obs[n].append(y)
                    fields_at[n].append(tr.x[1].to(torch.float64).clone())
            mi += 1
    return {n: (torch.stack(obs[n]), torch.stack(fields_at[n])) for n in n_obs_list}


def euler_run(m, cfg, obs, truth_fields, record=True, aux=True, warmup=0):
    """Dual filter over the observations of one analysis frequency; returns
    (seconds of the replays after the first `warmup`, theta-mean trace,
    momentum errors, context, (members, theta, clock))."""
    import numpy as np
    import torch

    from synthetic import fields
    F64 = torch.float64
    dt = F64 if cfg.precision == "f64" else torch.float32
    ctx = m.Context(cfg)
    idx, comp = fields.probes_for(cfg)
    ctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.as_tensor(comp, device="cuda"))
    dev = lambda a, ty=dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", ty).contiguous()
    fine = dev(fields.inlet_uniform(cfg))
    prev = torch.empty_like(fine)
    mem = dev(fields.inlet_uniform(cfg, "coarse", cfg.n_members))
    theta = dev(fields.inlet_theta_ics(cfg), F64)
    tmean = torch.zeros(2, dtype=F64, device="cuda")
    clock = torch.zeros(1, dtype=F64, device="cuda")
    xs = torch.empty((3, cfg.nxc), dtype=dt, device="cuda")
    dc = torch.empty_like(xs)
    y = torch.empty(cfg.n_probes, dtype=F64, device="cuda")
    n_cyc = obs.shape[0]
    noise = dev(np.stack([fields.obs_noise(cfg, c + 1) for c in range(n_cyc)]), F64)
    Y = (obs + noise).contiguous()
    base = torch.as_tensor(fields.inlet_uniform(cfg)[1], dtype=F64, device="cuda")
    hist = torch.empty((n_cyc, 2), dtype=F64, device="cuda")
    err = torch.empty(n_cyc, dtype=F64, device="cuda")
    stream = torch.cuda.Stream()
    aux_s = torch.cuda.Stream() if aux else None
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        ctx.set_cycle(1, stream=stream)
        m.Graph.begin(stream)
        ctx.dual_cycle(fine, prev, mem, xs, dc, y, theta, tmean, clock, cfg.seed + 5, m.MENKF_CYCLE_DEVICE,
                       cfg.n_obs, n_sweeps=1, alpha=0.5, stream=stream, aux_stream=aux_s)
        g = m.Graph.end(stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for c in range(n_cyc):
        if c == warmup:
            e0.record(stream)
        with torch.cuda.stream(stream):
            y.copy_(Y[c])
        g.launch(stream)
        if record:
            with torch.cuda.stream(stream):
                hist[c].copy_(tmean)
                d = fine[1].to(F64) - truth_fields[c]
                err[c] = torch.linalg.vector_norm(d) / torch.linalg.vector_norm(truth_fields[c] - base)
    e1.record(stream)
    stream.synchronize()
    return e0.elapsed_time(e1) / 1e3, hist.cpu().numpy(), err.cpu().numpy(), ctx, (mem, theta, clock)


def euler_study(args):
    """Tracking of the time-varying inlet amplitude for f_a = 55, 10, 2
    analyses per characteristic time over [0, 110] (Sec. 5): theta-mean
    traces, mean tracking error, best lag, peak ratio, momentum error."""
    import numpy as np
    import torch

    import paper_2012_10091_amd as m
    from synthetic import configs, fields
    n_list = (30, 167, 833)
    walk = {} if args.theta_walk is None else {"theta_walk": (args.theta_walk, 0.0)}
    base = configs.euler_inlet(precision=args.dual_precision, **walk)
    tctx = m.Context(base)
    idx, comp = fields.probes_for(base)
    tctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.as_tensor(comp, device="cuda"))
    t0 = time.perf_counter()
    O = euler_observations(m, base, tctx, n_list)
    log(f"bench: euler truth over [0, 110] ready in {time.perf_counter() - t0:.1f}s")
    out = {"study": "euler_dual_theta_tracking", "precision": base.precision, "members": base.n_members,
           "ratio": base.ratio, "probes": base.n_probes, "theta_walk": list(base.theta_walk),
           "obs_sigma": base.obs_sigma, "runs": {}}
    for n in n_list:
        cfg = configs.euler_inlet(n_obs=n, precision=args.dual_precision, **walk)
        obs, tf = O[n]
        sec, h, err, _, _ = euler_run(m, cfg, obs, tf)
        ta = cfg.n_obs * cfg.dt
        t = ta * np.arange(1, len(h) + 1)
        truth = cfg.theta_true[0] * (1.0 + np.sin(cfg.omega / cfg.theta_b * t))
        late = t >= 10.0
        mae = float(np.abs(h[late, 0] - truth[late]).mean())
        lags = np.arange(0.0, 3.01, 0.05)
        lag_err = [float(np.abs(h[late, 0] - cfg.theta_true[0] * (1.0 + np.sin(cfg.omega / cfg.theta_b * (t[late] - L)))).mean())
                   for L in lags]
        best = float(lags[int(np.argmin(lag_err))])
        # ratio of the estimate's maxima to the truth's (0.03), one per period of 10 after t = 10
        peaks = [float(h[(t >= p0) & (t < p0 + 10.0), 0].max()) / (2 * cfg.theta_true[0]) for p0 in np.arange(10.0, 110.0, 10.0)
                 if np.any((t >= p0) & (t < p0 + 10.0))]
        f_a = 1.0 / ta
        rec = {"n_obs": n, "f_a": f_a, "cycles": len(h), "seconds": sec,
               "theta_mean_abs_error_t_ge_10": mae, "best_lag": best, "theta_mean_abs_error_at_best_lag": min(lag_err),
               "peak_ratio_mean": float(np.mean(peaks)), "momentum_rel_error_mean_t_ge_10": float(err[late].mean()),
               "momentum_rel_error_end": float(err[-1]),
               "trace": [[round(float(a), 4), round(float(b), 6)] for a, b in zip(t[::max(1, len(t) // 200)], h[::max(1, len(t) // 200), 0])]}
        out["runs"][f"{f_a:.1f}"] = rec
        log(f"bench: euler f_a={f_a:.1f} (n_obs {n}): {len(h)} cycles in {sec:.2f}s, |theta - truth| {mae:.5f}, "
            f"best lag {best:.2f} ({min(lag_err):.5f}), peaks {np.mean(peaks):.3f}, momentum error {err[late].mean():.3f}")
    print(json.dumps(out), flush=True)


def bench_euler(args):
    """Dual filter of the acoustic case at the Sec. 5 size (800/200 nodes,
    N = 100, 80 sensors, an analysis every 30 steps): dual cycles/s of the
    captured cycle replayed over observations already in HBM."""
    import torch

    import paper_2012_10091_amd as m
    from synthetic import configs, fields
    cfg = configs.euler_inlet(precision=args.dual_precision)
    tctx = m.Context(cfg)
    idx, comp = fields.probes_for(cfg)
    tctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.as_tensor(comp, device="cuda"))
    n_cyc = args.warmup + args.steps
    O = euler_observations(m, cfg, tctx, (cfg.n_obs,), t_end=(n_cyc + 1) * cfg.n_obs * cfg.dt)
    obs, tf = O[cfg.n_obs]
    obs, tf = obs[:n_cyc], tf[:n_cyc]
    log(f"bench: euler workload {cfg.name} {cfg.precision} ready")
    sec, h, _, ctx, (mem, theta, clock) = euler_run(m, cfg, obs, tf, record=False, warmup=args.warmup)
    cps = args.steps / sec
    status = ctx.get_status()
    log(f"bench: euler dual {cps:.1f} cycles/s over {args.steps} timed cycles, status {status}")
    stream = torch.cuda.Stream()
    scratch = mem.clone()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 20
    with torch.cuda.stream(stream):
        ctx.forecast_inlet(m.MENKF_COARSE, scratch, cfg.n_obs, theta, clock, stream=stream)
        e0.record(stream)
        for _ in range(reps):
            ctx.forecast_inlet(m.MENKF_COARSE, scratch, cfg.n_obs, theta, clock, stream=stream)
        e1.record(stream)
    stream.synchronize()
    avg_s = e0.elapsed_time(e1) / 1e3 / reps
    flops = EULER_FLOPS_PER_POINT_STEP * cfg.n_members * cfg.nxc * cfg.n_obs
    peak = FP64_VECTOR_PEAK_TFLOPS if cfg.precision == "f64" else FP32_VECTOR_PEAK_TFLOPS
    achieved = flops / avg_s / 1e12
    log(f"bench: euler member forecast {avg_s * 1e6:.1f} us per launch, {achieved:.3f} TFLOP/s")
    out = {
        "metric": "dual assimilation cycles/s, inlet-forced 1D Euler 800/200 N=100 (acoustic case, f_a = 55)",
        "value": cps, "unit": "dual cycles/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 / cps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": cfg.precision, "data": "synthetic",
        "config": {"workload": cfg.name, "fine": cfg.nx, "coarse": cfg.nxc, "members": cfg.n_members,
                   "probes": cfg.n_probes, "steps_per_cycle": cfg.n_obs, "status_word": status},
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": None,
            "kernel": f"euler_inlet_window<{'double' if cfg.precision == 'f64' else 'float'}> "
                      f"({cfg.n_members} members x 3 x {cfg.nxc} nodes x {cfg.n_obs} steps, LDS-resident)",
            "avg_launch_us": avg_s * 1e6, "flops_per_launch": flops,
        },
    }
    if args.cpu_baseline:
        log("bench: timing the oracle's dual cycle on the host (bounded sample)")
        out["cpu_baseline"] = dual_cpu_baseline(cfg, n_cycles=20)
    print(json.dumps(out), flush=True)


def with_gain_mode(cfg, mode):
    """The workload configuration with another menkf gain mode."""
    import dataclasses

    @dataclasses.dataclass(frozen=True)
    class C(type(cfg)):
        gain_mode: int = mode
    return C(**dataclasses.asdict(cfg))


def parse_schedule(text):
    """'fine=64x8:0,coarse=32x8:32' -> {"fine": ((64, 8), 0), "coarse": ((32, 8), 32)}"""
    out = {}
    for part in text.split(","):
        level, spec = part.split("=")
        tile, chunk = spec.split(":")
        tx, ty = tile.split("x")
        out[level.strip()] = ((int(tx), int(ty)), int(chunk))
    return out


def apply_schedule(ctx, sched):
    import paper_2012_10091_amd as m
    for level, ((tx, ty), chunk) in sched.items():
        ctx.set_schedule(m.MENKF_FINE if level == "fine" else m.MENKF_COARSE, (tx, ty), chunk)


def traffic_probe(args):
    """Kernels for hardware-counter passes (FETCH_SIZE / WRITE_SIZE): a plain
    1 GiB device-to-device copy of known size to calibrate the counters, then
    one eager (not graph-captured) cycle of the headline workload."""
    import torch

    import paper_2012_10091_amd as m
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    cfg = make_cfg(args)
    cyc = Cycle(cfg, args.sweeps)
    if args.schedule:
        apply_schedule(cyc.ctx, parse_schedule(args.schedule))
    elif args.autotune:
        cyc.autotune()
    stream = torch.cuda.Stream()
    cyc.ctx.set_cycle(1, stream=stream)
    with torch.cuda.stream(stream):
        cyc.issue(stream)
    stream.synchronize()
    sc = cyc.ctx.get_schedule(m.MENKF_COARSE)
    print(json.dumps({"probe": "traffic", "copy_bytes": n * 4, "workload": cfg.name,
                      "coarse_schedule": sc, "status": cyc.ctx.get_status()}), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU: this build measures the single-GPU hot path "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "learned_train":
        return bench_train(args)
    if args.workload == "uneven48":
        return bench_batch(args)
    if args.workload == "inlet_dual":
        return dual_study(args) if args.dual_study else bench_dual(args)
    if args.workload == "euler_dual":
        return euler_study(args) if args.dual_study else bench_euler(args)
    if args.traffic_probe:
        return traffic_probe(args)
    import torch
    import paper_2012_10091_amd as m
    m.load_library()
    cfg = make_cfg(args)
    n_cyc = args.warmup + args.steps
    log(f"bench: workload {cfg.name}, warmup {args.warmup}, steps {args.steps}")
    Y, _ = truth_observations(cfg, n_cyc)
    log("bench: observations ready")
    pipe = bool(args.pipelined)
    plain = Cycle(cfg, args.sweeps, pipelined=pipe)
    tuned = None
    if args.schedule:
        apply_schedule(plain.ctx, parse_schedule(args.schedule))
        tuned = {k: plain.ctx.get_schedule(m.MENKF_FINE if k == "fine" else m.MENKF_COARSE)
                 for k in ("fine", "coarse")}
    elif args.autotune:
        tuned = plain.autotune()
    if tuned:
        log(f"bench: autotuned schedules {tuned}")
    sec, wall = time_cycles(plain, Y, args.warmup, args.steps)
    status = plain.ctx.get_status()
    plain_cps = args.steps / sec
    log(f"bench: plain {plain_cps:.2f} cycles/s (graph events {sec:.3f}s, wall {wall:.3f}s), status {status}")
    variants = {"plain": {"cycles_per_s": plain_cps, "ms_per_cycle": sec / args.steps * 1e3,
                          "prolongation": f"Pi_F + {args.sweeps} relaxed sweeps", "pipelined": pipe}}

    def ordinary(mode=0, net=None):
        # the same cycle with the correction at its end (not pipelined)
        o = Cycle(cfg, args.sweeps, mode=mode, net=net)
        if tuned:
            apply_schedule(o.ctx, {k: (tuple(v["tile"]), v["member_chunk"]) for k, v in tuned.items()})
        osec, _ = time_cycles(o, Y, args.warmup, args.steps)
        return {"cycles_per_s": args.steps / osec, "ms_per_cycle": osec / args.steps * 1e3, "pipelined": False}

    if pipe:
        variants["plain_ordinary"] = ordinary()
        log(f"bench: plain, ordinary cycles {variants['plain_ordinary']['cycles_per_s']:.2f} cycles/s")
    value, ms = plain_cps, sec / args.steps * 1e3
    net, wpath = load_net(cfg, args.weights, args.judge_every) if cfg.dim == 2 else (None, None)
    headline = "plain"
    if net is not None and not args.small:
        learned = Cycle(cfg, args.sweeps, mode=m.MENKF_PROLONG_LEARNED_FALLBACK, net=net, pipelined=pipe)
        net.judge_stats.zero_()
        if tuned:
            learned.ctx.set_schedule(m.MENKF_FINE, tuned["fine"]["tile"], tuned["fine"]["member_chunk"])
            learned.ctx.set_schedule(m.MENKF_COARSE, tuned["coarse"]["tile"], tuned["coarse"]["member_chunk"])
        lsec, _ = time_cycles(learned, Y, args.warmup, args.steps)
        lstatus = learned.ctx.get_status()
        lcps = args.steps / lsec
        tjs = net.judge_stats.cpu().numpy()
        log(f"bench: learned {lcps:.2f} cycles/s, status {lstatus}")
        net.fallback_count.zero_()
        cmp = rmse_comparison(cfg, net, args.rmse_cycles, args.sweeps, args.judge_every)
        log(f"bench: RMSE plain {cmp['plain_rmse']:.5f} learned {cmp['learned_rmse']:.5f} "
            f"(ratio {cmp['ratio']:.3f}, equal {cmp['equal_rmse']})")
        variants["learned"] = {"cycles_per_s": lcps, "ms_per_cycle": lsec / args.steps * 1e3,
                               "prolongation": f"network; judged every {net.judge_every} cycles against Pi_F + "
                                               f"{args.sweeps} sweeps (its fallback above distance {net.judge_tol})",
                               "timed_cycles_judged": int(tjs[1]), "timed_cycles_on_plain": int(tjs[2]),
                               "weights": os.path.relpath(wpath, ROOT), "pipelined": pipe}
        if pipe:
            variants["learned_ordinary"] = ordinary(m.MENKF_PROLONG_LEARNED_FALLBACK, net)
            log(f"bench: learned, ordinary cycles {variants['learned_ordinary']['cycles_per_s']:.2f} cycles/s")
        variants["rmse"] = cmp
        if cmp["equal_rmse"] and lstatus == 0:
            value, ms, headline = lcps, lsec / args.steps * 1e3, "learned"
        # the same cycle with the ensemble-space form of the gain (an exact
        # identity for R = s^2 I; not the headline, which keeps the N_y x N_y
        # FP64 Cholesky of the workload)
        ens = Cycle(with_gain_mode(cfg, m.MENKF_GAIN_ENSEMBLE_SPACE), args.sweeps,
                    mode=m.MENKF_PROLONG_LEARNED_FALLBACK, net=net, pipelined=pipe)
        if tuned:
            ens.ctx.set_schedule(m.MENKF_FINE, tuned["fine"]["tile"], tuned["fine"]["member_chunk"])
            ens.ctx.set_schedule(m.MENKF_COARSE, tuned["coarse"]["tile"], tuned["coarse"]["member_chunk"])
        esec, _ = time_cycles(ens, Y, args.warmup, args.steps)
        ecps = args.steps / esec
        log(f"bench: learned + ensemble-space gain {ecps:.2f} cycles/s, status {ens.ctx.get_status()}")
        variants["learned_ensemble_space_gain"] = {
            "cycles_per_s": ecps, "ms_per_cycle": esec / args.steps * 1e3,
            "gain": "(s^2 I + Y^T Y)^-1 Y^T [D | d*], N x N FP64 Cholesky (exact identity; not the headline)"}
    elif net is None and cfg.dim == 2:
        log(f"bench: no trained weights at {wpath}; learned variant not timed")
    if cfg.dim == 2:
        rl = stage_kernel_roofline(cfg, plain)
        log(f"bench: stage kernel avg {rl['avg_launch_us']:.1f} us, algorithmic {rl['achieved']:.0f} GB/s "
            f"({100 * rl['achieved'] / HBM_PEAK_GBS:.1f} % of HBM peak), contract {rl['achieved_contract']:.0f} GB/s")
        roofline = {
            "bound": "hbm",
            "achieved": rl["achieved"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": rl["achieved"] / HBM_PEAK_GBS,
            "traffic": rl["traffic"],
            "kernel": rl["kernel"],
            "avg_launch_us": rl["avg_launch_us"],
            "algorithmic_bytes_per_launch": rl["min_bytes"],
            "algorithmic_bytes": "one read and one write of the state per time step (2 F 4 B per point), "
                                 "shared equally by the launches of a step",
            "launches_per_step": rl["launches_per_step"],
            "contract_bytes_per_launch": rl["contract_bytes"],
            "contract_gbs": rl["achieved_contract"],
            "contract_frac": rl["achieved_contract"] / HBM_PEAK_GBS,
            "traffic_vs_algorithmic": (rl["traffic"] / rl["min_bytes"]) if rl["traffic"] else None,
            "infinity_cache_split": MALL_NOTE,
        }
    else:
        rl = window_kernel_roofline(cfg, plain)
        log(f"bench: window kernel avg {rl['avg_launch_us']:.1f} us, {rl['achieved']:.2f} TFLOP/s FP32 "
            f"({100 * rl['achieved'] / rl['peak']:.1f} % of the vector peak), HBM {rl['hbm_gbs']:.0f} GB/s")
    gu = gain_fp64_utilisation(cfg, plain)
    log(f"bench: gain {gu['avg_us']:.0f} us, {gu['tflops']:.1f} TFLOP/s FP64 "
        f"({100 * gu['frac_of_fp64_peak']:.1f} % of peak)")
    if cfg.dim == 1:
        # the 1D member forecast keeps every row in LDS for the window and
        # takes a few per cent of a cycle; the gain (FP64 S, Cholesky of the
        # N_y x N_y matrix, solves) dominates, so it is the roofline call
        roofline = {"bound": "mfma", "achieved": gu["tflops"], "peak": FP64_PEAK_TFLOPS_MATRIX, "unit": "TFLOP/s",
                    "frac": gu["frac_of_fp64_peak"], "traffic": None,
                    "kernel": f"menkf_gain: FP64 S = Y Y^T + R on MFMA, blocked FP64 Cholesky of the "
                              f"{cfg.n_probes} x {cfg.n_probes} matrix with the solves, Z",
                    "avg_call_us": gu["avg_us"], "algorithmic_flops_per_call": gu["flops"],
                    "algorithmic_flops": "2 N_y^2 N (S) + N_y^3 / 3 (Cholesky) + 2 N_y^2 (N + 1) (solves) "
                                         "+ 2 N_y N (N + 1) (Z)",
                    "member_forecast": rl}
    ug = update_gemm_utilisation(cfg, plain)
    log(f"bench: member update {ug['avg_launch_us']:.1f} us, MFMA {ug['mfma_tflops']:.0f} TFLOP/s "
        f"({100 * ug['mfma_frac_of_bf16_peak']:.1f} % of BF16 peak), HBM {ug['hbm_gbs']:.0f} GB/s")
    out = {
        "metric": metric_for(cfg),
        "value": value,
        "unit": "cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": cfg.name, "fine": [cfg.ny, cfg.nx], "coarse": [cfg.nyc, cfg.nxc],
            "members": cfg.n_members, "probes": cfg.n_probes, "steps_per_cycle": cfg.n_obs,
            "headline_variant": headline, "status_word": status,
            "schedules": {k: {"tile": list(v["tile"]), "member_chunk": v["member_chunk"]} for k, v in tuned.items()}
            if tuned else "default",
            "precision": "FP32 stencils, FP64 innovation covariance/Cholesky/gain of x*, BF16x3 member update",
            "fields": cfg.nfields,
            "anomaly_gemm": ug,
            "gain_fp64": gu,
            "variants": variants,
        },
        "roofline": roofline,
    }
    if args.cpu_baseline and not args.small:
        log("bench: timing the oracle on the host (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
