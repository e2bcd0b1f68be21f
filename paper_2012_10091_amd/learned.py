"""Training driver of the learned prolongation (GPU, through the C ABI).

Pairs come from the plain MEnKF itself: at every analysis of a run, the
inputs are Pi_F(delta^C) and the fine forecast x^F_f, and the target is the
plain fine correction x^F_a - x^F_f after Pi_F and the relaxed sweeps
(distillation of prolongation + smoothing).  Training samples random
periodic crops of these fields with Adam.  Everything numeric runs in
libmenkf; this module only orchestrates runs and stores parameters
(numpy .npz, no pickling).

    python -m paper_2012_10091_amd.learned --out weights.npz
"""

from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np
import torch

from . import binding as B

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
DEFAULT_WEIGHTS = os.path.join(WEIGHTS_DIR, "ns2d_1024_learned_prolong.npz")


def weights_for(workload_name: str) -> str:
    """Committed weights trained on the workload's own grid (fine side in the name)."""
    side = "512" if "_512_" in workload_name else "1024"
    return os.path.join(WEIGHTS_DIR, f"ns2d_{side}_learned_prolong.npz")


def default_scaling(gamma=1.4, mach=0.3):
    """Fixed per-field affine input maps (rho, rho u, rho v, E) and output scale."""
    p0 = 1.0 / (gamma * mach * mach)
    e0 = p0 / (gamma - 1.0)
    d_scale = [100.0, 20.0, 20.0, 10.0]
    in_scale = d_scale + [10.0, 1.0, 1.0, 1.0]
    in_offset = [0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, e0]
    return in_scale, in_offset, list(d_scale)


def init_params(seed=2012, last_gain=0.0):
    """He-initialised hidden layers; last layer scaled by last_gain (0 = plain prolongation)."""
    rng = np.random.default_rng(seed)

    def he(o, c):
        return rng.standard_normal((o, c, 3, 3)) * math.sqrt(2.0 / (9 * c))
    w1, w2 = he(32, 8), he(32, 32)
    w3 = he(4, 32) * last_gain
    return B.pack_params([w1, np.zeros(32), w2, np.zeros(32), w3, np.zeros(4)])


def save(net: B.Net, path: str, meta: dict):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=net.params.detach().cpu().numpy(), in_scale=np.array(net.in_scale),
             in_offset=np.array(net.in_offset), out_scale=np.array(net.out_scale),
             **{k: np.array(v) for k, v in meta.items()})


def load(path: str, guard=10.0, device="cuda") -> B.Net:
    z = np.load(path, allow_pickle=False)
    return B.Net(z["params"], z["in_scale"], z["in_offset"], z["out_scale"], guard=guard, device=device)


class Run:
    """One assimilation run on the device (plain or learned prolongation)."""

    def __init__(self, cfg, truth_ic, model_ic, member_ics, probes, obs_noise, n_sweeps=3):
        self.cfg = cfg
        self.ctx = B.Context(cfg)
        idx, comp = probes
        self.ctx.set_probes(torch.as_tensor(idx, device="cuda"), torch.as_tensor(comp, device="cuda"))
        f32 = torch.float32
        self.truth = torch.as_tensor(truth_ic, dtype=f32, device="cuda").contiguous()
        self.fine = torch.as_tensor(model_ic, dtype=f32, device="cuda").contiguous()
        self.members = torch.as_tensor(member_ics, dtype=f32, device="cuda").contiguous()
        self.prev = torch.empty_like(self.fine)
        self.xs = torch.empty((4, cfg.nyc, cfg.nxc), dtype=f32, device="cuda")
        self.dc = torch.empty_like(self.xs)
        self.obs_noise = obs_noise
        self.n_sweeps = n_sweeps
        self.cycle = 0
        self.diag = torch.zeros(3, dtype=torch.float64, device="cuda")

    def forecast_and_gain(self):
        c, cfg = self.ctx, self.cfg
        self.cycle += 1
        c.forecast(B.MENKF_FINE, self.truth, cfg.n_obs)
        y = c.observe(B.MENKF_FINE, self.truth)[0] + torch.as_tensor(self.obs_noise(self.cycle), device="cuda")
        c.forecast(B.MENKF_FINE, self.fine, cfg.n_obs, prev=self.prev)
        c.forecast(B.MENKF_COARSE, self.members, cfg.n_obs)
        c.restrict(self.fine, self.xs)
        c.gain(self.members, self.xs, y, cfg.seed + 5, self.cycle)
        c.update(self.members, self.dc)

    def correct(self, mode=B.MENKF_PROLONG_PLAIN, net=None):
        self.ctx.prolong_smooth(self.dc, self.fine, self.prev, n_sweeps=self.n_sweeps if mode != 1 else 0,
                                alpha=0.5, mode=mode, net=net)

    def velocity_rmse(self) -> float:
        self.ctx.diagnostics(self.fine, self.truth, out=self.diag)
        d = self.diag.cpu().numpy()
        return float(math.sqrt(d[0] / d[1]))


def generate_pairs(cfg, n_runs, cycles_per_run, skip=2, n_sweeps=3, log=print):
    """(dproj, xf, target) fields from plain MEnKF runs, stacked on the device."""
    from synthetic import fields
    dps, xfs, tgs = [], [], []
    for run_i in range(n_runs):
        rc = cfg.with_(seed=cfg.seed + 1000 * (run_i + 1))
        run = Run(rc, fields.truth_ic(rc), fields.model_ic(rc), fields.member_ics(rc), fields.probes_for(rc),
                  lambda c, rc=rc: fields.obs_noise(rc, c), n_sweeps=n_sweeps)
        zero = torch.zeros_like(run.fine)
        for c in range(cycles_per_run):
            run.forecast_and_gain()
            xf = run.fine.clone()
            dproj = zero.clone()
            run.ctx.prolong_smooth(run.dc, dproj, None, n_sweeps=0)
            run.correct(B.MENKF_PROLONG_PLAIN)
            if c >= skip:
                dps.append(dproj)
                xfs.append(xf)
                tgs.append(run.fine - xf)
        if run.ctx.get_status() != 0:
            raise RuntimeError("analysis failed while generating pairs")
        log(f"pairs: run {run_i + 1}/{n_runs} done, rmse {run.velocity_rmse():.4f}")
    return (torch.stack(dps).contiguous(), torch.stack(xfs).contiguous(), torch.stack(tgs).contiguous())


def evaluate(cfg, net: B.Net, n_cycles=40, seed_offset=9000, n_sweeps=3, log=print):
    """Held-out runs (unseen seeds) of the plain and the learned MEnKF.

    Returns the second-half mean velocity RMSE of both runs and, on the
    plain run, how far the learned and the sweep-free (Pi_F only)
    corrections are from the plain correction (relative L2, averaged)."""
    from synthetic import fields
    rc = cfg.with_(seed=cfg.seed + seed_offset)
    args = (rc, fields.truth_ic(rc), fields.model_ic(rc), fields.member_ics(rc), fields.probes_for(rc),
            lambda c: fields.obs_noise(rc, c))
    plain = Run(*args, n_sweeps=n_sweeps)
    learned = Run(*args, n_sweeps=n_sweeps)
    rm_p, rm_l, d_net, d_pif = [], [], [], []
    gam = {"plain": [], "learned": [], "pif": []}
    res_buf = torch.empty_like(plain.fine)

    def gamma_rms(x, prev):
        # Gamma of the transversal momentum (Sec. 6): -(x_{k-1} + dt F(x) - x)/dt on rho v
        plain.ctx.residual(x, prev, out=res_buf)
        return float(torch.linalg.vector_norm(res_buf[2]) / math.sqrt(res_buf[2].numel()) / cfg.dt)

    for c in range(n_cycles):
        for r in (plain, learned):
            r.forecast_and_gain()
        xf = plain.fine.clone()
        pif = xf.clone()
        plain.ctx.prolong_smooth(plain.dc, pif, None, n_sweeps=0)
        nn = xf.clone()
        plain.ctx.prolong_smooth(plain.dc, nn, None, n_sweeps=0, mode=B.MENKF_PROLONG_LEARNED, net=net)
        plain.correct(B.MENKF_PROLONG_PLAIN)
        learned.correct(B.MENKF_PROLONG_LEARNED, net=net)
        ref = plain.fine - xf
        nrm = torch.linalg.vector_norm(ref)
        d_net.append(float(torch.linalg.vector_norm(nn - plain.fine) / nrm))
        d_pif.append(float(torch.linalg.vector_norm(pif - plain.fine) / nrm))
        gam["plain"].append(gamma_rms(plain.fine, plain.prev))
        gam["learned"].append(gamma_rms(nn, plain.prev))
        gam["pif"].append(gamma_rms(pif, plain.prev))
        rm_p.append(plain.velocity_rmse())
        rm_l.append(learned.velocity_rmse())
    half = n_cycles // 2
    res = {"plain_rmse": float(np.mean(rm_p[half:])), "learned_rmse": float(np.mean(rm_l[half:])),
           "net_vs_plain_correction": float(np.mean(d_net)), "pif_vs_plain_correction": float(np.mean(d_pif)),
           "gamma_plain": float(np.mean(gam["plain"])), "gamma_learned": float(np.mean(gam["learned"])),
           "gamma_pif": float(np.mean(gam["pif"])), "cycles": n_cycles}
    res["ratio"] = res["learned_rmse"] / res["plain_rmse"]
    log(f"evaluate: {res}")
    return res


def train(net: B.Net, pairs, steps, batch=16, crop=128, lr=1e-3, seed=0, log=print):
    dproj, xf, target = pairs
    P, _, H, W = dproj.shape
    tr = B.Trainer(net, batch=batch, crop=crop, lr=lr)
    g = np.random.default_rng(seed)
    hist = []
    lr_min = lr * 0.01
    for s in range(steps):
        tr.lr = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * s / steps))   # cosine decay
        crops = np.stack([g.integers(0, P, batch), g.integers(0, H, batch), g.integers(0, W, batch)], axis=1)
        loss = tr.step(dproj, xf, target, torch.as_tensor(crops.astype(np.int32), device="cuda"))
        if s % 100 == 0 or s == steps - 1:
            hist.append((s, float(loss.item())))
            log(f"train: step {s} loss {hist[-1][1]:.4e}")
    return hist


def main(argv=None):
    from synthetic import configs
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="C4", choices=["C3", "C4"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--runs", type=int, default=4)
    ap.add_argument("--cycles", type=int, default=34)
    ap.add_argument("--eval-cycles", type=int, default=40)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--crop", type=int, default=128)
    ap.add_argument("--lr", type=float, default=1e-3)
    args = ap.parse_args(argv)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    cfg = configs.CONFIGS[args.workload]
    out = args.out or weights_for(cfg.name)
    t0 = time.perf_counter()
    pairs = generate_pairs(cfg, args.runs, args.cycles, log=log)
    log(f"pairs: {pairs[0].shape[0]} fields of {tuple(pairs[0].shape[1:])} in {time.perf_counter() - t0:.1f}s")
    s, o, os_ = default_scaling(cfg.gamma, cfg.mach)
    net = B.Net(init_params(seed=cfg.seed), s, o, os_)
    t1 = time.perf_counter()
    hist = train(net, pairs, args.steps, args.batch, args.crop, args.lr, log=log)
    torch.cuda.synchronize()
    log(f"train: {args.steps} steps x {args.batch} crops of {args.crop}^2 in {time.perf_counter() - t1:.1f}s")
    del pairs
    ev = evaluate(cfg, net, n_cycles=args.eval_cycles, log=log)
    save(net, out, {"loss_history": np.array(hist), "pairs": args.runs * (args.cycles - 2),
                    "crop_samples": args.steps * args.batch, "workload": cfg.name,
                    **{f"eval_{k}": v for k, v in ev.items()}})
    log(f"saved {out}")


if __name__ == "__main__":
    main()
