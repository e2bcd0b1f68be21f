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


def load(path: str, guard=10.0, device="cuda", judge_every=0, judge_tol=None) -> B.Net:
    """A committed network; judge_tol defaults to the tolerance stored with
    the weights (1.0 when none is)."""
    z = np.load(path, allow_pickle=False)
    if judge_tol is None:
        judge_tol = float(z["judge_tol"]) if "judge_tol" in z.files else 1.0
    return B.Net(z["params"], z["in_scale"], z["in_offset"], z["out_scale"], guard=guard, device=device,
                 judge_every=judge_every, judge_tol=judge_tol)


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


def train_flops_per_crop(crop: int) -> float:
    """Useful arithmetic of one training crop (forward, data and weight
    gradients): the three valid convolutions on (C+4)^2, (C+2)^2 and C^2
    output pixels, 2 flops per multiply-add, backward about twice the
    forward (no data gradient for the input layer)."""
    fwd = 2.0 * (9 * 8 * 32 * (crop + 4) ** 2 + 9 * 32 * 32 * (crop + 2) ** 2 + 9 * 32 * 4 * crop ** 2)
    bwd_w = fwd
    bwd_d = 2.0 * (9 * 32 * 32 * (crop + 2) ** 2 + 9 * 32 * 4 * crop ** 2)
    return fwd + bwd_w + bwd_d


def train_streamed(cfg, net: B.Net, n_pairs=20000, ring=1024, n_parallel=8, cycles_per_run=120,
                   steps_per_pair=0.25, batch=16, crop=128, lr=1e-3, n_sweeps=3, seed=0, relative=True,
                   log=print):
    """Train on pairs that plain MEnKF runs generate while training goes on.

    n_parallel independent runs (own seeds: truth, model and member initial
    conditions, probes, noise) are advanced cycle by cycle; every analysis
    gives one pair (inputs Pi_F(delta^C) and x^F_f, target the plain fine
    correction x^F_a - x^F_f after Pi_F and n_sweeps sweeps), written into a
    device ring buffer of `ring` pairs, so the n_pairs pairs are never
    stored together.  A run is replaced by a fresh one after cycles_per_run
    cycles, so the pairs cover whole assimilation runs.  Adam steps on
    random periodic crops of the pairs in the ring are interleaved, about
    steps_per_pair per new pair, with a cosine learning-rate decay.  With
    relative, a pair is drawn with probability proportional to
    1 / |target|^2, so the expected loss is the mean squared error relative
    to each pair's own correction (the measure of the judge), and the small
    corrections of late cycles weigh as much as the first analyses' large
    ones.  Returns the loss history and the throughput record."""
    from synthetic import fields
    shape = (4, cfg.ny, cfg.nx)
    f32 = torch.float32
    ring = min(ring, n_pairs)
    dp = torch.zeros((ring,) + shape, dtype=f32, device="cuda")
    xr = torch.zeros_like(dp)
    tg = torch.zeros_like(dp)
    tnorm = torch.ones(ring, dtype=torch.float64, device="cuda")
    made, filled, steps, next_seed = 0, 0, 0, 0
    total_steps = max(1, int(round(n_pairs * steps_per_pair)))

    def new_run():
        nonlocal next_seed
        next_seed += 1
        rc = cfg.with_(seed=cfg.seed + 1000 * next_seed)
        return Run(rc, fields.truth_ic(rc), fields.model_ic(rc), fields.member_ics(rc), fields.probes_for(rc),
                   lambda c, rc=rc: fields.obs_noise(rc, c), n_sweeps=n_sweeps)

    runs = [new_run() for _ in range(n_parallel)]
    tr = B.Trainer(net, batch=batch, crop=crop, lr=lr)
    g = np.random.default_rng(seed)
    lr_min = lr * 0.01
    hist = []
    t_gen = t_train = 0.0
    n_runs = n_parallel
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while made < n_pairs:
        ta = time.perf_counter()
        for i in range(len(runs)):
            if made >= n_pairs:
                break
            run = runs[i]
            run.forecast_and_gain()
            k = made % ring
            xr[k].copy_(run.fine)
            dp[k].zero_()
            run.ctx.prolong_smooth(run.dc, dp[k], None, n_sweeps=0)
            run.correct(B.MENKF_PROLONG_PLAIN)
            torch.sub(run.fine, xr[k], out=tg[k])
            tnorm[k] = torch.linalg.vector_norm(tg[k].double())
            made += 1
            filled = min(filled + 1, ring)
            if run.cycle >= cycles_per_run:
                if run.ctx.get_status() != 0:
                    raise RuntimeError("analysis failed while generating pairs")
                runs[i] = new_run()
                n_runs += 1
        torch.cuda.synchronize()
        tb = time.perf_counter()
        t_gen += tb - ta
        if relative:
            w = 1.0 / np.maximum(tnorm[:filled].cpu().numpy(), 1e-30) ** 2
            w /= w.sum()
        while steps < total_steps * made / n_pairs:
            tr.lr = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * steps / total_steps))
            pick = g.choice(filled, batch, p=w) if relative else g.integers(0, filled, batch)
            crops = np.stack([pick, g.integers(0, cfg.ny, batch), g.integers(0, cfg.nx, batch)], axis=1)
            loss = tr.step(dp, xr, tg, torch.as_tensor(crops.astype(np.int32), device="cuda"))
            if steps % 250 == 0 or steps == total_steps - 1:
                hist.append((steps, float(loss.item())))
                log(f"train: pairs {made} step {steps} loss {hist[-1][1]:.4e}")
            steps += 1
        torch.cuda.synchronize()
        t_train += time.perf_counter() - tb
    wall = time.perf_counter() - t0
    fl = train_flops_per_crop(crop) * batch * steps
    rec = {"pairs": made, "runs": n_runs, "ring": ring, "adam_steps": steps, "batch": batch, "crop": crop,
           "relative_sampling": int(relative),
           "wall_s": wall, "generation_s": t_gen, "training_s": t_train,
           "pairs_per_s": made / t_gen, "adam_steps_per_s": steps / t_train,
           "training_crops_per_s": steps * batch / t_train, "training_tflops": fl / t_train / 1e12,
           "workload": cfg.name}
    log(f"train: {rec}")
    return hist, rec


def evaluate(cfg, net: B.Net, n_cycles=100, seed_offset=9000, n_sweeps=3, judge_every=10, log=print):
    """Held-out runs (unseen seeds) of the plain and the learned MEnKF.

    The learned run uses LEARNED_FALLBACK with the judge (every judge_every
    cycles the plain correction is formed and compared).  Returns the
    second-half mean velocity RMSE of both runs, and on the plain run the
    distance of the network's and of the sweep-free (Pi_F only) corrections
    to the plain correction (relative L2, mean and the values at every
    tenth cycle), the conservativity indicator Gamma (Sec. 6) of the three,
    and the learned run's judge counts."""
    from synthetic import fields
    rc = cfg.with_(seed=cfg.seed + seed_offset)
    args = (rc, fields.truth_ic(rc), fields.model_ic(rc), fields.member_ics(rc), fields.probes_for(rc),
            lambda c: fields.obs_noise(rc, c))
    plain = Run(*args, n_sweeps=n_sweeps)
    learned = Run(*args, n_sweeps=n_sweeps)
    net.judge_stats.zero_()
    every, net.judge_every = net.judge_every, judge_every
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
        learned.ctx.prolong_smooth(learned.dc, learned.fine, learned.prev, n_sweeps=n_sweeps, alpha=0.5,
                                   mode=B.MENKF_PROLONG_LEARNED_FALLBACK, net=net)
        ref = plain.fine - xf
        nrm = torch.linalg.vector_norm(ref)
        d_net.append(float(torch.linalg.vector_norm(nn - plain.fine) / nrm))
        d_pif.append(float(torch.linalg.vector_norm(pif - plain.fine) / nrm))
        gam["plain"].append(gamma_rms(plain.fine, plain.prev))
        gam["learned"].append(gamma_rms(nn, plain.prev))
        gam["pif"].append(gamma_rms(pif, plain.prev))
        rm_p.append(plain.velocity_rmse())
        rm_l.append(learned.velocity_rmse())
    net.judge_every = every
    st = net.judge_stats.cpu().numpy()
    half = n_cycles // 2
    res = {"plain_rmse": float(np.mean(rm_p[half:])), "learned_rmse": float(np.mean(rm_l[half:])),
           "net_vs_plain_correction": float(np.mean(d_net)),
           "net_vs_plain_correction_every_10": [round(v, 4) for v in d_net[9::10]],
           "pif_vs_plain_correction": float(np.mean(d_pif)),
           "gamma_plain": float(np.mean(gam["plain"])), "gamma_learned": float(np.mean(gam["learned"])),
           "gamma_pif": float(np.mean(gam["pif"])), "cycles": n_cycles,
           "judged": int(st[1]), "plain_corrected_cycles": int(st[2]), "guarded_cycles": int(st[3])}
    res["ratio"] = res["learned_rmse"] / res["plain_rmse"]
    log(f"evaluate: {res}")
    return res


def main(argv=None):
    from synthetic import configs
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="C4", choices=["C3", "C4"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--ring", type=int, default=1024)
    ap.add_argument("--parallel", type=int, default=8)
    ap.add_argument("--cycles-per-run", type=int, default=120)
    ap.add_argument("--steps-per-pair", type=float, default=0.25)
    ap.add_argument("--eval-cycles", type=int, default=100)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--crop", type=int, default=128)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--judge-tol", type=float, default=1.0)
    ap.add_argument("--uniform", action="store_true", help="draw pairs uniformly instead of by 1/|target|^2")
    args = ap.parse_args(argv)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    cfg = configs.CONFIGS[args.workload]
    out = args.out or weights_for(cfg.name)
    s, o, os_ = default_scaling(cfg.gamma, cfg.mach)
    net = B.Net(init_params(seed=cfg.seed), s, o, os_, judge_tol=args.judge_tol)
    hist, rec = train_streamed(cfg, net, n_pairs=args.pairs, ring=args.ring, n_parallel=args.parallel,
                               cycles_per_run=args.cycles_per_run, steps_per_pair=args.steps_per_pair,
                               batch=args.batch, crop=args.crop, lr=args.lr, relative=not args.uniform, log=log)
    torch.cuda.empty_cache()
    ev = evaluate(cfg, net, n_cycles=args.eval_cycles, log=log)
    meta = {"loss_history": np.array(hist), "pairs": rec["pairs"], "runs": rec["runs"],
            "cycles_per_run": args.cycles_per_run, "adam_steps": rec["adam_steps"],
            "crop_samples": rec["adam_steps"] * args.batch, "workload": cfg.name, "judge_tol": args.judge_tol,
            **{f"train_{k}": v for k, v in rec.items() if isinstance(v, (int, float))},
            **{f"eval_{k}": v for k, v in ev.items()}}
    save(net, out, meta)
    log(f"saved {out}")


if __name__ == "__main__":
    main()
