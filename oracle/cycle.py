"""One MEnKF assimilation cycle (Algo. 4 with the state part of Algo. 3).

Per cycle (an analysis every ``n_obs`` time steps; the workloads have no
model parameters, so the parameter steps of the dual filter are inactive):

  1. fine forecast   x^F_f = M^F(x^F_a), n_obs explicit steps; keep x^F_{k-1}
  2. member forecast x^(i) = M^C(x^(i)), n_obs explicit steps, same dt
  3. x* = Pi_C(x^F_f)
  4. EnKF analysis on the coarse members and delta^C = K (y^o - H^C(x*))
  5. x' = x^F_f + Pi_F(delta^C)
  6. n_s relaxed Jacobi sweeps (alpha = 0.5) -> x^F_a
  7. optional fine-to-coarse feedback: members recentred on Pi_C(x^F_a)

``n_sweeps = 0`` is the multilevel EnKF without regularisation that the
paper also discusses (Sec. 3) and uses as its "classical Dual EnKF on the
coarse grid" comparison (Sec. 6).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import enkf, grids, obs, rng, smooth
from .models import Model


@dataclasses.dataclass
class State:
    fine: np.ndarray       # (F, [ny,] nx)
    members: np.ndarray    # (N, F, [nyc,] nxc)
    cycle: int = 0


def make_H(cfg, idx, comp):
    def H(xc):
        return obs.observe_coarse(xc, idx, comp, cfg.dim, cfg.ratio, cfg.nx)
    return H


def observe_truth(cfg, truth, idx, comp):
    return obs.observe_fine(truth, idx, comp, cfg.dim)


def recentre(members, fine, cfg):
    """Fine-to-coarse feedback (the paper's closing section names driving the
    coarse ensemble by the fine-grid analysis as future work): shift the
    members so that their mean is Pi_C(x^F_a), keeping every anomaly:
    x^(i) <- x^(i) - mean_i x^(i) + Pi_C(x^F_a)."""
    target = grids.restrict(fine, cfg.ratio, cfg.dim)
    return members - members.mean(axis=0, keepdims=True) + target[None]


def cycle(cfg, st: State, y_obs, idx, comp, n_sweeps=1, alpha=0.5, eps=None,
          seed=None, mode="exact_r", return_parts=False, feedback=False):
    fine_model = Model(cfg, "fine")
    coarse_model = Model(cfg, "coarse")
    xf, xf_prev = fine_model.forecast(st.fine, cfg.n_obs)
    mem_f, _ = coarse_model.forecast(st.members, cfg.n_obs)
    xstar = grids.restrict(xf, cfg.ratio, cfg.dim)
    c = st.cycle + 1
    if eps is None:
        eps = rng.perturbations(cfg.seed + 5 if seed is None else seed, c,
                                cfg.n_members, cfg.n_probes, cfg.obs_sigma)
    res = enkf.analysis(mem_f, xstar, y_obs, eps, make_H(cfg, idx, comp), cfg.obs_sigma, mode=mode)
    x = xf + grids.prolong(res["delta"], cfg.ratio, cfg.dim)
    x = smooth.smooth(x, xf_prev, fine_model, n_sweeps, alpha)
    members = recentre(res["members"], x, cfg) if feedback else res["members"]
    new = State(fine=x, members=members, cycle=c)
    if return_parts:
        return new, {"xf": xf, "xf_prev": xf_prev, "members_f": mem_f, "xstar": xstar,
                     "eps": eps, **res}
    return new


def free_run(cfg, fine, n_cycles):
    m = Model(cfg, "fine")
    out = []
    for _ in range(n_cycles):
        fine, _ = m.forecast(fine, cfg.n_obs)
        out.append(fine)
    return out
