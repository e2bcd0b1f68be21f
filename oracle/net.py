"""Learned convolutional prolongation (not in the paper; the paper's closing
section names better coarse-to-fine projectors as future work).

Network: conv3x3(8->32) -> ReLU -> conv3x3(32->32) -> ReLU -> conv3x3(32->4),
circular padding (periodic domain), cross-correlation convention

  out[o, y, x] = b[o] + sum_{c, a, b} w[o, c, a, b] in[c, (y + a - 1) mod H, (x + b - 1) mod W].

Input (8 channels): the prolonged coarse correction Pi_F(delta^C) and the
fine forecast x^F_f, each field mapped by a fixed affine scaling
(v - offset) * scale.  Output (4 channels): a residual on top of
Pi_F(delta^C) in units of 1/out_scale, so the fine correction is
Pi_F(delta^C) + out / out_scale; a zero last layer reproduces the plain
prolongation exactly.  Loss: mean squared error over channels and pixels of
the scaled residual.  Optimiser: Adam (Kingma & Ba 2015).

FP64 explicit loops over the nine taps; batch dimension optional.
"""

from __future__ import annotations

import dataclasses

import numpy as np

CH = (8, 32, 32, 4)


@dataclasses.dataclass
class Params:
    w1: np.ndarray
    b1: np.ndarray
    w2: np.ndarray
    b2: np.ndarray
    w3: np.ndarray
    b3: np.ndarray
    in_scale: np.ndarray    # (8,)
    in_offset: np.ndarray   # (8,)
    out_scale: np.ndarray   # (4,)

    def tensors(self):
        return [self.w1, self.b1, self.w2, self.b2, self.w3, self.b3]


def default_scaling(cfg):
    """Fixed per-field affine input maps for the 2D conservative fields."""
    p0 = 1.0 / (cfg.gamma * cfg.mach ** 2)
    e0 = p0 / (cfg.gamma - 1.0)
    d_scale = np.array([100.0, 20.0, 20.0, 10.0])
    x_scale = np.array([10.0, 1.0, 1.0, 1.0])
    x_off = np.array([1.0, 0.0, 0.0, e0])
    in_scale = np.concatenate([d_scale, x_scale])
    in_offset = np.concatenate([np.zeros(4), x_off])
    return in_scale, in_offset, d_scale.copy()


def init_params(cfg, seed=2012, zero_last=True):
    rng = np.random.default_rng(seed)

    def he(o, c):
        return rng.standard_normal((o, c, 3, 3)) * np.sqrt(2.0 / (9 * c))
    w3 = np.zeros((4, 32, 3, 3)) if zero_last else he(4, 32) * 0.1
    s, o, os_ = default_scaling(cfg)
    return Params(he(32, 8), np.zeros(32), he(32, 32), np.zeros(32), w3, np.zeros(4), s, o, os_)


def _shift(x, a, b):
    """x[..., (y + a - 1) mod H, (x + b - 1) mod W]."""
    return np.roll(np.roll(x, -(a - 1), axis=-2), -(b - 1), axis=-1)


def conv(x, w, b):
    out = np.zeros(x.shape[:-3] + (w.shape[0],) + x.shape[-2:])
    for a in range(3):
        for bb in range(3):
            out += np.einsum("oc,...chw->...ohw", w[:, :, a, bb], _shift(x, a, bb))
    return out + b[:, None, None]


def conv_backward(x, w, g):
    """Gradients of conv(x, w, b) given upstream g: (dx, dw, db)."""
    dw = np.zeros_like(w)
    dx = np.zeros_like(x)
    for a in range(3):
        for bb in range(3):
            xs = _shift(x, a, bb)
            dw[:, :, a, bb] = np.einsum("bohw,bchw->oc", g.reshape((-1,) + g.shape[-3:]),
                                        xs.reshape((-1,) + xs.shape[-3:]))
            # d in[c, y', x'] gets w[o,c,a,b] g[o, y'-a+1, x'-b+1]
            gs = np.roll(np.roll(g, a - 1, axis=-2), bb - 1, axis=-1)
            dx += np.einsum("oc,...ohw->...chw", w[:, :, a, bb], gs)
    db = g.sum(axis=tuple(range(g.ndim - 3)) + (-2, -1))
    return dx, dw, db


def make_input(params: Params, dproj, xf):
    """Scaled 8-channel input from Pi_F(delta^C) and x^F_f, each (..., 4, H, W)."""
    raw = np.concatenate([np.asarray(dproj, dtype=np.float64), np.asarray(xf, dtype=np.float64)], axis=-3)
    return (raw - params.in_offset[:, None, None]) * params.in_scale[:, None, None]


def forward(params: Params, inp):
    z1 = conv(inp, params.w1, params.b1)
    a1 = np.maximum(z1, 0.0)
    z2 = conv(a1, params.w2, params.b2)
    a2 = np.maximum(z2, 0.0)
    out = conv(a2, params.w3, params.b3)
    return out, (inp, z1, a1, z2, a2)


def backward(params: Params, cache, gout):
    inp, z1, a1, z2, a2 = cache
    da2, dw3, db3 = conv_backward(a2, params.w3, gout)
    dz2 = da2 * (z2 > 0)
    da1, dw2, db2 = conv_backward(a1, params.w2, dz2)
    dz1 = da1 * (z1 > 0)
    dinp, dw1, db1 = conv_backward(inp, params.w1, dz1)
    return [dw1, db1, dw2, db2, dw3, db3], dinp


def mse(out, target):
    diff = out - target
    n = diff.size
    return float(np.sum(diff * diff) / n), 2.0 * diff / n


def target_residual(params: Params, dproj, correction):
    """Scaled training target: (correction - Pi_F delta) * out_scale."""
    return (np.asarray(correction) - np.asarray(dproj)) * params.out_scale[:, None, None]


def learned_correction(params: Params, dproj, xf):
    out, _ = forward(params, make_input(params, dproj, xf))
    return np.asarray(dproj, dtype=np.float64) + out / params.out_scale[:, None, None]


def adam_update(tensors, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place; ``t`` is the 1-based step count."""
    for p, g, mm, vv in zip(tensors, grads, m, v):
        mm *= beta1
        mm += (1.0 - beta1) * g
        vv *= beta2
        vv += (1.0 - beta2) * g * g
        mhat = mm / (1.0 - beta1 ** t)
        vhat = vv / (1.0 - beta2 ** t)
        p -= lr * mhat / (np.sqrt(vhat) + eps)
