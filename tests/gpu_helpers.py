"""Shared helpers for the GPU tests (marshalling between numpy and the binding)."""

import sys

import numpy as np
import torch

from synthetic import fields


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def to_dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype).contiguous()


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def make_ctx(cfg):
    from paper_2012_10091_amd import Context
    ctx = Context(cfg)
    idx, comp = fields.probes_for(cfg)
    ctx.set_probes(torch.as_tensor(idx, dtype=torch.int32, device="cuda"),
                   torch.as_tensor(comp, dtype=torch.int32, device="cuda"))
    return ctx, idx, comp
