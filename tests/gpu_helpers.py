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


def bf16_round(a):
    """Round to BF16 (nearest, ties to even) through FP32, returned as FP64:
    the storage rounding of the GPU path's BF16 activations and weights."""
    x = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


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
