"""Counter-based random numbers for the perturbed observations.

The stochastic EnKF draws eps^(i) ~ N(0, R) for every member (perturbed
observations, Sec. 2.1.2; Algo. 1 step 2, Algo. 3 step 3).  The paper does
not say how.  Reading: Philox4x32 with 10 rounds (Salmon, Moraes, Dror &
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) and the
Box-Muller transform (1958) in FP64, so that the CPU and GPU produce the
same draws from their own implementations.

Draw convention (member i, probe p, cycle c, 64-bit seed s):
  key     = (s mod 2^32, s >> 32)
  counter = (p >> 1, i, c mod 2^32, 0x5045)
  (r0, r1, r2, r3) = Philox4x32-10(counter, key)
  u1 = ((r0 >> 5) 2^26 + (r1 >> 6) + 1/2) 2^-53,  u2 likewise from (r2, r3)
  z0 = sqrt(-2 ln u1) cos(2 pi u2),  z1 = sqrt(-2 ln u1) sin(2 pi u2)
  eps[i, p] = sigma * (z0 if p is even else z1)
"""

from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF
STREAM_PERTURB = 0x5045


def philox4x32_10(ctr, key):
    """Philox4x32-10 on arrays of counters.

    ``ctr`` is a sequence of four uint-valued arrays, ``key`` two; returns
    four uint64 arrays holding 32-bit outputs.  Round: the products
    M0*c0 and M1*c2 split into hi/lo words; new counter
    (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); key bumped by the Weyl
    constants (W0, W1) between rounds.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) & MASK for k in key)
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(W0)) & MASK
            k1 = (k1 + np.uint64(W1)) & MASK
        p0 = c0 * m0                      # < 2^64, exact in uint64
        p1 = c2 * m1
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return c0, c1, c2, c3


def _u53(a, b):
    k = (a >> np.uint64(5)).astype(np.float64) * 67108864.0 + (b >> np.uint64(6)).astype(np.float64)
    return (k + 0.5) * (2.0 ** -53)


def perturbations(seed: int, cycle: int, n_members: int, n_probes: int, sigma: float):
    """eps[i, p] ~ N(0, sigma^2), shape (n_members, n_probes), FP64."""
    i = np.arange(n_members, dtype=np.uint64)[:, None]
    p = np.arange(n_probes, dtype=np.uint64)[None, :]
    shape = (n_members, n_probes)
    ctr = (np.broadcast_to(p >> np.uint64(1), shape),
           np.broadcast_to(i, shape),
           np.full(shape, cycle & MASK, dtype=np.uint64),
           np.full(shape, STREAM_PERTURB, dtype=np.uint64))
    key = (np.uint64(seed & MASK), np.uint64((seed >> 32) & MASK))
    r0, r1, r2, r3 = philox4x32_10(ctr, key)
    u1 = _u53(r0, r1)
    u2 = _u53(r2, r3)
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.where((p % np.uint64(2)) == 0, rad * np.cos(2.0 * np.pi * u2), rad * np.sin(2.0 * np.pi * u2))
    return sigma * z
