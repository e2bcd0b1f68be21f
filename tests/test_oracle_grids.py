"""Pins of the oracle's projection operators against what the definition of a
fourth-order Lagrange interpolator on nested periodic grids fixes."""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import grids


def _golden_weights(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "lagrange4_weights.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows.append((float(Fraction(parts[0])), [float(Fraction(p)) for p in parts[1:]]))
    return rows


def test_lagrange_weights_match_exact_rationals(golden_dir):
    for s, w in _golden_weights(golden_dir):
        np.testing.assert_allclose(grids.lagrange4_weights(s), w, rtol=0, atol=1e-15)


@pytest.mark.parametrize("s", [0.0, 0.25, 0.5, 0.75, 0.3])
def test_lagrange_reproduces_cubics(s):
    w = grids.lagrange4_weights(s)
    nodes = np.array([-1.0, 0.0, 1.0, 2.0])
    for p in range(4):
        assert abs(np.dot(w, nodes ** p) - s ** p) < 1e-14
    assert abs(w.sum() - 1.0) < 1e-15


@pytest.mark.parametrize("ratio", [1, 2, 4, 8])
def test_restrict_after_prolong_is_identity(ratio):
    rng = np.random.default_rng(0)
    xc1 = rng.standard_normal((3, 16))
    np.testing.assert_array_equal(grids.restrict(grids.prolong(xc1, ratio, 1), ratio, 1), xc1)
    xc2 = rng.standard_normal((2, 12, 10))
    np.testing.assert_array_equal(grids.restrict(grids.prolong(xc2, ratio, 2), ratio, 2), xc2)


def test_prolong_reproduces_cubic_polynomial_in_interior():
    ratio, nc = 4, 32
    X = np.arange(nc, dtype=float)           # coarse coordinate in coarse cells
    p = lambda t: 0.3 - 1.2 * t + 0.05 * t ** 2 + 0.002 * t ** 3
    xf = grids.prolong(p(X), ratio, 1)
    t = np.arange(nc * ratio) / ratio
    interior = (t >= 1) & (t <= nc - 3)      # stencil does not wrap
    np.testing.assert_allclose(xf[interior], p(t[interior]), rtol=0, atol=1e-11)


def test_prolong_conserves_integral_on_periodic_grid():
    rng = np.random.default_rng(1)
    ratio = 4
    xc = rng.standard_normal((10, 14))
    xf = grids.prolong(xc, ratio, 2)
    hc, hf = 1.0, 1.0 / ratio
    assert abs(xf.sum() * hf * hf - xc.sum() * hc * hc) < 1e-12
    x1 = rng.standard_normal(40)
    assert abs(grids.prolong(x1, ratio, 1).sum() * hf - x1.sum() * hc) < 1e-12


def test_prolong_fourth_order_convergence():
    errs = []
    for nc in (16, 32, 64):
        X = np.arange(nc) * 2 * math.pi / nc
        xf = grids.prolong(np.sin(X), 4, 1)
        x = np.arange(4 * nc) * 2 * math.pi / (4 * nc)
        errs.append(np.max(np.abs(xf - np.sin(x))))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.7 < o < 4.3 for o in orders), orders
