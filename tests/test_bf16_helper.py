"""The BF16 rounding the training-gradient test applies to the oracle's
steps: round to nearest with ties to even, as torch's float32 -> bfloat16
conversion does."""

import numpy as np
import torch

from tests.gpu_helpers import bf16_round


def test_ties_to_even_and_halfway_cases():
    e = 2.0 ** -8   # half the BF16 spacing at 1
    assert bf16_round(1.0) == 1.0
    assert bf16_round(1.0 + e) == 1.0                      # tie, even neighbour below
    assert bf16_round(1.0 + 3 * e) == 1.0 + 4 * e          # tie, even neighbour above
    assert bf16_round(1.0 + e + 2.0 ** -20) == 1.0 + 2 * e
    assert bf16_round(-(1.0 + 3 * e)) == -(1.0 + 4 * e)
    assert bf16_round(0.0) == 0.0


def test_matches_torch_bfloat16():
    x = np.random.default_rng(3).standard_normal(100000).astype(np.float32) * 10.0 ** np.random.default_rng(4).integers(-20, 20, 100000)
    ref = torch.as_tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(bf16_round(x), ref)
