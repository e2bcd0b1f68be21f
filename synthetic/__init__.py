"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This package only *generates inputs*: workload configurations, initial
conditions, probe placements and the observation-noise draws that stand in
for the paper's self-generated reference simulations.  It holds none of the
assimilation method's arithmetic (no model right-hand side, no projection
operator, no observation operator, no Kalman algebra), so both the CPU
oracle and the GPU path can consume what it produces without sharing code.
"""

from .configs import CONFIGS, Config, tiny_1d, tiny_2d, ragged_2d, uneven_batch
from .fields import (
    burgers_truth_ic,
    burgers_model_ic,
    burgers_member_ics,
    ns_tgv_primitives,
    ns_truth_ic,
    ns_model_ic,
    ns_member_ics,
    probes_for,
    obs_noise,
    random_members_like,
    truth_ic,
    model_ic,
    member_ics,
)

__all__ = [
    "CONFIGS", "Config", "tiny_1d", "tiny_2d", "ragged_2d", "uneven_batch",
    "burgers_truth_ic", "burgers_model_ic", "burgers_member_ics",
    "ns_tgv_primitives", "ns_truth_ic", "ns_model_ic", "ns_member_ics",
    "probes_for", "obs_noise", "random_members_like",
    "truth_ic", "model_ic", "member_ics",
]
