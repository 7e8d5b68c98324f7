"""Sensitivity of the evolution to rounding (CPU, oracle only).

The random-phase network is chaotic: a difference of one unit in the last
place of phi in the initial condition (section 2's random-phase start,
64^3 radiation era, seed 0) grows step by step.  How far it has grown by
step 100 is the floor below which no two correct FP64 implementations, which
round differently, can be expected to agree on that run; the FP64 parity
tolerance of the 100-step run (1e-10, field-scaled per field) must sit well
above it, and it must not be so far above it that a real slip could hide.
"""
import pytest

from helpers import rounding_floor

pytestmark = pytest.mark.slow

FP64_TOL_100_STEPS = 1e-10


def test_rounding_floor_of_the_100_step_run(oracle_mod):
    err = rounding_floor(oracle_mod)
    worst = max(err.values())
    print("one-ulp start, 64^3, 100 steps:", {k: f"{v:.2e}" for k, v in err.items()})
    # grown well past the initial ulp (the dynamics amplify) ...
    assert worst > 1e-14, err
    # ... and still far below the parity tolerance
    assert worst < FP64_TOL_100_STEPS / 100, err
    # every field carries it (the fields are coupled)
    assert min(err.values()) > 1e-15, err
