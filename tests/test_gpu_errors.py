"""Numerical failures on the device are reported, not carried on.

A Gaussian field so large that the interaction exponentials overflow (finite
field values, so the host accepts them) makes the stabilisation flag the
context (vanishing QR scale, singular LU pivot or non-finite G): dqmc_init
returns DQMC_E_NUMERIC, later sweeps refuse with DQMC_E_STATE, and a sane
field with a new dqmc_init brings the chain back to parity with the oracle.
"""
import numpy as np
import pytest

from gpu_util import maxabs, pair
from oracle import sweep as osweep
from paper_1704_00131_amd._lib import DQMCError

pytestmark = pytest.mark.gpu

DQMC_E_NUMERIC, DQMC_E_STATE = 4, 6


def test_overflowing_field_is_flagged_and_recoverable():
    print("numerical failure: square 4x4, Gaussian field of 1e200", flush=True)
    om, ch, _ = pair("square", 4, 4, 4.0, 2.0, 0.1, 10, seed=5, field="gauss")
    ch.random_field()
    f0, _ = ch.get_state()
    ch.set_state(np.full_like(f0, 1e200))
    with pytest.raises(DQMCError) as e_init:
        ch.init()
    assert e_init.value.status == DQMC_E_NUMERIC
    with pytest.raises(DQMCError) as e_sweep:
        ch.sweep(1)
    assert e_sweep.value.status == DQMC_E_STATE
    # recovery: the same chain, a sane field, a new initialisation
    ch.set_state(f0)
    ch.init()
    oc = osweep.Chain(om, f0).init()
    ch.sweep(1)
    oc.sweep()
    f, _ = ch.get_state()
    assert np.array_equal(f, oc.field)
    assert maxabs(ch.G.cpu().numpy(), oc.G) < 1e-9
