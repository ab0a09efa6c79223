"""GPU parity of the rest of the Z4c derivative set (Sec. ssec:z4c): Kreiss-Oliger dissipation
(Eq. dissdef).  Every output node against the oracle on the same seeded inputs (NaN-prefilled
output); bar 1e-12 relative max-norm per (block, operator, field) in FP64, 1e-5 in FP32.
"""
import numpy as np
import pytest

import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("deg", [4, 6, 8, 10])
def test_dissipation_closure_blocks(cuda, deg, dtype):
    """Q^(deg) along x, y, z on uneven closure blocks (ng = 5 >= deg/2), beside the centred D1."""
    wl = synth.batch64(nblocks=6, nfields=3, sizes=(7, 16, 23, 48), ng=5, seed=31)
    ko = f"KO{deg}[0.04]"
    ops = [(ko, d) for d in range(3)] + [("(1)Q1_3[1]", 0), (ko, 1, 2)]
    plan = H.make_plan(wl, ops, dtype=dtype)
    err = H.full_parity(plan, wl, ops, dtype)
    assert err <= H.tol_for(dtype), err


@pytest.mark.parametrize("dtype", [0, 1])
def test_dissipation_periodic(cuda, dtype):
    wl = synth.periodic_box(n=(64, 5, 9), nfields=2, seed=32)
    ops = [("KO8[0.3]", d) for d in range(3)] + [("KO4[1]", 0)]
    plan = H.make_plan(wl, ops, dtype=dtype)
    err = H.full_parity(plan, wl, ops, dtype)
    assert err <= H.tol_for(dtype), err
