"""GPU parity: the HIP library against the oracle on seeded synthetic workloads.

Bar: relative max-norm error per (block, operator, field) <= 1e-12 in FP64 and
<= 1e-5 in FP32, against the FP64 oracle on the same inputs.
"""
import numpy as np
import pytest

import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

D12_TRI = [("(1)Q1_3[1]", 0), ("(1)Q1_3[1]", 1), ("(1)Q1_3[1]", 2),
           ("(2)Q1_3[1]", 0), ("(2)Q1_3[1]", 1), ("(2)Q1_3[1]", 2)]
D12_PENTA = [("(1)QP_O8[1]", 0), ("(1)QP_O8[1]", 1), ("(1)QP_O8[1]", 2),
             ("(2)QP_O8[1]", 0), ("(2)QP_O8[1]", 1), ("(2)QP_O8[1]", 2)]


@pytest.mark.parametrize("scheme", ["(1)P1_2", "(1)Q1_3[1]"])
def test_periodic32_dx(cuda, scheme):
    wl = synth.periodic32()
    ops = [(scheme, 0)]
    plan = H.make_plan(wl, ops)
    g = H.gpu_run(plan, wl, ops)
    o = H.oracle_run(wl, ops)
    assert H.max_rel_err(g, o) <= H.ERR_F64


@pytest.mark.parametrize("n", [24, 40])
def test_block_tri_d1_d2_small(cuda, n):
    wl = synth.block128(n=n)
    plan = H.make_plan(wl, D12_TRI)
    g = H.gpu_run(plan, wl, D12_TRI)
    o = H.oracle_run(wl, D12_TRI)
    assert H.max_rel_err(g, o) <= H.ERR_F64


def test_batch_penta_small_f64(cuda):
    wl = synth.batch64(nblocks=6, nfields=3)
    plan = H.make_plan(wl, D12_PENTA)
    g = H.gpu_run(plan, wl, D12_PENTA)
    o = H.oracle_run(wl, D12_PENTA)
    assert H.max_rel_err(g, o) <= H.ERR_F64


def test_batch_penta_small_f32(cuda):
    wl = synth.batch64(nblocks=6, nfields=3)
    plan = H.make_plan(wl, D12_PENTA, dtype=1)
    g = H.gpu_run(plan, wl, D12_PENTA, dtype=1)
    o = H.oracle_run(wl, D12_PENTA)
    assert H.max_rel_err(g, o) <= H.ERR_F32


@pytest.mark.parametrize("n", [64])
def test_periodic_dxyz(cuda, n):
    wl = synth.periodic256(n=n, nfields=2, kmax=n // 3)
    ops = [("(1)Q1_3[1]", 0), ("(1)Q1_3[1]", 1), ("(1)Q1_3[1]", 2)]
    plan = H.make_plan(wl, ops)
    g = H.gpu_run(plan, wl, ops)
    o = H.oracle_run(wl, ops)
    assert H.max_rel_err(g, o) <= H.ERR_F64
