"""GPU parity of the dense mixed-precision periodic path (BF16 MFMA products,
FP32 accumulation, one FP64-residual refinement) against the FP64 oracle.

Bar: relative max-norm error <= 1e-5 per (block, operator, field).
"""
import numpy as np
import pytest

import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu
MIXED = 2


@pytest.mark.parametrize("n,scheme", [(64, "(1)Q1_3[1]"), (96, "(2)Q1_3[1]"), (32, "(1)QP_O8[1]"),
                                      (128, "(1)P1_2")])
def test_dense_periodic_dxyz(cuda, n, scheme):
    wl = synth.periodic256(n=n, nfields=2, nmodes=16, kmax=n // 3)
    ops = [(scheme, 0), (scheme, 1), (scheme, 2)]
    plan = H.make_plan(wl, ops, dtype=MIXED)
    g = H.gpu_run(plan, wl, ops, dtype=MIXED)
    o = H.oracle_run(wl, ops)
    assert H.max_rel_err(g, o) <= H.ERR_F32


def test_dense_longest_line_penta_d2(cuda):
    wl = synth.periodic_box(n=(256, 3, 2), nfields=1, kmax=60)
    ops = [("(2)QP_O8[1]", 0)]
    plan = H.make_plan(wl, ops, dtype=MIXED)
    g = H.gpu_run(plan, wl, ops, dtype=MIXED)
    o = H.oracle_run(wl, ops)
    assert H.max_rel_err(g, o) <= H.ERR_F32


@pytest.mark.parametrize("n", [(64, 5, 7), (32, 1, 1), (5, 96, 3), (3, 2, 160)])
def test_dense_ragged_line_counts(cuda, n):
    """Line counts that leave a partial 32-line tile; one periodic direction each."""
    d = int(np.argmax(n))
    wl = synth.periodic_box(n=n, nfields=3, kmax=10)
    ops = [("(1)Q1_3[1]", d)]
    plan = H.make_plan(wl, ops, dtype=MIXED)
    g = H.gpu_run(plan, wl, ops, dtype=MIXED)
    o = H.oracle_run(wl, ops)
    assert H.max_rel_err(g, o) <= H.ERR_F32


def test_dense_graph_replay_and_grids(cuda):
    import torch
    wl = synth.periodic256(n=64, nfields=2, nmodes=16, kmax=20)
    ops = [("(1)Q1_3[1]", 0), ("(1)Q1_3[1]", 1), ("(1)Q1_3[1]", 2)]
    plan = H.make_plan(wl, ops, dtype=MIXED)
    o = H.oracle_run(wl, ops)
    for pers in (True, False):
        plan.set_schedule(persistent=pers)
        assert H.max_rel_err(H.gpu_run(plan, wl, ops, dtype=MIXED), o) <= H.ERR_F32
    nin, nout = plan.sizes()
    x = torch.from_numpy(wl.data).to(device="cuda", dtype=torch.float32)
    y = torch.full((nout,), float("nan"), dtype=torch.float32, device="cuda")
    plan.capture_graph(x, y)
    ref = None
    for rep in range(3):
        y.fill_(float("nan"))
        plan.launch_graph()
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        if ref is None:
            ref = got
            assert H.max_rel_err(H.unpack(wl, ops, got.astype(np.float64), plan.offsets()[1]), o) <= H.ERR_F32
        else:
            assert np.array_equal(got, ref)


def test_dense_agrees_with_fp32_banded(cuda):
    """Mixed and FP32 banded results agree with each other to the FP32 bar."""
    wl = synth.periodic256(n=64, nfields=1, nmodes=16, kmax=20)
    ops = [("(1)Q1_3[1]", 0), ("(1)Q1_3[1]", 1), ("(1)Q1_3[1]", 2)]
    gm = H.gpu_run(H.make_plan(wl, ops, dtype=MIXED), wl, ops, dtype=MIXED)
    gf = H.gpu_run(H.make_plan(wl, ops, dtype=1), wl, ops, dtype=1)
    for o in range(3):
        assert H.rel_err(gm[0][o][0], gf[0][o][0]) <= 2 * H.ERR_F32


@pytest.mark.parametrize("scheme,d", [("(1)E5", 0), ("(2)E4", 2)])
def test_dense_wide_explicit_stencil(cuda, scheme, d):
    """RHS half-width above 3 (explicit schemes, A = I): the residual's general stencil path."""
    wl = synth.periodic_box(n=(64, 32, 96), nfields=2, kmax=12)
    ops = [(scheme, d)]
    plan = H.make_plan(wl, ops, dtype=MIXED)
    g = H.gpu_run(plan, wl, ops, dtype=MIXED)
    o = H.oracle_run(wl, ops)
    assert H.max_rel_err(g, o) <= H.ERR_F32


def test_dense_several_tables_in_one_launch(cuda):
    """y and z lines of three schemes share one kernel class: workgroups re-stage the circulant
    tables whenever the item's table changes (persistent and one-workgroup-per-item grids)."""
    wl = synth.periodic_box(n=(24, 64, 64), nfields=2, kmax=12)
    ops = [("(1)Q1_3[1]", 1), ("(2)Q1_3[1]", 2), ("(1)QP_O8[1]", 2), ("(2)QP_O8[1]", 1)]
    plan = H.make_plan(wl, ops, dtype=MIXED)
    o = H.oracle_run(wl, ops)
    for pers in (True, False):
        plan.set_schedule(persistent=pers)
        assert H.max_rel_err(H.gpu_run(plan, wl, ops, dtype=MIXED), o) <= H.ERR_F32


def test_dense_rejects_fields_over_4GiB(cuda):
    """The dense kernels address a field with 32-bit byte offsets: larger fields are refused at plan creation."""
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd import _lib
    sch = P.Scheme.named("(1)Q1_3[1]")
    blocks = [dict(n=(256, 4096, 1100), ng=0, h=(0.1, 0.1, 0.1), boundary=(synth.PERIODIC,) * 3)]
    with pytest.raises(P.CfdError) as e:
        P.Plan(blocks, 1, [(sch, 0, -1)], dtype=MIXED)
    assert e.value.status == _lib.CFD_EUNSUPPORTED


def test_dense_x_lines_unaligned_input(cuda):
    """An odd ghost width puts x-line inputs off 16-byte alignment: the per-element load path."""
    rng = np.random.default_rng(12)
    n = (64, 6, 5)
    h = tuple(2 * np.pi / v for v in n)
    blk = synth.Block(n, 1, h, (synth.PERIODIC,) * 3, (0.0, 0.0, 0.0))
    modes = [synth._random_modes(rng, 8, 0, 10, 1.0, exclude_zero=True) for _ in range(2)]
    for m in modes:
        m.k = np.minimum(m.k, np.array([max(0, v // 2 - 1) for v in n]))
    data, offs = synth._fill([blk], 2, lambda b, f, x, y, z: synth.eval_modes(modes[f], x, y, z))
    wl = synth.Workload("unaligned", [blk], 2, data, offs, [[m] for m in modes])
    ops = [("(1)Q1_3[1]", 0)]
    plan = H.make_plan(wl, ops, dtype=MIXED)
    g = H.gpu_run(plan, wl, ops, dtype=MIXED)
    o = H.oracle_run(wl, ops)
    assert H.max_rel_err(g, o) <= H.ERR_F32
