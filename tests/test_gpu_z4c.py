"""GPU parity of the rest of the Z4c derivative set (Sec. ssec:z4c): Kreiss-Oliger dissipation
(Eq. dissdef) and the symmetrised mixed second derivatives 1/2 (D_i D_j + D_j D_i).  Every output
node against the oracle on the same seeded inputs (NaN-prefilled output).

Bars: mixed derivatives, relative max-norm error per (block, operator, field) <= 1e-12 in FP64
and <= 1e-5 in FP32.  Dissipation: Q^(2r) of smooth data cancels to a small fraction
(sin^(2r)(k h / 2)) of its inputs, so its error is bounded against the scale its evaluation rounds
at, S = sum_n |q_n| max|f| / h = sigma max|f| / h: |error| <= 32 * 2^-53 * S in FP64 (both the
oracle's 2r repeated differences and the library's binomial sum round at that scale) and
<= 8 * 2^-24 * S in FP32 (input rounding plus the FP32 sums).
"""
import numpy as np
import pytest

import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


KO_BAR = {0: 32 * 2.0 ** -53, 1: 8 * 2.0 ** -24}


def _ko_scaled_error(plan, wl, ops, dtype):
    """Worst |error| / (sum|q| max|f| / h) over every (block, Kreiss-Oliger operator, field); the
    other operators of the plan are held to the relative bar of their precision here."""
    import torch
    _, nout = plan.sizes()
    _, ooffs = plan.offsets()
    tdt = torch.float64 if dtype == 0 else torch.float32
    x = torch.from_numpy(wl.data).to(device="cuda", dtype=tdt)
    y = torch.full((nout,), float("nan"), dtype=tdt, device="cuda")
    plan.apply(x, y)
    torch.cuda.synchronize()
    got = y.double().cpu().numpy()
    ref = H.oracle_flat(wl, ops, ooffs, nout)
    H.compare_flat(got, ref, wl, ops, ooffs)          # every node written, finite
    nf = H.op_fields(wl, ops)
    worst = 0.0
    for b, blk in enumerate(wl.blocks):
        npts = int(np.prod(blk.n))
        slot = 0
        for o, op in enumerate(ops):
            ko = H.ko_name(op[0])
            fsel = list(range(wl.nfields)) if (len(op) < 3 or op[2] < 0) else [op[2]]
            for j, f in enumerate(fsel):
                off = ooffs[b] + (slot + j) * npts
                if ko is None:
                    assert H.rel_err(got[off:off + npts], ref[off:off + npts]) <= H.tol_for(dtype), op
                    continue
                r, sigma = ko
                qsum = sigma * 4.0 ** -r * sum(abs(np.polynomial.polynomial.polypow([1, 1], 2 * r)))
                scale = qsum * np.max(np.abs(wl.field_view(b, f))) / blk.h[op[1]]
                worst = max(worst, np.max(np.abs(got[off:off + npts] - ref[off:off + npts])) / scale)
            slot += nf[o]
    return worst


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("deg", [4, 6, 8, 10])
def test_dissipation_closure_blocks(cuda, deg, dtype):
    """Q^(deg) along x, y, z on uneven closure blocks (ng = 5 >= deg/2), beside the centred D1."""
    wl = synth.batch64(nblocks=6, nfields=3, sizes=(7, 16, 23, 48), ng=5, seed=31)
    ko = f"KO{deg}[0.04]"
    ops = [(ko, d) for d in range(3)] + [(ko, 1, 2)]
    plan = H.make_plan(wl, ops, dtype=dtype)
    err = _ko_scaled_error(plan, wl, ops, dtype)
    assert err <= KO_BAR[dtype], err


def test_dissipation_beside_centred_operators(cuda):
    wl = synth.batch64(nblocks=4, nfields=2, ng=5, seed=33)
    ops = [("KO8[0.04]", 0), ("(1)QP_O8[1]", 0), ("(2)QP_O8[1]", 0), ("KO8[0.04]", 2), ("(1)Q1_3[1]", 2)]
    plan = H.make_plan(wl, ops)
    assert _ko_scaled_error(plan, wl, ops, 0) <= KO_BAR[0]


@pytest.mark.parametrize("dtype", [0, 1])
def test_dissipation_periodic(cuda, dtype):
    wl = synth.periodic_box(n=(64, 16, 24), nfields=2, seed=32)
    ops = [("KO8[0.3]", d) for d in range(3)] + [("KO4[1]", 0)]
    plan = H.make_plan(wl, ops, dtype=dtype)
    assert _ko_scaled_error(plan, wl, ops, dtype) <= KO_BAR[dtype]


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("name", ["(1)Q1_3[1]", "(1)QP_O8[1]", "(1)P1_2", "(1)E3"])
def test_mixed_closure_blocks(cuda, name, dtype):
    """All three pairs on uneven closure blocks (edge ghosts read), one op on a single field,
    beside ordinary operators in the same plan."""
    wl = synth.batch64(nblocks=5, nfields=3, sizes=(7, 16, 23, 48), ng=5, seed=34)
    ops = [(name, 0, -1, -1, 1), (name, 0, 2, -1, 2), (name, 2, -1, -1, 1), ("(1)Q1_3[1]", 1), ("(2)Q1_3[1]", 1)]
    plan = H.make_plan(wl, ops, dtype=dtype)
    err = H.full_parity(plan, wl, ops, dtype)
    assert err <= H.tol_for(dtype), err


@pytest.mark.parametrize("dtype", [0, 1])
def test_mixed_periodic_and_schedules(cuda, dtype):
    """Periodic box (no extension along periodic directions), then every launch shape."""
    import paper_2302_14858_amd as P
    wl = synth.periodic_box(n=(64, 16, 32), nfields=2, seed=35)
    ops = [("(1)Q1_3[1]", 0, -1, -1, 1), ("(1)QP_O8[1]", 1, -1, -1, 2), ("(1)Q1_3[1]", 2, 1, -1, 0)]
    plan = H.make_plan(wl, ops, dtype=dtype)
    _, ooffs = plan.offsets()
    _, nout = plan.sizes()
    ref = H.oracle_flat(wl, ops, ooffs, nout)
    for flags in (dict(persistent=True), dict(persistent=False), dict(persistent=True, split_x=True),
                  dict(persistent=True, xcd=True), dict(persistent=True, split_x=True, concurrent=True)):
        plan.set_schedule(0, **flags)
        assert H.full_parity(plan, wl, ops, dtype, ref) <= H.tol_for(dtype), flags


def test_mixed_graph_replay(cuda):
    import torch
    wl = synth.batch64(nblocks=4, nfields=2, ng=4, seed=36)
    ops = [("(1)Q1_3[1]", 0, -1, -1, 1), ("(1)Q1_3[1]", 1, -1, -1, 2), ("(1)Q1_3[1]", 0)]
    plan = H.make_plan(wl, ops)
    _, nout = plan.sizes()
    x = torch.from_numpy(wl.data).cuda()
    y0 = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.apply(x, y0)
    y1 = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.capture_graph(x, y1)
    for _ in range(3):
        plan.launch_graph()
        torch.cuda.synchronize()
        assert torch.equal(y0, y1)
        y1.fill_(float("nan"))
        torch.cuda.synchronize()


def test_mixed_plan_validation(cuda):
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd import _lib
    wl = synth.batch64(nblocks=2, nfields=2, ng=4, seed=37)
    bd = H.block_dicts(wl)
    q = P.Scheme.named("(1)Q1_3[1]")
    for bad in ((q, 0, -1, -1, 0), (q, 0, -1, -1, 3)):
        with pytest.raises(P.CfdError) as e:
            P.Plan(bd, 2, [bad])
        assert e.value.status == _lib.CFD_EINVAL
    for s in (P.Scheme.named("(2)Q1_3[1]"), P.Scheme.named("(1)X2-"), P.Scheme.dissipation(2, 0.1)):
        with pytest.raises(P.CfdError) as e:
            P.Plan(bd, 2, [(s, 0, -1, -1, 1)])
        assert e.value.status == _lib.CFD_EINVAL
    with pytest.raises(P.CfdError) as e:                 # (1)QP_O8[1] needs 5 ghost layers
        P.Plan(bd, 2, [(P.Scheme.named("(1)QP_O8[1]"), 0, -1, -1, 1)])
    assert e.value.status == _lib.CFD_EGHOST


@pytest.mark.parametrize("dtype", [0, 1])
def test_mixed_long_periodic_lines_accumulate(cuda, dtype):
    """Second orders that accumulate along 192-node periodic lines (eight partitions: the 8-wave
    accumulating class) and along short lines, against the oracle at every node."""
    wl = synth.periodic_box(n=(192, 8, 12), nfields=2, seed=37)
    ops = [("(1)Q1_3[1]", 1, -1, -1, 0), ("(1)Q1_3[1]", 2, 0, -1, 0), ("(1)Q1_3[1]", 1, 1, -1, 2)]
    plan = H.make_plan(wl, ops, dtype=dtype)
    assert H.full_parity(plan, wl, ops, dtype) <= H.tol_for(dtype)
