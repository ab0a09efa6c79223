"""GPU parity on kernel paths and plan shapes the benchmark workloads do not reach.

Every test compares every output node with the oracle (NaN-prefilled output, so an unwritten node
fails).  Bar: relative max-norm error per (block, operator, field) <= 1e-12 in FP64 and <= 1e-5 in
FP32, against the FP64 oracle on the same inputs.
"""
import numpy as np
import pytest

import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _ops(d1, d2=None, dirs=(0, 1, 2)):
    ops = [(d1, d) for d in dirs]
    if d2:
        ops += [(d2, d) for d in dirs]
    return ops


def _each_partition(plan, wl, ops, dtype, Ns):
    """Full parity under every partition count the plan accepts, for x and y/z lines of each length."""
    import paper_2302_14858_amd as P
    _, ooffs = plan.offsets()
    _, nout = plan.sizes()
    ref = H.oracle_flat(wl, ops, ooffs, nout)
    tried = 0
    for N in Ns:
        for xl in (0, 1):
            for parts in (1, 2, 4, 8):
                try:
                    plan.set_schedule(N, xl, parts)
                except P.CfdError:
                    continue
                err = H.full_parity(plan, wl, ops, dtype, ref)
                assert err <= H.tol_for(dtype), (N, xl, parts, err)
                tried += 1
                plan.set_schedule(N, xl, 0)
    return tried


@pytest.mark.parametrize("dtype", [0, 1])
def test_penta_padded_closure_lines(cuda, dtype):
    """Pentadiagonal closure lines whose length is no multiple of a compiled partition length: the
    last partition is padded with decoupled identity rows (N = 17, 21, 29, 37, 45)."""
    ops = _ops("(1)QP_O8[1]", "(2)QP_O8[1]")
    wl = synth.batch64(nblocks=10, nfields=2, sizes=(17, 21, 29, 37, 45), seed=11)
    plan = H.make_plan(wl, ops, dtype=dtype)
    assert _each_partition(plan, wl, ops, dtype, (17, 21, 29, 37, 45)) >= 10


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("d1,d2", [("(2)Q1_3[1]", None), ("(1)QP_O8[1]", None), ("(2)QP_O8[1]", None),
                                   ("(1)Q1_3[1]", "(2)Q1_3[1]"), ("(1)QP_O8[1]", "(2)QP_O8[1]")])
def test_periodic_banded_variants(cuda, d1, d2, dtype):
    """Banded periodic lines beyond tridiagonal D1: D2, pentadiagonal D1 and D2, and the fused D1+D2
    pass, on a box with a different line length per direction, every partition count."""
    ops = _ops(d1, d2)
    wl = synth.periodic_box(n=(48, 24, 32), nfields=2, nmodes=12, kmax=10, seed=21)
    plan = H.make_plan(wl, ops, dtype=dtype)
    assert _each_partition(plan, wl, ops, dtype, (48, 24, 32)) >= 4


@pytest.mark.parametrize("dtype", [0, 1])
def test_ghosts_above_requirement(cuda, dtype):
    """Blocks carrying more ghost layers than the scheme reaches (penta at ng = 6, tri at ng = 5)."""
    ops = _ops("(1)QP_O8[1]", "(2)QP_O8[1]")
    wl = synth.batch64(nblocks=4, nfields=2, ng=6, seed=12)
    assert H.full_parity(H.make_plan(wl, ops, dtype=dtype), wl, ops, dtype) <= H.tol_for(dtype)
    ops = _ops("(1)Q1_3[1]", "(2)Q1_3[1]")
    wl = synth.block128(n=40, ng=5)
    assert H.full_parity(H.make_plan(wl, ops, dtype=dtype), wl, ops, dtype) <= H.tol_for(dtype)


@pytest.mark.parametrize("dtype", [0, 1])
def test_order_only_closures_at_three_ghosts(cuda, dtype):
    """Schemes whose reach is below the compiled ring half-width: the explicit (1)E3 on N = 17 and the
    order-only (2)Q1_3[1]:E on N = 49, both at ng = 3, lines along x, y and z.  Partitions whose halo
    would leave the stored line read zeros there."""
    for scheme, n in (("(1)E3", 17), ("(2)Q1_3[1]:E", 49), ("(1)Q1_3[1]:E", 33)):
        ops = _ops(scheme)
        wl = synth.batch64(nblocks=2, nfields=2, ng=3, sizes=(n,), seed=13)
        plan = H.make_plan(wl, ops, dtype=dtype)
        assert _each_partition(plan, wl, ops, dtype, (n,)) >= 2, scheme


SWEEP = [("(1)Q1_3[1]", "(2)Q1_3[1]", 9), ("(1)QP_O8[1]", "(2)QP_O8[1]", 11), ("(1)P1_2", "(2)P1_2", 9),
         ("(1)Q1_3[4pi/5]", None, 9), ("(2)QP_O8[1]", None, 11), ("(1)P1_3", "(2)P1_3", 11),
         ("(1)E3", None, 8), ("(1)Q1_3[1]:E", "(2)Q1_3[1]:E", 8)]


@pytest.mark.parametrize("d1,d2,lo", SWEEP)
def test_seeded_shape_sweep(cuda, d1, d2, lo):
    """Seeded sweep of block extents in [lo, 64] along every direction, per scheme, FP64, default and
    autotuned schedules."""
    import torch
    from oracle import schemes as OS
    ops = _ops(d1, d2)
    ng = max(OS.required_ghosts(OS.named(n), False) for n in (d1, d2) if n)
    seed = 100 + SWEEP.index((d1, d2, lo))
    wl = synth.batch64(nblocks=8, nfields=1, ng=ng, sizes=tuple(range(lo, 65)), seed=seed)
    plan = H.make_plan(wl, ops)
    _, ooffs = plan.offsets()
    _, nout = plan.sizes()
    ref = H.oracle_flat(wl, ops, ooffs, nout)
    assert H.full_parity(plan, wl, ops, 0, ref) <= H.ERR_F64
    x = torch.from_numpy(wl.data).cuda()
    y = torch.empty(nout, dtype=torch.float64, device="cuda")
    plan.autotune(x, y)
    assert H.full_parity(plan, wl, ops, 0, ref) <= H.ERR_F64


def test_unaligned_buffers_rejected(cuda):
    import torch
    import paper_2302_14858_amd as P
    ops = _ops("(1)Q1_3[1]")
    wl = synth.block128(n=24)
    plan = H.make_plan(wl, ops)
    nin, nout = plan.sizes()
    x = torch.zeros(nin + 2, dtype=torch.float64, device="cuda")
    y = torch.zeros(nout + 2, dtype=torch.float64, device="cuda")
    for a, b in ((x[1:], y[:-2]), (x[:-2], y[1:])):
        with pytest.raises(P.CfdError) as e:
            plan.apply(a, b)
        assert e.value.status == P._lib.CFD_EINVAL
    plan.apply(x[2:], y[2:])   # 16-byte aligned views are accepted
    torch.cuda.synchronize()


def test_allocation_failures_return_enomem_without_leaks(cuda):
    """Fail each device allocation of plan creation in turn: CFD_ENOMEM every time, device memory back
    where it was, and plan creation succeeds once the failure comes after its last allocation."""
    import torch
    import paper_2302_14858_amd as P
    ops = _ops("(1)QP_O8[1]", "(2)QP_O8[1]")
    wl = synth.batch64(nblocks=3, nfields=2, seed=14)
    H.make_plan(wl, ops)   # device probe and first-use allocations out of the way
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    failures = 0
    try:
        for k in range(64):
            P.cfd_debug_fail_alloc(k)
            try:
                plan = H.make_plan(wl, ops)
            except P.CfdError as e:
                assert e.status == P._lib.CFD_ENOMEM, str(e)
                failures += 1
                torch.cuda.synchronize()
                assert torch.cuda.mem_get_info()[0] >= free0 - (2 << 20), k
                continue
            P.cfd_debug_fail_alloc(-1)
            assert H.full_parity(plan, wl, ops) <= H.ERR_F64
            break
        else:
            pytest.fail("plan creation never got past the injected failure")
    finally:
        P.cfd_debug_fail_alloc(-1)
    assert failures >= 5


@pytest.mark.parametrize("dtype", [0, 1])
def test_eight_partition_long_lines(cuda, dtype):
    """Lines cut into 8 partitions (8-wave workgroups): closure lines of 128 nodes (tridiagonal D1+D2,
    16-row partitions) and periodic lines of 256 nodes (D1, 32-row partitions), x and y/z, every node
    against the oracle; then the default and every other partition count give the same bar."""
    import paper_2302_14858_amd as P
    # one 128^3 closure block of smooth modes (the batch64 recipe): well conditioned for FP32 D2
    wl = synth.batch64(nblocks=1, nfields=1, sizes=(128,), ng=4, seed=40)
    ops = _ops("(1)Q1_3[1]", "(2)Q1_3[1]")
    plan = H.make_plan(wl, ops, dtype=dtype)
    _, ooffs = plan.offsets()
    _, nout = plan.sizes()
    ref = H.oracle_flat(wl, ops, ooffs, nout)
    for xl in (0, 1):
        plan.set_schedule(128, xl, 8)
    assert H.full_parity(plan, wl, ops, dtype, ref) <= H.tol_for(dtype)
    assert _each_partition(plan, wl, ops, dtype, (128,)) >= 4
    wlp = synth.periodic_box(n=(256, 256, 8), nfields=1, nmodes=8, kmax=100, seed=41)
    opsp = [("(1)Q1_3[1]", 0), ("(1)Q1_3[1]", 1)]
    plan = H.make_plan(wlp, opsp, dtype=dtype)
    for xl in (0, 1):
        plan.set_schedule(256, xl, 8)
    assert H.full_parity(plan, wlp, opsp, dtype) <= H.tol_for(dtype)


@pytest.mark.parametrize("dtype", [0, 1])
def test_second_derivative_alone_on_long_lines(cuda, dtype):
    """A tridiagonal second derivative without a first-derivative partner on lines longer than four
    partitions of 32 rows: periodic 256-node and 192-node lines and 200-node closure lines, x, y and z
    (the 8-wave and 48/64-row classes of the even parity), against the oracle at every node."""
    for wl in (synth.periodic_box(n=(256, 8, 192), nfields=2, seed=61),
               synth.batch64(nblocks=2, nfields=2, sizes=(200, 9), ng=4, seed=62)):
        ops = [("(2)Q1_3[1]", d) for d in range(3)]
        plan = H.make_plan(wl, ops, dtype=dtype)
        err = H.full_parity(plan, wl, ops, dtype)
        assert err <= H.tol_for(dtype), (wl.name, err)
