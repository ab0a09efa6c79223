"""The allocation-free entry point cfd_apply_block_noalloc through the C ABI, against the plan path
(cfd_plan_create + cfd_apply with the same single operator) and against the oracle.

Each case calls it twice in a row, the second time on a smaller block, so stale contents of the
shared device array from the first call would show.  Bar: bit for bit equal to the plan path (same
kernels, tables and partitions), and within 1e-12 (FP64) / 1e-5 (FP32) of the oracle.
"""
import numpy as np
import pytest

import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _block_workload(n, ng, nfields, periodic, seed):
    import synth as S
    if periodic:
        return S.periodic_box(n=n, nfields=nfields, nmodes=10, kmax=min(n) // 3, seed=seed)
    wl = S.batch64(nblocks=1, nfields=nfields, ng=ng, sizes=(n[0],), seed=seed)
    blk = wl.blocks[0]
    if tuple(blk.n) != tuple(n):   # anisotropic extents: rebuild with the exact shape
        b = S.Block(tuple(n), ng, blk.h, blk.boundary, blk.origin)
        m = wl.modes
        data, offs = S._fill([b], nfields, lambda bb, f, x, y, z: S.eval_modes(m[f][0], x, y, z))
        wl = S.Workload("block", [b], nfields, data, offs, m)
    return wl


def _case(scheme, d, field, dtype, wl):
    import torch
    import paper_2302_14858_amd as P
    blk = wl.blocks[0]
    bd = dict(n=blk.n, ng=blk.ng, h=blk.h, boundary=blk.boundary)
    tdt = torch.float64 if dtype == 0 else torch.float32
    x = torch.from_numpy(wl.data).to(device="cuda", dtype=tdt)
    nf_out = wl.nfields if field < 0 else 1
    npts = int(np.prod(blk.n))
    y = torch.full((nf_out * npts,), float("nan"), dtype=tdt, device="cuda")
    P.cfd_apply_block_noalloc(P.Scheme.named(scheme), bd, d, wl.nfields, x, y, field=field, dtype=dtype)
    torch.cuda.synchronize()
    # the plan path with the same single operator
    ops = [(scheme, d, field)]
    plan = H.make_plan(wl, ops, dtype=dtype)
    _, nout = plan.sizes()
    assert nout == y.numel()
    y_plan = torch.full((nout,), float("nan"), dtype=tdt, device="cuda")
    plan.apply(x, y_plan)
    torch.cuda.synchronize()
    assert torch.equal(y, y_plan), (scheme, d, field, dtype)
    _, ooffs = plan.offsets()
    ref = H.oracle_flat(wl, ops, ooffs, nout)
    err = H.compare_flat(y.double().cpu().numpy(), ref, wl, ops, ooffs)
    assert err <= H.tol_for(dtype), err
    return err


CASES = [
    # scheme, direction, field, dtype, (first block, second block), ng, periodic
    ("(1)Q1_3[1]", 0, -1, 0, ((40, 36, 44), (24, 20, 28)), 4, False),
    ("(1)Q1_3[1]", 1, -1, 0, ((40, 36, 44), (24, 20, 28)), 4, False),
    ("(1)Q1_3[1]", 2, -1, 0, ((40, 36, 44), (24, 20, 28)), 4, False),
    ("(2)QP_O8[1]", 1, 1, 0, ((48, 32, 40), (17, 21, 29)), 5, False),
    ("(1)QP_O8[1]", 0, -1, 1, ((45, 32, 24), (16, 16, 16)), 5, False),
    ("(1)Q1_3[1]", 0, -1, 1, ((64, 48, 32), (32, 24, 16)), 0, True),
    ("(2)Q1_3[1]", 2, 0, 0, ((64, 48, 32), (32, 24, 16)), 0, True),
]


@pytest.mark.parametrize("scheme,d,field,dtype,shapes,ng,periodic", CASES)
def test_noalloc_matches_plan_twice(cuda, scheme, d, field, dtype, shapes, ng, periodic):
    for k, n in enumerate(shapes):
        wl = _block_workload(n, ng, 3, periodic, seed=40 + k)
        print(f"noalloc {scheme} dir={d} field={field} dtype={dtype} n={n} call={k}", flush=True)
        _case(scheme, d, field, dtype, wl)


def test_noalloc_refuses_oversized_work_lists(cuda):
    """A work list beyond the fixed device array is refused before anything is launched."""
    import torch
    import paper_2302_14858_amd as P
    x = torch.zeros(64, dtype=torch.float64, device="cuda")
    bd = dict(n=(8, 512, 512), ng=4, h=(0.1, 0.1, 0.1), boundary=(0, 0, 0))
    with pytest.raises(P.CfdError) as e:
        P.cfd_apply_block_noalloc(P.Scheme.named("(1)Q1_3[1]"), bd, 0, 600, x, x)
    assert e.value.status == P._lib.CFD_EUNSUPPORTED
    with pytest.raises(P.CfdError) as e:
        P.cfd_apply_block_noalloc(P.Scheme.named("(1)Q1_3[1]"), dict(bd, ng=2), 0, 1, x, x)
    assert e.value.status == P._lib.CFD_EGHOST
