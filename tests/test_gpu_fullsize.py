"""GPU parity at the full workload sizes, in the launch configuration bench.py times
(autotuned schedule, captured graph, replayed), on outputs the oracle computes one
block-field at a time.

Bar: relative max-norm error per (block, operator, field) <= 1e-12 in FP64 and
<= 1e-5 in FP32 / mixed precision, against the FP64 oracle on the same inputs.
"""
import numpy as np
import pytest

import synth
from oracle import lines as OL
from oracle import schemes as OS
from oracle import wave as W
from tests import helpers as H

pytestmark = pytest.mark.gpu

OPS_PENTA = [("(1)QP_O8[1]", 0), ("(1)QP_O8[1]", 1), ("(1)QP_O8[1]", 2),
             ("(2)QP_O8[1]", 0), ("(2)QP_O8[1]", 1), ("(2)QP_O8[1]", 2)]
OPS_TRI = [("(1)Q1_3[1]", 0), ("(1)Q1_3[1]", 1), ("(1)Q1_3[1]", 2),
           ("(2)Q1_3[1]", 0), ("(2)Q1_3[1]", 1), ("(2)Q1_3[1]", 2)]
OPS_D1 = OPS_TRI[:3]


def _graph_run(wl, ops, dtype, autotune=True):
    """Plan, autotune, capture, replay twice; returns (plan, output tensor)."""
    import torch
    plan = H.make_plan(wl, ops, dtype=dtype)
    nin, nout = plan.sizes()
    tdt = torch.float64 if dtype == 0 else torch.float32
    x = torch.from_numpy(wl.data).to(device="cuda", dtype=tdt)
    y = torch.full((nout,), float("nan"), dtype=tdt, device="cuda")
    if autotune:
        plan.autotune(x, y)
    plan.capture_graph(x, y)
    for _ in range(2):
        plan.launch_graph()
    torch.cuda.synchronize()
    return plan, y


def _sampled_err(plan, y, wl, ops, blocks, fields):
    """Worst relative error over the sampled (block, field) pairs, every operator, every node."""
    _, ooffs = plan.offsets()
    schemes = {name: OS.named(name) for name, _ in ops}
    worst = 0.0
    for b in blocks:
        blk = wl.blocks[b]
        npts = int(np.prod(blk.n))
        for o, (name, d) in enumerate(ops):
            for f in fields:
                off = ooffs[b] + (o * wl.nfields + f) * npts
                got = y[off:off + npts].double().cpu().numpy().reshape(blk.n[2], blk.n[1], blk.n[0])
                ref = OL.apply_block(schemes[name], wl.field_view(b, f), blk.ng, blk.h[d], d,
                                     periodic=blk.boundary[d] == synth.PERIODIC)
                worst = max(worst, H.rel_err(got, ref))
    return worst


@pytest.mark.parametrize("dtype,tol", [(0, H.ERR_F64), (1, H.ERR_F32)])
def test_batch64_full_autotuned_graph(cuda, dtype, tol):
    """The benchmark step: 64 blocks x 22 fields x penta D1+D2 along x, y, z, one graph."""
    wl = synth.batch64()
    plan, y = _graph_run(wl, OPS_PENTA, dtype)
    # blocks of every extent class, first/middle/last fields
    sizes = {}
    for b, blk in enumerate(wl.blocks):
        sizes.setdefault(blk.n, b)
    blocks = sorted(set(list(sizes.values())[:6] + [0, len(wl.blocks) - 1]))
    assert _sampled_err(plan, y, wl, OPS_PENTA, blocks, [0, 11, 21]) <= tol


def test_block128_full(cuda):
    wl = synth.block128()
    plan, y = _graph_run(wl, OPS_TRI, 0)
    assert _sampled_err(plan, y, wl, OPS_TRI, [0], [0]) <= H.ERR_F64


@pytest.mark.parametrize("dtype,tol", [(0, H.ERR_F64), (1, H.ERR_F32), (2, H.ERR_F32)])
def test_periodic256_full(cuda, dtype, tol):
    """Periodic 256^3 x 8 fields, tri D1 along x, y, z: banded FP64, banded FP32, dense mixed."""
    wl = synth.periodic256()
    plan, y = _graph_run(wl, OPS_D1, dtype)
    assert _sampled_err(plan, y, wl, OPS_D1, [0], [0, 7]) <= tol


@pytest.mark.parametrize("dtype,tol", [(0, 1e-12), (1, 1e-5)])
def test_wave192_full_closed_form(cuda, dtype, tol):
    """RK4 on the periodic 192^3 grid against the discrete closed form (every mode evolves by R(dt L))."""
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd.wave import WaveRK4
    n, steps = 192, 20
    wl = synth.wave192(n=n)
    h = wl.blocks[0].h[0]
    dt = 0.25 * h
    rk = WaveRK4([dict(n=b.n, ng=b.ng, h=b.h, boundary=b.boundary) for b in wl.blocks],
                 P.Scheme.named("(1)Q1_3[1]"), dt, dtype=dtype)
    rk.load(wl.data)
    rk.capture()
    rk.load(wl.data)
    rk.run(steps)
    got = rk.u.double().cpu().numpy().reshape(5, n, n, n)
    amp = W.mode_evolution(OS.named("(1)Q1_3[1]"), synth.WAVE_K, h, dt, steps)
    x = np.arange(n) * h
    for f in range(5):
        ref = W.mode_field(amp[f], synth.WAVE_K, x, x, x)
        assert np.max(np.abs(got[f] - ref)) <= tol * np.max(np.abs(ref)), f
