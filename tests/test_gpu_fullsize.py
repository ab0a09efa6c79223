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


def _full_err(plan, y, wl, ops, ref=None):
    """Worst relative error over every block, operator, field and node; also checks that no
    output node is left NaN (the output buffer is NaN-prefilled)."""
    _, ooffs = plan.offsets()
    got = y.double().cpu().numpy()
    if ref is None:
        ref = H.oracle_flat(wl, ops, ooffs, got.size)
    return H.compare_flat(got, ref, wl, ops, ooffs)


_BATCH64 = {}


def _batch64_ref():
    """The batch64 workload and the oracle's full result (computed once for FP64 and FP32)."""
    if not _BATCH64:
        wl = synth.batch64()
        import paper_2302_14858_amd as P
        plan = H.make_plan(wl, OPS_PENTA)
        _, ooffs = plan.offsets()
        _, nout = plan.sizes()
        _BATCH64["wl"] = wl
        _BATCH64["ref"] = H.oracle_flat(wl, OPS_PENTA, ooffs, nout)
    return _BATCH64["wl"], _BATCH64["ref"]


@pytest.mark.parametrize("dtype,tol", [(0, H.ERR_F64), (1, H.ERR_F32)])
def test_batch64_full_autotuned_graph(cuda, dtype, tol):
    """The benchmark step: 64 blocks x 22 fields x penta D1+D2 along x, y, z, one graph; every output
    node of every block, field and operator against the oracle."""
    wl, ref = _batch64_ref()
    plan, y = _graph_run(wl, OPS_PENTA, dtype)
    print(f"batch64 dtype={dtype} schedule={plan.get_schedule()}", flush=True)
    assert _full_err(plan, y, wl, OPS_PENTA, ref) <= tol


@pytest.mark.parametrize("flags", [{"persistent": False, "xcd": True, "split_x": True, "concurrent": True},
                                   {"persistent": True, "xcd": True}, {"persistent": False}])
def test_batch64_full_each_launch_shape(cuda, flags):
    """Every output node of batch64 (FP64) under the XCD-interleaved per-item order, the XCD-queue
    persistent grid and the plain per-item grid, default partitions."""
    import paper_2302_14858_amd as P
    wl, ref = _batch64_ref()
    plan = H.make_plan(wl, OPS_PENTA)
    try:
        plan.set_schedule(0, **flags)
    except P.CfdError as e:
        assert e.status == P._lib.CFD_EUNSUPPORTED and not flags["persistent"]
        pytest.skip("XCD-interleaved per-item order not offered on this device")
    import torch
    nin, nout = plan.sizes()
    x = torch.from_numpy(wl.data).cuda()
    y = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.capture_graph(x, y)
    plan.launch_graph()
    torch.cuda.synchronize()
    assert _full_err(plan, y, wl, OPS_PENTA, ref) <= H.ERR_F64


def test_block128_full(cuda):
    wl = synth.block128()
    plan, y = _graph_run(wl, OPS_TRI, 0)
    assert _full_err(plan, y, wl, OPS_TRI) <= H.ERR_F64


def test_block128_ng3_order_only_closures(cuda):
    """The 128^3 block at the literal 3 ghost layers: the order-only closures (1)/(2)Q1_3[1]:E."""
    ops = [("(1)Q1_3[1]:E", d) for d in range(3)] + [("(2)Q1_3[1]:E", d) for d in range(3)]
    wl = synth.block128(ng=3)
    plan, y = _graph_run(wl, ops, 0)
    assert _full_err(plan, y, wl, ops) <= H.ERR_F64


_P256 = {}


def _periodic256_ref():
    if not _P256:
        wl = synth.periodic256()
        plan = H.make_plan(wl, OPS_D1)
        _, ooffs = plan.offsets()
        _, nout = plan.sizes()
        _P256["wl"] = wl
        _P256["ref"] = H.oracle_flat(wl, OPS_D1, ooffs, nout)
    return _P256["wl"], _P256["ref"]


@pytest.mark.parametrize("dtype,tol", [(0, H.ERR_F64), (1, H.ERR_F32), (2, H.ERR_F32)])
def test_periodic256_full(cuda, dtype, tol):
    """Periodic 256^3 x 8 fields, tri D1 along x, y, z: banded FP64, banded FP32, dense mixed; all
    8 fields, every node."""
    wl, ref = _periodic256_ref()
    plan, y = _graph_run(wl, OPS_D1, dtype)
    assert _full_err(plan, y, wl, OPS_D1, ref) <= tol


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
