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


def _schedules(plan_Ns):
    for N in plan_Ns:
        for x in (0, 1):
            for P in (1, 2, 4):
                yield N, x, P


def test_every_schedule_same_result(cuda):
    """Partition counts, persistent / per-item grids and fused / split x launches all agree with the oracle."""
    import paper_2302_14858_amd as P
    wl = synth.batch64(nblocks=4, nfields=2, sizes=(16, 24, 32, 48), seed=5)
    plan = H.make_plan(wl, D12_PENTA)
    o = H.oracle_run(wl, D12_PENTA)
    tried = 0
    for N in sorted({b.n[d] for b in wl.blocks for d in range(3)}):
        for x in (0, 1):
            for parts in (1, 2, 4):
                try:
                    plan.set_schedule(N, x, parts, persistent=(parts != 2), split_x=(parts == 2),
                                      xcd=(parts == 4))
                except P.CfdError:
                    continue
                g = H.gpu_run(plan, wl, D12_PENTA)
                assert H.max_rel_err(g, o) <= H.ERR_F64, (N, x, parts)
                tried += 1
    assert tried >= 8
    for mode in ({"persistent": True, "xcd": True}, {"persistent": True, "xcd": True, "split_x": True},
                 {"persistent": False}, {"persistent": False, "split_x": True, "concurrent": True},
                 {"persistent": False, "xcd": True}, {"persistent": False, "xcd": True, "split_x": True,
                                                      "concurrent": True},
                 {"persistent": True, "split_x": True, "concurrent": True}):
        plan.set_schedule(0, **mode)
        g = H.gpu_run(plan, wl, D12_PENTA)
        assert H.max_rel_err(g, o) <= H.ERR_F64, mode


def test_periodic_partitions_long_lines(cuda):
    """Cyclic solve split over 1, 2 and 4 partitions (the reduced system closes the wrap)."""
    wl = synth.periodic256(n=128, nfields=1, nmodes=8, kmax=40)
    ops = [("(1)Q1_3[1]", 0), ("(1)Q1_3[1]", 1), ("(1)Q1_3[1]", 2)]
    plan = H.make_plan(wl, ops)
    o = H.oracle_run(wl, ops)
    for x in (0, 1):
        for parts in (2, 4):
            plan.set_schedule(128, x, parts)
            g = H.gpu_run(plan, wl, ops)
            assert H.max_rel_err(g, o) <= H.ERR_F64, (x, parts)


def test_graph_replay_matches_eager(cuda):
    import torch
    wl = synth.batch64(nblocks=3, nfields=2)
    plan = H.make_plan(wl, D12_PENTA)
    nin, nout = plan.sizes()
    x = torch.from_numpy(wl.data).cuda()
    y_eager = torch.empty(nout, dtype=torch.float64, device="cuda")
    y_graph = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.apply(x, y_eager)
    plan.capture_graph(x, y_graph)
    for rep in range(4):
        y_graph.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.launch_graph()
        torch.cuda.synchronize()
        assert torch.equal(y_graph, y_eager), rep
        x.mul_(1.0)   # unrelated eager work between replays


def test_concurrent_graph_replay(cuda):
    """x and y/z launches on forked streams inside the captured graph: every replay equals the eager result."""
    import torch
    wl = synth.batch64(nblocks=4, nfields=2, seed=7)
    plan = H.make_plan(wl, D12_PENTA)
    plan.set_schedule(0, persistent=True, split_x=True, concurrent=True)
    assert plan.get_schedule()["concurrent"]
    nin, nout = plan.sizes()
    x = torch.from_numpy(wl.data).cuda()
    y_eager = torch.empty(nout, dtype=torch.float64, device="cuda")
    y_graph = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.apply(x, y_eager)
    torch.cuda.synchronize()
    o = H.oracle_run(wl, D12_PENTA, blocks=[0, 1])
    g = H.unpack(wl, D12_PENTA, y_eager.cpu().numpy(), plan.offsets()[1])
    assert H.max_rel_err({b: g[b] for b in (0, 1)}, o) <= H.ERR_F64
    plan.capture_graph(x, y_graph)
    for rep in range(4):
        y_graph.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.launch_graph()
        torch.cuda.synchronize()
        assert torch.equal(y_graph, y_eager), rep
        x.mul_(1.0)


def test_autotune_cache_round_trip(cuda, tmp_path):
    """Autotuning writes its per-class choices to the cache file; a second plan tuned from that file
    takes them and still matches the oracle."""
    import torch
    wl = synth.batch64(nblocks=4, nfields=2, sizes=(16, 24, 32, 48), seed=9)
    o = H.oracle_run(wl, D12_PENTA)
    cache = str(tmp_path / "tune.txt")
    for _ in range(2):
        plan = H.make_plan(wl, D12_PENTA)
        nin, nout = plan.sizes()
        x = torch.from_numpy(wl.data).cuda()
        y = torch.empty(nout, dtype=torch.float64, device="cuda")
        plan.autotune(x, y, cache_path=cache)
        assert H.max_rel_err(H.gpu_run(plan, wl, D12_PENTA), o) <= H.ERR_F64
    lines = open(cache).read().split()
    assert lines and lines[0].startswith("v5:")


def test_graph_capture_fallback_and_nonfinite_count(cuda):
    """When the capture fails the plan replays the apply eagerly (graph status 2) with the same
    result; the non-finite count sees an unwritten (NaN) output and a complete one."""
    import torch
    import paper_2302_14858_amd as P
    wl = synth.batch64(nblocks=3, nfields=2, seed=51)
    ops = [("(1)QP_O8[1]", 0), ("(2)QP_O8[1]", 1), ("(1)QP_O8[1]", 2)]
    plan = H.make_plan(wl, ops)
    _, nout = plan.sizes()
    x = torch.from_numpy(wl.data).cuda()
    y0 = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    assert plan.count_nonfinite(y0) == nout
    plan.apply(x, y0)
    assert plan.count_nonfinite(y0) == 0
    assert plan.graph_status() == 0
    P.cfd_debug_fail_capture(True)
    y1 = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.capture_graph(x, y1)
    assert plan.graph_status() == 2
    for _ in range(2):
        plan.launch_graph()
        torch.cuda.synchronize()
        assert torch.equal(y0, y1)
        y1.fill_(float("nan"))
    plan.capture_graph(x, y1)            # hook consumed: a real graph this time
    assert plan.graph_status() == 1
    plan.launch_graph()
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
