"""Shared test helpers: run a workload through the GPU library and through the oracle."""
from __future__ import annotations

import numpy as np

import synth
from oracle import lines as OL
from oracle import schemes as OS

ERR_F64 = 1e-12   # relative max-norm bound for FP64 results
ERR_F32 = 1e-5    # relative max-norm bound for FP32 results


def block_dicts(wl: synth.Workload):
    return [dict(n=b.n, ng=b.ng, h=b.h, boundary=b.boundary) for b in wl.blocks]


def op_fields(wl, ops):
    return [wl.nfields if (len(op) < 3 or op[2] < 0) else 1 for op in ops]


def make_plan(wl, ops, dtype=0):
    import paper_2302_14858_amd as P
    schemes = {}
    pops = []
    for op in ops:
        name = op[0]
        if name not in schemes:
            schemes[name] = P.Scheme.named(name)
        pops.append((schemes[name], op[1], op[2] if len(op) > 2 else -1))
    return P.Plan(block_dicts(wl), wl.nfields, pops, dtype=dtype)


def gpu_run(plan, wl, ops, dtype=0, graph=False, stream=None):
    """Apply the plan to the workload's data; returns per-block lists of [op][field] arrays."""
    import torch
    tdt = torch.float64 if dtype == 0 else torch.float32
    nin, nout = plan.sizes()
    assert nin == wl.data.size
    ioffs, ooffs = plan.offsets()
    assert list(ioffs) == list(wl.in_offsets)
    x = torch.from_numpy(wl.data).to(device="cuda", dtype=tdt)
    y = torch.full((nout,), float("nan"), dtype=tdt, device="cuda")
    if graph:
        plan.capture_graph(x, y)
        plan.launch_graph()
    else:
        plan.apply(x, y)
    torch.cuda.synchronize()
    return unpack(wl, ops, y.double().cpu().numpy(), ooffs)


def unpack(wl, ops, flat, ooffs):
    nf = op_fields(wl, ops)
    res = []
    for b, blk in enumerate(wl.blocks):
        nx, ny, nz = blk.n
        npts = nx * ny * nz
        per = []
        slot = 0
        for o in range(len(ops)):
            fl = []
            for f in range(nf[o]):
                off = ooffs[b] + (slot + f) * npts
                fl.append(flat[off:off + npts].reshape(nz, ny, nx))
            per.append(fl)
            slot += nf[o]
        res.append(per)
    return res


def oracle_run(wl, ops, blocks=None):
    blocks = range(len(wl.blocks)) if blocks is None else blocks
    res = {}
    for b in blocks:
        blk = wl.blocks[b]
        per = []
        for op in ops:
            s = OS.named(op[0])
            d = op[1]
            fsel = list(range(wl.nfields)) if (len(op) < 3 or op[2] < 0) else [op[2]]
            fl = []
            for f in fsel:
                fl.append(OL.apply_block(s, wl.field_view(b, f), blk.ng, blk.h[d], d,
                                         periodic=blk.boundary[d] == synth.PERIODIC))
            per.append(fl)
        res[b] = per
    return res


def rel_err(a, ref):
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(a - ref)) / (den if den > 0 else 1.0))


def max_rel_err(gpu, ora):
    worst = 0.0
    for b, per in ora.items():
        for o, fl in enumerate(per):
            for f, ref in enumerate(fl):
                worst = max(worst, rel_err(gpu[b][o][f], ref))
    return worst
