"""Shared test helpers: run a workload through the GPU library and through the oracle."""
from __future__ import annotations

import numpy as np

import synth
from oracle import biased as OB
from oracle import dissipation as ODS
from oracle import mixed as OM
from oracle import lines as OL
from oracle import schemes as OS

ERR_F64 = 1e-12   # relative max-norm bound for FP64 results
ERR_F32 = 1e-5    # relative max-norm bound for FP32 results


def block_dicts(wl: synth.Workload):
    return [dict(n=b.n, ng=b.ng, h=b.h, boundary=b.boundary) for b in wl.blocks]


def op_fields(wl, ops):
    return [wl.nfields if (len(op) < 3 or op[2] < 0) else 1 for op in ops]


def biased_name(name):
    """(base name, bias) for a biased scheme name ("(1)X2-" -> ("(1)X2", -1); "(1)X2" -> upwind, 0;
    "(1)X2s" -> symmetrised, 2), else None."""
    if len(name) >= 5 and name.startswith("(1)") and name[3] in "UVXW" and name[4].isdigit():
        base, tail = name[:5], name[5:]
        return base, {"-": -1, "+": 1, "": 0, "s": 2}[tail]
    return None


def ko_name(name):
    """(r, sigma) for a Kreiss-Oliger operator named "KO<2r>[<sigma>]", else None."""
    if name.startswith("KO") and "[" in name and name.endswith("]"):
        deg, sig = name[2:-1].split("[")
        return int(deg) // 2, float(sig)
    return None


def scheme_for(name):
    import paper_2302_14858_amd as P
    ko = ko_name(name)
    return P.Scheme.dissipation(*ko) if ko else P.Scheme.named(name)


def make_plan(wl, ops, dtype=0):
    import paper_2302_14858_amd as P
    schemes = {}
    pops = []
    for op in ops:
        name = op[0]
        if name not in schemes:
            schemes[name] = scheme_for(name)
        pops.append((schemes[name], op[1], op[2] if len(op) > 2 else -1, op[3] if len(op) > 3 else -1,
                     op[4] if len(op) > 4 else -1, op[5] if len(op) > 5 else -1))
    return P.Plan(block_dicts(wl), wl.nfields, pops, dtype=dtype)


def oracle_block_op(wl, b, op, f, out=None):
    """The oracle's result of one operator on field f of block b ([z][y][x] interior)."""
    blk = wl.blocks[b]
    d = op[1]
    per = blk.boundary[d] == synth.PERIODIC
    ko = ko_name(op[0])
    if ko is not None:
        r = ODS.ko_block(wl.field_view(b, f), blk.ng, blk.h[d], d, ko[0], ko[1], periodic=per)
        if out is not None:
            out[...] = r
            return out
        return r
    if len(op) > 4 and op[4] >= 0:     # symmetrised mixed derivative along op[1], op[4]
        r = OM.mixed_block(OS.named(op[0]), wl.field_view(b, f), blk.ng, blk.h,
                           tuple(bd == synth.PERIODIC for bd in blk.boundary), d, op[4])
        if out is not None:
            out[...] = r
            return out
        return r
    bn = biased_name(op[0])
    if bn is None:
        return OL.apply_block(OS.named(op[0]), wl.field_view(b, f), blk.ng, blk.h[d], d, periodic=per, out=out)
    base, bias = bn
    ng = blk.ng
    interior = (slice(ng, ng + blk.n[2]), slice(ng, ng + blk.n[1]), slice(ng, ng + blk.n[0]))
    # U schemes: the sampled f'' is the field op[5] (interior)
    f2 = wl.field_view(b, op[5])[interior] if len(op) > 5 and op[5] >= 0 else None
    if bias == 0:
        c = wl.field_view(b, op[3])[interior]
        r = OB.upwind_block(base, wl.field_view(b, f), c, ng, blk.h[d], d, periodic=per, f2=f2)
    elif bias == 2:
        r = OB.symmetrised_block(base, wl.field_view(b, f), blk.ng, blk.h[d], d, periodic=per, f2=f2)
    elif f2 is not None:
        r = OB.apply_block_hermite(base, bias, wl.field_view(b, f), f2, blk.ng, blk.h[d], d, periodic=per)
    else:
        r = OB.apply_block(base, bias, wl.field_view(b, f), blk.ng, blk.h[d], d, periodic=per)
    if out is not None:
        out[...] = r
        return out
    return r


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
            fsel = list(range(wl.nfields)) if (len(op) < 3 or op[2] < 0) else [op[2]]
            per.append([oracle_block_op(wl, b, op, f) for f in fsel])
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


def oracle_flat(wl, ops, ooffs, nout, blocks=None):
    """The oracle's result in the plan's packed output layout (float64, NaN where nothing is written)."""
    ref = np.full(nout, np.nan)
    nf = op_fields(wl, ops)
    blocks = range(len(wl.blocks)) if blocks is None else blocks
    for b in blocks:
        blk = wl.blocks[b]
        nx, ny, nz = blk.n
        npts = nx * ny * nz
        slot = 0
        for o, op in enumerate(ops):
            d = op[1]
            fsel = list(range(wl.nfields)) if (len(op) < 3 or op[2] < 0) else [op[2]]
            for j, f in enumerate(fsel):
                off = ooffs[b] + (slot + j) * npts
                view = ref[off:off + npts].reshape(nz, ny, nx)
                oracle_block_op(wl, b, op, f, out=view)
            slot += nf[o]
    return ref


def compare_flat(got, ref, wl, ops, ooffs, blocks=None):
    """Worst relative max-norm error over every (block, operator, field) and every node.

    ``got`` is the whole output buffer as float64.  Raises if any output node is NaN or
    if a node the oracle defines was not written (the buffer is NaN-prefilled)."""
    assert got.shape == ref.shape
    written = ~np.isnan(ref)
    bad = np.isnan(got) & written
    assert not bad.any(), f"{int(bad.sum())} output nodes left unwritten (NaN), first at {int(np.argmax(bad))}"
    assert np.isfinite(got[written]).all(), "non-finite output"
    nf = op_fields(wl, ops)
    blocks = range(len(wl.blocks)) if blocks is None else blocks
    worst = 0.0
    for b in blocks:
        blk = wl.blocks[b]
        npts = int(np.prod(blk.n))
        for s in range(sum(nf)):
            off = ooffs[b] + s * npts
            worst = max(worst, rel_err(got[off:off + npts], ref[off:off + npts]))
    return worst


def full_parity(plan, wl, ops, dtype=0, ref=None):
    """Apply the plan once (eager, NaN-prefilled output) and return the worst relative error over
    every output node against the oracle (see compare_flat)."""
    import torch
    tdt = torch.float64 if dtype == 0 else torch.float32
    _, nout = plan.sizes()
    _, ooffs = plan.offsets()
    x = torch.from_numpy(wl.data).to(device="cuda", dtype=tdt)
    y = torch.full((nout,), float("nan"), dtype=tdt, device="cuda")
    plan.apply(x, y)
    torch.cuda.synchronize()
    got = y.double().cpu().numpy()
    if ref is None:
        ref = oracle_flat(wl, ops, ooffs, nout)
    return compare_flat(got, ref, wl, ops, ooffs)


def tol_for(dtype):
    return ERR_F64 if dtype == 0 else ERR_F32
