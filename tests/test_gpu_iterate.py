"""GPU parity of the hybrid closure iteration (Sec. ssec:domdec_iter, Eq. iter_center_P) against
the oracle (oracle/iterate.py), every output node, on periodic lattices of blocks.

Bar: relative max-norm error per (block, operator, field) <= 1e-12 in FP64 and <= 1e-5 in FP32.
"""
import numpy as np
import pytest

import synth
from oracle import iterate as IT
from oracle import lines as OL
from oracle import schemes as OS
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _ops(names, dirs=(0, 1, 2)):
    return [(n, d) for n in names for d in dirs]


def _iter_ref(wl, ops, lat, iters, ooffs, nout):
    """The oracle's iterate [iters] in the plan's output layout."""
    ref = np.full(nout, np.nan)
    nb = len(wl.blocks)
    n = wl.blocks[0].n
    npts = int(np.prod(n))
    keys = [(b % lat[0], (b // lat[0]) % lat[1], b // (lat[0] * lat[1])) for b in range(nb)]
    for o, (name, d) in enumerate(ops):
        s = OS.named(name)
        for f in range(wl.nfields):
            fields = {keys[b]: wl.field_view(b, f) for b in range(nb)}
            res = IT.iterate_lattice(s, fields, lat, wl.blocks[0].ng, wl.blocks[0].h[d], d, iters)
            for b in range(nb):
                off = ooffs[b] + (o * wl.nfields + f) * npts
                ref[off:off + npts] = res[keys[b]].ravel()
    return ref


def _run(plan, wl, dtype, graph=False):
    import torch
    tdt = torch.float64 if dtype == 0 else torch.float32
    _, nout = plan.sizes()
    x = torch.from_numpy(wl.data).to(device="cuda", dtype=tdt)
    y = torch.full((nout,), float("nan"), dtype=tdt, device="cuda")
    if graph:
        plan.capture_graph(x, y)
        plan.launch_graph()
    else:
        plan.apply(x, y)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("names", [("(1)Q1_3[1]", "(2)Q1_3[1]"), ("(1)P1_2",), ("(2)Q1_3[1]",)])
def test_iterates_match_oracle(cuda, names, dtype):
    lat = (3, 2, 2)
    wl = synth.lattice(n=(16, 12, 20), lat=lat, ng=4, nfields=2, seed=8)
    ops = _ops(names)
    plan = H.make_plan(wl, ops, dtype=dtype)
    _, ooffs = plan.offsets()
    _, nout = plan.sizes()
    for iters in (1, 2, 5):
        plan.set_iteration(iters, *lat)
        got = _run(plan, wl, dtype)
        ref = _iter_ref(wl, ops, lat, iters, ooffs, nout)
        err = H.compare_flat(got, ref, wl, ops, ooffs)
        print(f"iterate {iters} {names} dtype {dtype}: {err:.3e}", flush=True)
        assert err <= H.tol_for(dtype), (iters, err)
    # back to the plain block closure
    plan.set_iteration(0)
    got = _run(plan, wl, dtype)
    assert H.compare_flat(got, H.oracle_flat(wl, ops, ooffs, nout), wl, ops, ooffs) <= H.tol_for(dtype)


def test_iterates_converge_to_global_periodic_operator(cuda):
    """Many iterations give the global periodic operator on the box the lattice tiles."""
    lat = (2, 2, 3)
    n = (16, 16, 12)
    wl = synth.lattice(n=n, lat=lat, ng=4, nfields=1, seed=9)
    ops = _ops(["(1)Q1_3[1]"])
    plan = H.make_plan(wl, ops)
    plan.set_iteration(40, *lat)
    got = _run(plan, wl, 0, graph=True)
    _, ooffs = plan.offsets()
    NG = [n[d] * lat[d] for d in range(3)]
    s = OS.named("(1)Q1_3[1]")
    hh = wl.blocks[0].h
    glob = synth.Block(tuple(NG), 0, hh, (synth.PERIODIC,) * 3, tuple(0.5 * v for v in hh))
    data, offs = synth._fill([glob], 1, lambda b, f, x, y, z: synth.eval_modes(wl.modes[0][0], x, y, z))
    gw = synth.Workload("global", [glob], 1, data, offs)
    worst = 0.0
    npts = int(np.prod(n))
    for d in range(3):
        gref = OL.apply_block(s, gw.field_view(0, 0), 0, wl.blocks[0].h[d], d, periodic=True)
        for b, blk in enumerate(wl.blocks):
            kx, ky, kz = b % lat[0], (b // lat[0]) % lat[1], b // (lat[0] * lat[1])
            sub = gref[kz * n[2]:(kz + 1) * n[2], ky * n[1]:(ky + 1) * n[1], kx * n[0]:(kx + 1) * n[0]]
            off = ooffs[b] + d * npts
            worst = max(worst, H.rel_err(got[off:off + npts].reshape(n[2], n[1], n[0]), sub))
    assert worst <= 1e-12, worst


def test_iteration_graph_replays_equal_eager(cuda):
    import torch
    lat = (2, 2, 2)
    wl = synth.lattice(n=(16, 16, 16), lat=lat, ng=4, nfields=2, seed=10)
    ops = _ops(["(1)Q1_3[1]", "(2)Q1_3[1]"])
    plan = H.make_plan(wl, ops)
    plan.set_iteration(3, *lat)
    _, nout = plan.sizes()
    x = torch.from_numpy(wl.data).cuda()
    y0 = torch.empty(nout, dtype=torch.float64, device="cuda")
    plan.apply(x, y0)
    y = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.capture_graph(x, y)
    for rep in range(3):
        y.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.launch_graph()
        torch.cuda.synchronize()
        assert torch.equal(y, y0), rep
        x.mul_(1.0)


def test_iteration_rejects_what_it_cannot_do(cuda):
    import paper_2302_14858_amd as P
    lat = (2, 2, 2)
    wl = synth.lattice(n=(16, 16, 16), lat=lat, ng=5, nfields=1, seed=11)
    plan = H.make_plan(wl, _ops(["(1)QP_O8[1]"]))
    with pytest.raises(P.CfdError) as e:
        plan.set_iteration(2, *lat)
    assert e.value.status == P._lib.CFD_EUNSUPPORTED
    plan = H.make_plan(wl, _ops(["(1)Q1_3[1]"]))
    with pytest.raises(P.CfdError) as e:
        plan.set_iteration(2, 2, 2, 1)
    assert e.value.status == P._lib.CFD_EINVAL
    wl3 = synth.lattice(n=(16, 16, 16), lat=lat, ng=3, nfields=1, seed=11)
    plan = H.make_plan(wl3, _ops(["(1)Q1_3[1]:E"]))
    with pytest.raises(P.CfdError) as e:
        plan.set_iteration(2, *lat)
    assert e.value.status == P._lib.CFD_EGHOST


@pytest.mark.parametrize("name,fn", [("(1)P1_2", synth.paper_g), ("(1)Q1_3[1]", synth.paper_g),
                                     ("(2)P1_2", synth.paper_h)])
def test_decomposition_study_on_the_gpu(cuda, name, fn):
    """The decomposition study of Sec. 2.5 (the paper's g or h on N_M = 128 cell-centred samples, blocks
    of N_B = 16 with N_g = 4): the library's iterates 0..3 on the block lattice and its global periodic
    derivative match the oracle node by node, and give the oracle's modal RMS errors (Eq.
    err_met_rms_sp)."""
    import torch
    import paper_2302_14858_amd as P
    NM, NB, ng = 128, 16, 4
    s = OS.named(name)
    wl = synth.decomp_line(fn, NM=NM, NB=NB, ng=ng, ny=2, nz=2)
    h = wl.blocks[0].h[0]
    xg = (np.arange(NM) + 0.5) * h
    glob_ref = OL.apply_line(s, fn(xg), 0, h, periodic=True)
    scale = np.max(np.abs(glob_ref))
    # global periodic line on the GPU
    gb = [dict(n=(NM, 2, 2), ng=0, h=(h,) * 3, boundary=(synth.PERIODIC,) * 3)]
    gplan = P.Plan(gb, 1, [(P.Scheme.named(name), 0)])
    gx = torch.from_numpy(np.broadcast_to(fn(xg)[None, None, :], (2, 2, NM)).copy().ravel()).cuda()
    gy = torch.full((NM * 4,), float("nan"), dtype=torch.float64, device="cuda")
    gplan.apply(gx, gy)
    torch.cuda.synchronize()
    glob = gy.cpu().numpy().reshape(2, 2, NM)[0, 0]
    assert np.max(np.abs(glob - glob_ref)) <= 1e-12 * scale
    # decomposed, iterated
    blocks = [dict(n=b.n, ng=b.ng, h=b.h, boundary=b.boundary) for b in wl.blocks]
    plan = P.Plan(blocks, 1, [(P.Scheme.named(name), 0)])
    lines = np.stack([wl.field_view(b, 0)[ng, ng, :] for b in range(len(wl.blocks))])
    ref_its = IT.iterate_1d(s, lines, ng, h, 3)
    x = torch.from_numpy(wl.data).cuda()
    _, nout = plan.sizes()
    for i in range(4):
        plan.set_iteration(i, NM // NB, 1, 1)
        y = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
        plan.apply(x, y)
        torch.cuda.synchronize()
        got = y.cpu().numpy().reshape(NM // NB, 2, 2, NB)[:, 0, 0, :].reshape(-1)
        ref = ref_its[i].reshape(-1)
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale, i
        ea, et = IT.modal_rms_error(glob, got)
        ra, rt = IT.modal_rms_error(glob_ref, ref)
        if i <= 2:
            assert abs(ea - ra) <= 1e-3 * ra and abs(et - rt) <= 1e-3 * rt, (i, ea, ra, et, rt)


def _biased_lattice_iter(wl, lat, base, bias, d, f, iters):
    """The oracle's biased iterate [iters] (Eq. iter_left_X and its mirror) along direction d of a
    periodic lattice: block index -> interior [z][y][x]."""
    from oracle import biased as OB
    nb = len(wl.blocks)
    ng = wl.blocks[0].ng
    h = wl.blocks[0].h[d]
    ax = 2 - d
    keys = [(b % lat[0], (b // lat[0]) % lat[1], b // (lat[0] * lat[1])) for b in range(nb)]
    rows = {}
    for b, k in enumerate(keys):
        rows.setdefault(tuple(v for i, v in enumerate(k) if i != d), {})[k[d]] = b
    out = {}
    for members in rows.values():
        order = [members[i] for i in range(lat[d])]
        stack = np.stack([np.moveaxis(wl.field_view(b, f), ax, 0) for b in order])   # (NS, N+2ng, a, b)
        stack = stack[:, :, ng:-ng, ng:-ng]
        shp = stack.shape
        res = OB.iterate_1d(base, bias, stack.reshape(shp[0], shp[1], -1), ng, h, iters)[-1]
        res = res.reshape((shp[0], shp[1] - 2 * ng) + shp[2:])
        for i, b in enumerate(order):
            out[b] = np.moveaxis(res[i], 0, ax)
    return out


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("base", ["(1)X2", "(1)V3"])
def test_biased_iterates_match_oracle(cuda, base, dtype):
    """Iterated biased closures (Eq. iter_left_X and its mirror image) on a periodic lattice: the left
    and right biases, the upwind pair and the symmetrised mean along x, y and z, iterates 0..3,
    against the oracle at every output node."""
    import torch
    lat = (3, 2, 2)
    wl = synth.lattice(n=(16, 12, 20), lat=lat, ng=5, nfields=3, seed=12)
    ops = []
    for d in range(3):
        ops += [(base + "-", d, 1), (base + "+", d, 2), (base, d, 0, 1), (base + "s", d, 2)]
    plan = H.make_plan(wl, ops, dtype=dtype)
    _, nout = plan.sizes()
    _, ooffs = plan.offsets()
    tdt = torch.float64 if dtype == 0 else torch.float32
    x = torch.from_numpy(wl.data).to(device="cuda", dtype=tdt)
    nb = len(wl.blocks)
    ng = wl.blocks[0].ng
    for iters in range(4):
        plan.set_iteration(iters, *lat)
        y = torch.full((nout,), float("nan"), dtype=tdt, device="cuda")
        plan.apply(x, y)
        torch.cuda.synchronize()
        got = H.unpack(wl, ops, y.double().cpu().numpy(), ooffs)
        for o, op in enumerate(ops):
            d = op[1]
            L = _biased_lattice_iter(wl, lat, base, -1, d, op[2], iters)
            R = _biased_lattice_iter(wl, lat, base, +1, d, op[2], iters)
            for b in range(nb):
                if op[0].endswith("-"):
                    ref = L[b]
                elif op[0].endswith("+"):
                    ref = R[b]
                elif op[0].endswith("s"):
                    ref = 0.5 * (L[b] + R[b])
                else:
                    n = wl.blocks[b].n
                    c = wl.field_view(b, op[3])[ng:ng + n[2], ng:ng + n[1], ng:ng + n[0]]
                    ref = 0.5 * (c - np.abs(c)) * R[b] + 0.5 * (c + np.abs(c)) * L[b]
                g = got[b][o][0]
                err = np.max(np.abs(g - ref)) / max(np.max(np.abs(ref)), 1e-300)
                assert err <= H.tol_for(dtype), (iters, op, b, err)
    plan.set_iteration(0)


def test_biased_and_centred_iterate_together_and_replay(cuda):
    """A plan holding centred and biased operators iterates both (each against its oracle), and a
    captured graph of the iterated apply replays the eager result bit for bit."""
    import torch
    lat = (2, 2, 1)
    wl = synth.lattice(n=(16, 16, 12), lat=lat, ng=5, nfields=2, seed=13)
    ops = [("(1)Q1_3[1]", 0), ("(1)X2-", 1), ("(1)X2", 0, 0, 1), ("(2)Q1_3[1]", 1)]
    plan = H.make_plan(wl, ops)
    _, nout = plan.sizes()
    _, ooffs = plan.offsets()
    plan.set_iteration(2, *lat)
    x = torch.from_numpy(wl.data).cuda()
    y = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.apply(x, y)
    torch.cuda.synchronize()
    got = H.unpack(wl, ops, y.cpu().numpy(), ooffs)
    nb = len(wl.blocks)
    ng = wl.blocks[0].ng
    keys = [(b % lat[0], (b // lat[0]) % lat[1], b // (lat[0] * lat[1])) for b in range(nb)]
    for o, op in enumerate(ops):
        d = op[1]
        nfo = wl.nfields if len(op) < 3 or op[2] < 0 else 1
        for fi in range(nfo):
            f = fi if nfo > 1 else op[2]
            if op[0].startswith("(1)X2"):
                L = _biased_lattice_iter(wl, lat, "(1)X2", -1, d, f, 2)
                R = _biased_lattice_iter(wl, lat, "(1)X2", +1, d, f, 2)
            else:
                s = OS.named(op[0])
                ref_c = IT.iterate_lattice(s, {keys[b]: wl.field_view(b, f) for b in range(nb)}, lat, ng,
                                           wl.blocks[0].h[d], d, 2)
            for b in range(nb):
                if op[0] == "(1)X2-":
                    ref = L[b]
                elif op[0] == "(1)X2":
                    n = wl.blocks[b].n
                    c = wl.field_view(b, op[3])[ng:ng + n[2], ng:ng + n[1], ng:ng + n[0]]
                    ref = 0.5 * (c - np.abs(c)) * R[b] + 0.5 * (c + np.abs(c)) * L[b]
                else:
                    ref = ref_c[keys[b]]
                err = np.max(np.abs(got[b][o][fi] - ref)) / np.max(np.abs(ref))
                assert err <= H.ERR_F64, (op, b, fi, err)
    y1 = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.capture_graph(x, y1)
    for _ in range(3):
        plan.launch_graph()
        torch.cuda.synchronize()
        assert torch.equal(y, y1)
        y1.fill_(float("nan"))
        torch.cuda.synchronize()
    plan.set_iteration(0)


@pytest.mark.parametrize("seed", range(4))
def test_biased_iteration_seeded_sweep(cuda, seed):
    """Seeded random lattices, block extents, biased schemes, biases and iteration counts, against the
    oracle."""
    import torch
    rng = np.random.default_rng(200 + seed)
    base = ["(1)V1", "(1)V2", "(1)X1", "(1)X2", "(1)X3"][int(rng.integers(0, 5))]
    lat = tuple(int(v) for v in rng.integers(1, 4, size=3))
    if np.prod(lat) == 1:
        lat = (2, 1, 1)
    n = tuple(int(v) for v in rng.integers(9, 33, size=3))
    d = int(rng.integers(0, 3))
    iters = int(rng.integers(1, 4))
    suffix = ["-", "+", "s"][int(rng.integers(0, 3))]
    wl = synth.lattice(n=n, lat=lat, ng=5, nfields=1, seed=300 + seed)
    ops = [(base + suffix, d)]
    plan = H.make_plan(wl, ops)
    plan.set_iteration(iters, *lat)
    _, nout = plan.sizes()
    _, ooffs = plan.offsets()
    x = torch.from_numpy(wl.data).cuda()
    y = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.apply(x, y)
    torch.cuda.synchronize()
    got = H.unpack(wl, ops, y.cpu().numpy(), ooffs)
    L = _biased_lattice_iter(wl, lat, base, -1, d, 0, iters)
    R = _biased_lattice_iter(wl, lat, base, +1, d, 0, iters)
    for b in range(len(wl.blocks)):
        ref = {"-": L[b], "+": R[b], "s": 0.5 * (L[b] + R[b])}[suffix]
        err = np.max(np.abs(got[b][0][0] - ref)) / np.max(np.abs(ref))
        assert err <= H.ERR_F64, (seed, base + suffix, lat, n, d, iters, b, err)
