"""GPU parity of the time-stepping glue: ghost exchange, RK4 stages, graph capture."""
import numpy as np
import pytest

import synth
from oracle import schemes as S
from oracle import wave as W

pytestmark = pytest.mark.gpu


def _blocks(wl):
    return [dict(n=b.n, ng=b.ng, h=b.h, boundary=b.boundary) for b in wl.blocks]


def test_halo_exchange_matches_oracle(cuda):
    import torch
    import paper_2302_14858_amd as P
    wl = synth.wave192(n=24, blocks_per_dim=2, ng=4)
    sch = P.Scheme.named("(1)Q1_3[1]")
    plan = P.Plan(_blocks(wl), 5, [(sch, 0)])
    rng = np.random.default_rng(7)
    data = rng.standard_normal(wl.data.size)
    x = torch.from_numpy(data).cuda()
    plan.halo_exchange(x, 2, 2, 2)
    got = x.cpu().numpy()
    wl.data[:] = data
    st = [[wl.field_view(b, f).copy() for f in range(5)] for b in range(8)]
    W.fill_ghosts(st, 12, 4, (2, 2, 2))
    ref = np.concatenate([a.ravel() for blk in st for a in blk])
    # faces equal the oracle exactly; edges and corners are left untouched by both
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dtype,tol", [(0, 1e-12), (1, 1e-5)])
def test_rk4_periodic_closed_form(cuda, dtype, tol):
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd.wave import WaveRK4
    n, steps = 24, 4
    wl = synth.wave192(n=n)
    h = wl.blocks[0].h[0]
    dt = 0.25 * h
    rk = WaveRK4(_blocks(wl), P.Scheme.named("(1)Q1_3[1]"), dt, dtype=dtype)
    rk.load(wl.data)
    rk.run(steps)
    got = rk.u.double().cpu().numpy().reshape(5, n, n, n)
    amp = W.mode_evolution(S.named("(1)Q1_3[1]"), synth.WAVE_K, h, dt, steps)
    x = np.arange(n) * h
    for f in range(5):
        ref = W.mode_field(amp[f], synth.WAVE_K, x, x, x)
        assert np.max(np.abs(got[f] - ref)) <= tol * np.max(np.abs(ref)), f


def test_rk4_blocks_with_closures_and_halo(cuda):
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd.wave import WaveRK4
    nb, ng, steps = 12, 4, 3
    wl = synth.wave192(n=24, blocks_per_dim=2, ng=ng)
    h = wl.blocks[0].h[0]
    dt = 0.25 * h
    rk = WaveRK4(_blocks(wl), P.Scheme.named("(1)Q1_3[1]"), dt, lattice=(2, 2, 2))
    rk.load(wl.data)
    rk.run(steps)
    got = rk.u.cpu().numpy()
    st = [[wl.field_view(b, f).copy() for f in range(5)] for b in range(8)]
    W.rk4_blocks(S.named("(1)Q1_3[1]"), st, nb, ng, h, dt, steps, lattice=(2, 2, 2))
    ref = np.concatenate([a.ravel() for blk in st for a in blk])
    sl = (slice(ng, ng + nb),) * 3
    g = got.reshape(8, 5, nb + 2 * ng, nb + 2 * ng, nb + 2 * ng)
    r = ref.reshape(8, 5, nb + 2 * ng, nb + 2 * ng, nb + 2 * ng)
    for f in range(5):
        gi = g[:, f][(slice(None),) + sl]
        ri = r[:, f][(slice(None),) + sl]
        assert np.max(np.abs(gi - ri)) <= 1e-12 * np.max(np.abs(ri)), f


def test_rk4_graph_replay_matches_eager(cuda):
    import torch
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd.wave import WaveRK4
    wl = synth.wave192(n=24, blocks_per_dim=2, ng=4)
    h = wl.blocks[0].h[0]
    a = WaveRK4(_blocks(wl), P.Scheme.named("(1)Q1_3[1]"), 0.25 * h, lattice=(2, 2, 2))
    b = WaveRK4(_blocks(wl), P.Scheme.named("(1)Q1_3[1]"), 0.25 * h, lattice=(2, 2, 2))
    a.load(wl.data)
    b.load(wl.data)
    b.capture()                  # capture runs one warm-up step
    b.load(wl.data)
    for rep in range(3):
        a.run(1)
        b.run(1)
        torch.cuda.synchronize()
        assert torch.equal(a.u, b.u), rep


@pytest.mark.parametrize("lattice,nb", [((2, 2, 2), 12), ((3, 1, 2), 8)])
@pytest.mark.parametrize("dtype", [0, 1])
def test_fused_stage_halo_equals_stage_then_exchange(cuda, lattice, nb, dtype):
    """cfd_wave_rk_stage_halo = cfd_wave_rk_stage followed by cfd_halo_exchange of the state the next
    stage reads (stage, or acc when no stage is written), bit for bit, also with a lattice of extent 1."""
    import torch
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd.wave import wave_ops
    bx, by, bz = lattice
    blocks = [dict(n=(nb, nb, nb), ng=4, h=(0.1, 0.1, 0.1), boundary=(synth.CLOSURE,) * 3)
              for _ in range(bx * by * bz)]
    plan = P.Plan(blocks, 5, wave_ops(P.Scheme.named("(1)Q1_3[1]")), dtype=dtype)
    nin, nout = plan.sizes()
    tdt = torch.float64 if dtype == 0 else torch.float32
    rng = np.random.default_rng(11)
    u, src, stage0, acc0 = (torch.from_numpy(rng.standard_normal(nin)).to(device="cuda", dtype=tdt)
                            for _ in range(4))
    d = torch.from_numpy(rng.standard_normal(nout)).to(device="cuda", dtype=tdt)
    for with_stage in (True, False):
        res = []
        for fused in (False, True):
            stage, acc = stage0.clone(), acc0.clone()
            st = stage if with_stage else None
            if fused:
                plan.wave_rk_stage_halo(u, src, st, acc, d, 0.25, 0.125, *lattice)
            else:
                plan.wave_rk_stage(u, src, st, acc, d, 0.25, 0.125)
                plan.halo_exchange(stage if with_stage else acc, *lattice)
            torch.cuda.synchronize()
            res.append((stage.cpu().numpy(), acc.cpu().numpy()))
        assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1]), with_stage


def test_fused_stage_halo_rejects_bad_lattices(cuda):
    """Lattice checks of cfd_wave_rk_stage_halo, made on the host before any launch."""
    import torch
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd import _lib
    from paper_2302_14858_amd.wave import wave_ops
    sch = P.Scheme.named("(1)Q1_3[1]")

    def plan_of(shapes, ng=4):
        return P.Plan([dict(n=n, ng=ng, h=(0.1, 0.1, 0.1), boundary=(synth.CLOSURE,) * 3) for n in shapes], 5,
                      wave_ops(sch))

    def call(plan, lattice):
        nin, nout = plan.sizes()
        u = torch.zeros(nin, dtype=torch.float64, device="cuda")
        d = torch.zeros(nout, dtype=torch.float64, device="cuda")
        plan.wave_rk_stage_halo(u, u, u.clone(), u.clone(), d, 0.5, 0.5, *lattice)

    good = plan_of([(8, 8, 8)] * 2)
    for lattice, status in (((2, 2, 1), _lib.CFD_EINVAL), ((1, 1, 1), _lib.CFD_EINVAL), ((0, 2, 1), _lib.CFD_EINVAL)):
        with pytest.raises(P.CfdError) as e:
            call(good, lattice)
        assert e.value.status == status, lattice
    with pytest.raises(P.CfdError) as e:   # blocks of different shapes
        call(plan_of([(8, 8, 8), (8, 8, 12)]), (2, 1, 1))
    assert e.value.status == _lib.CFD_EINVAL
    call(good, (2, 1, 1))                  # the valid lattice runs
    torch.cuda.synchronize()


def _lattice_table(bx, by, bz):
    t = []
    for b in range(bx * by * bz):
        kx, ky, kz = b % bx, (b // bx) % by, b // (bx * by)
        idx = lambda x, y, z: ((z % bz) * by + (y % by)) * bx + (x % bx)
        t.append([idx(kx - 1, ky, kz), idx(kx + 1, ky, kz), idx(kx, ky - 1, kz), idx(kx, ky + 1, kz),
                  idx(kx, ky, kz - 1), idx(kx, ky, kz + 1)])
    return t


def _split_state(data, blocks, nfields):
    """Per-block, per-field [z][y][x] views of the flat plan input (default layout)."""
    out, off = [], 0
    for b in blocks:
        ng = b["ng"]
        shp = tuple(e + 2 * ng for e in reversed(b["n"]))
        size = int(np.prod(shp))
        out.append([data[off + f * size: off + (f + 1) * size].reshape(shp) for f in range(nfields)])
        off += nfields * size
    return out


def test_halo_table_equals_lattice_exchange_and_oracle(cuda):
    """cfd_halo_exchange_table with a periodic lattice's table = cfd_halo_exchange = the oracle."""
    import torch
    import paper_2302_14858_amd as P
    wl = synth.wave192(n=24, blocks_per_dim=2, ng=4)
    blocks = _blocks(wl)
    plan = P.Plan(blocks, 5, [(P.Scheme.named("(1)Q1_3[1]"), 0)])
    plan.set_neighbors(_lattice_table(2, 2, 2))
    rng = np.random.default_rng(8)
    data = rng.standard_normal(wl.data.size)
    x = torch.from_numpy(data).cuda()
    y = x.clone()
    plan.halo_exchange(x, 2, 2, 2)
    plan.halo_exchange_table(y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    st = _split_state(data.copy(), blocks, 5)
    W.fill_ghosts_table(st, 4, _lattice_table(2, 2, 2))
    ref = np.concatenate([a.ravel() for blk in st for a in blk])
    assert np.array_equal(y.cpu().numpy(), ref)


@pytest.mark.parametrize("dtype", [0, 1])
def test_halo_table_uneven_tiling(cuda, dtype):
    """Blocks of different extents along x (conforming faces), blocks that are their own neighbour and
    faces left alone (-1), against the oracle; replayed from a captured graph too."""
    import torch
    import paper_2302_14858_amd as P
    ng = 4
    C = synth.CLOSURE
    blocks = [dict(n=(nx, 10, 6), ng=ng, h=(0.1, 0.1, 0.1), boundary=(C, C, C)) for nx in (12, 20, 8)]
    blocks.append(dict(n=(12, 9, 6), ng=ng, h=(0.1, 0.1, 0.1), boundary=(C, C, C)))   # only its own neighbour
    table = [[2, 1, 0, 0, 0, 0], [0, 2, 1, 1, -1, -1], [1, 0, 2, 2, 2, 2], [3, 3, -1, 3, 3, -1]]
    plan = P.Plan(blocks, 3, [(P.Scheme.named("(1)Q1_3[1]"), 0)], dtype=dtype)
    plan.set_neighbors(table)
    nin, _ = plan.sizes()
    tdt = torch.float64 if dtype == 0 else torch.float32
    rng = np.random.default_rng(9)
    host = rng.standard_normal(nin).astype(np.float64 if dtype == 0 else np.float32)
    x = torch.from_numpy(host.copy()).cuda()
    plan.halo_exchange_table(x)
    torch.cuda.synchronize()
    st = _split_state(host.astype(np.float64), blocks, 3)
    W.fill_ghosts_table(st, ng, table)
    ref = np.concatenate([a.ravel() for blk in st for a in blk])
    assert np.array_equal(x.double().cpu().numpy(), ref)
    # captured: the same exchange replayed on fresh data
    g = torch.cuda.CUDAGraph()
    z = torch.from_numpy(host.copy()).cuda()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.halo_exchange_table(z, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    z.copy_(torch.from_numpy(host.copy()).to(device="cuda", dtype=tdt))
    with torch.cuda.graph(g):
        plan.halo_exchange_table(z, stream=torch.cuda.current_stream())
    for _ in range(2):
        z.copy_(torch.from_numpy(host.copy()).to(device="cuda", dtype=tdt))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(z, x)


def test_halo_table_rejections(cuda):
    """Host checks of cfd_plan_set_neighbors and cfd_halo_exchange_table."""
    import torch
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd import _lib
    C = synth.CLOSURE
    blocks = [dict(n=(12, 10, 6), ng=4, h=(0.1,) * 3, boundary=(C,) * 3),
              dict(n=(12, 8, 6), ng=4, h=(0.1,) * 3, boundary=(C,) * 3),
              dict(n=(3, 10, 6), ng=4, h=(0.1,) * 3, boundary=(C,) * 3)]
    plan = P.Plan(blocks, 1, [(P.Scheme.named("(1)E3"), 1)])
    nin, _ = plan.sizes()
    x = torch.zeros(nin, dtype=torch.float64, device="cuda")

    def status(fn):
        with pytest.raises(P.CfdError) as e:
            fn()
        return e.value.status

    assert status(lambda: plan.halo_exchange_table(x)) == _lib.CFD_EINVAL                  # no table yet
    none = [[-1] * 6 for _ in range(3)]
    bad = [r[:] for r in none]
    bad[0][1] = 3
    assert status(lambda: plan.set_neighbors(bad)) == _lib.CFD_EINVAL                       # out of range
    bad = [r[:] for r in none]
    bad[0][1] = 1                                                                           # ny 10 vs 8
    assert status(lambda: plan.set_neighbors(bad)) == _lib.CFD_ESHAPE
    bad = [r[:] for r in none]
    bad[0][1] = 2                                                                           # 3 < ng nodes
    assert status(lambda: plan.set_neighbors(bad)) == _lib.CFD_ESHAPE
    ok = [r[:] for r in none]
    ok[0][0] = ok[0][1] = 0
    plan.set_neighbors(ok)
    plan.halo_exchange_table(x)
    torch.cuda.synchronize()


def _vc_tiling():
    """Three vertex-centred blocks along x (11, 7 and 9 nodes: N_B + 1 each), y and z periodic onto
    themselves; ng = 4."""
    C = synth.CLOSURE
    blocks = [dict(n=(nx, 7, 6), ng=4, h=(0.1,) * 3, boundary=(C,) * 3) for nx in (11, 7, 9)]
    table = [[2, 1, 0, 0, 0, 0], [0, 2, 1, 1, 1, 1], [1, 0, 2, 2, 2, 2]]
    return blocks, table


@pytest.mark.parametrize("dtype", [0, 1])
def test_vertex_centred_exchange_and_average(cuda, dtype):
    """Vertex-centred tiling: the exchange continues past the shared node and the shared-node average
    (input layout, then the derivatives of the output layout) equals the oracle bit for bit."""
    import torch
    import paper_2302_14858_amd as P
    blocks, table = _vc_tiling()
    sch = P.Scheme.named("(1)Q1_3[1]")
    plan = P.Plan(blocks, 2, [(sch, 0), (sch, 1)], dtype=dtype)
    plan.set_neighbors_vc(table)
    nin, nout = plan.sizes()
    npdt = np.float64 if dtype == 0 else np.float32
    rng = np.random.default_rng(10)
    host = rng.standard_normal(nin).astype(npdt)
    x = torch.from_numpy(host.copy()).cuda()
    plan.halo_exchange_table(x)
    plan.shared_node_average(x)
    torch.cuda.synchronize()
    st = _split_state(host.copy(), blocks, 2)
    W.fill_ghosts_table(st, 4, table, shared=1)
    W.shared_node_average(st, 4, table)
    ref = np.concatenate([a.ravel() for blk in st for a in blk])
    assert np.array_equal(x.cpu().numpy(), ref)
    # derivatives of the exchanged, averaged data; then their shared nodes averaged
    y = torch.full((nout,), float("nan"), dtype=x.dtype, device="cuda")
    plan.apply(x, y)
    torch.cuda.synchronize()
    raw = y.cpu().numpy().copy()
    plan.shared_node_average(y, output=True)
    torch.cuda.synchronize()
    outs, off = [], 0
    for b in blocks:
        shp = tuple(reversed(b["n"]))
        size = int(np.prod(shp))
        outs.append([raw[off + k * size: off + (k + 1) * size].reshape(shp) for k in range(2 * 2)])
        off += 4 * size
    W.shared_node_average(outs, 0, table)
    ref_out = np.concatenate([a.ravel() for blk in outs for a in blk])
    assert np.array_equal(y.cpu().numpy(), ref_out)


def test_vertex_centred_corner_nodes_on_a_lattice(cuda):
    """A 2x2x2 periodic lattice of vertex-centred blocks: nodes shared by 2, 4 and 8 blocks end with
    the mean of their copies, as in the oracle."""
    import torch
    import paper_2302_14858_amd as P
    C = synth.CLOSURE
    blocks = [dict(n=(6, 6, 6), ng=4, h=(0.1,) * 3, boundary=(C,) * 3) for _ in range(8)]
    plan = P.Plan(blocks, 1, [(P.Scheme.named("(1)Q1_3[1]"), 0)])
    table = _lattice_table(2, 2, 2)
    plan.set_neighbors_vc(table)
    nin, _ = plan.sizes()
    host = np.random.default_rng(11).standard_normal(nin)
    x = torch.from_numpy(host.copy()).cuda()
    plan.shared_node_average(x)
    torch.cuda.synchronize()
    st = _split_state(host.copy(), blocks, 1)
    W.shared_node_average(st, 4, table)
    assert np.array_equal(x.cpu().numpy(), np.concatenate([a.ravel() for blk in st for a in blk]))


def test_vertex_centred_rejections(cuda):
    import torch
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd import _lib
    blocks, table = _vc_tiling()
    plan = P.Plan(blocks, 1, [(P.Scheme.named("(1)Q1_3[1]"), 1)])
    nin, _ = plan.sizes()
    x = torch.zeros(nin, dtype=torch.float64, device="cuda")

    def status(fn):
        with pytest.raises(P.CfdError) as e:
            fn()
        return e.value.status

    assert status(lambda: plan.shared_node_average(x)) == _lib.CFD_EINVAL       # no table
    plan.set_neighbors(table)                                                  # cell-centred table
    assert status(lambda: plan.shared_node_average(x)) == _lib.CFD_EINVAL
    bad = [r[:] for r in table]
    bad[0][1] = 2                                                               # 0 -> 2, but 2's x- is 1
    assert status(lambda: plan.set_neighbors_vc(bad)) == _lib.CFD_EINVAL
    thin = [dict(n=(11, 7, 6), ng=4, h=(0.1,) * 3, boundary=(synth.CLOSURE,) * 3),
            dict(n=(4, 7, 6), ng=4, h=(0.1,) * 3, boundary=(synth.CLOSURE,) * 3)]
    p2 = P.Plan(thin, 1, [(P.Scheme.named("(1)Q1_3[1]"), 1)])
    with pytest.raises(P.CfdError) as e:                                        # 4 nodes < ng + 1
        p2.set_neighbors_vc([[1, 1, -1, -1, -1, -1], [0, 0, -1, -1, -1, -1]])
    assert e.value.status == _lib.CFD_ESHAPE
    plan.set_neighbors_vc(table)
    plan.halo_exchange_table(x)
    plan.shared_node_average(x)
    torch.cuda.synchronize()


@pytest.mark.parametrize("seed", range(6))
def test_halo_table_seeded_sweep(cuda, seed):
    """Seeded random conforming tilings: a row of blocks along one direction with random extents along
    it (equal across it), random open faces, either sampling, random ghost width and dtype; the
    exchange (and for vertex-centred tilings the shared-node average) against the oracle."""
    import torch
    import paper_2302_14858_amd as P
    rng = np.random.default_rng(100 + seed)
    d = int(rng.integers(0, 3))
    nb = int(rng.integers(1, 5))
    ng = int(rng.integers(1, 5))
    vc = bool(rng.integers(0, 2))
    dtype = int(rng.integers(0, 2))
    base = [int(rng.integers(ng + 2, 14)) for _ in range(3)]
    blocks = []
    for i in range(nb):
        n = list(base)
        n[d] = int(rng.integers(ng + 2, 20))
        blocks.append(dict(n=tuple(n), ng=ng, h=(0.1,) * 3, boundary=(synth.CLOSURE,) * 3))
    table = []
    for i in range(nb):
        row = [i, i, i, i, i, i]                       # transverse faces: periodic onto the block itself
        row[2 * d] = (i - 1) % nb
        row[2 * d + 1] = (i + 1) % nb
        table.append(row)
    if not vc:                                         # open a few faces (vertex-centred faces must stay mutual)
        for i in range(nb):
            for f in range(6):
                if rng.random() < 0.2:
                    table[i][f] = -1
    plan = P.Plan(blocks, 2, [(P.Scheme.named("(1)E1"), (d + 1) % 3)], dtype=dtype)
    (plan.set_neighbors_vc if vc else plan.set_neighbors)(table)
    nin, _ = plan.sizes()
    npdt = np.float64 if dtype == 0 else np.float32
    host = rng.standard_normal(nin).astype(npdt)
    x = torch.from_numpy(host.copy()).cuda()
    plan.halo_exchange_table(x)
    if vc:
        plan.shared_node_average(x)
    torch.cuda.synchronize()
    st = _split_state(host.copy(), blocks, 2)
    W.fill_ghosts_table(st, ng, table, shared=1 if vc else 0)
    if vc:
        W.shared_node_average(st, ng, table)
    assert np.array_equal(x.cpu().numpy(), np.concatenate([a.ravel() for blk in st for a in blk])), (seed, d, nb, vc)
