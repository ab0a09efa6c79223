"""GPU: the Runge-Kutta stage of the first-order wave system with the derivatives folded into the line
kernels (cfd_wave_rk_stage_fused) against the derivative apply followed by the separate stage kernel
(cfd_wave_rk_stage, cfd_wave_rk_stage_halo), bit for bit, and RK4 built on it against the closed form."""
import numpy as np
import pytest

import synth
from oracle import schemes as S
from oracle import wave as W

pytestmark = pytest.mark.gpu

SCHEME = "(1)Q1_3[1]"


def _blocks_of(case):
    """(blocks, lattice) of a test case."""
    P, C = synth.PERIODIC, synth.CLOSURE
    if case == "periodic":      # one periodic block, unequal extents (several partition counts)
        return [dict(n=(32, 24, 48), ng=4, h=(0.11, 0.12, 0.13), boundary=(P, P, P))], None
    if case == "closure":       # one block with closures on padded lines, ghosts as given
        return [dict(n=(20, 29, 17), ng=4, h=(0.1, 0.1, 0.1), boundary=(C, C, C))], None
    if case == "mixed":         # periodic along x, closures along y and z
        return [dict(n=(24, 21, 16), ng=4, h=(0.1, 0.1, 0.1), boundary=(P, C, C))], None
    if case == "lattice222":
        return [dict(n=(12, 12, 12), ng=4, h=(0.1, 0.1, 0.1), boundary=(C, C, C)) for _ in range(8)], (2, 2, 2)
    if case == "lattice312":
        return [dict(n=(8, 8, 8), ng=4, h=(0.1, 0.1, 0.1), boundary=(C, C, C)) for _ in range(6)], (3, 1, 2)
    raise ValueError(case)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("case", ["periodic", "closure", "mixed", "lattice222", "lattice312"])
def test_fused_stage_equals_apply_then_stage(cuda, case, dtype):
    """Every stage form of classical RK4 (acc_in = u0 with a stage state; in-place acc with a stage
    state; no stage state, acc written over u0's buffer) gives the same stage and acc buffers, ghosts
    included, as cfd_apply + the stage kernel."""
    import torch
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd.wave import wave_ops
    blocks, lattice = _blocks_of(case)
    plan = P.Plan(blocks, 5, wave_ops(P.Scheme.named(SCHEME)), dtype=dtype)
    nin, nout = plan.sizes()
    tdt = torch.float64 if dtype == 0 else torch.float32
    rng = np.random.default_rng(5)
    u0, src, stage0, acc0 = (torch.from_numpy(rng.standard_normal(nin)).to(device="cuda", dtype=tdt)
                             for _ in range(4))
    a, b = 0.0625, 0.03125
    for form in ("first", "middle", "last"):
        res = []
        for fused in (False, True):
            u, stage, acc = u0.clone(), stage0.clone(), acc0.clone()
            d = torch.full((nout,), float("nan"), device="cuda", dtype=tdt)
            if form == "first":
                args = dict(u0=u, stage=stage, acc=acc, acc_in=u)
            elif form == "middle":
                args = dict(u0=u, stage=stage, acc=acc, acc_in=acc)
            else:
                args = dict(u0=u, stage=None, acc=u, acc_in=acc)
            if fused:
                plan.wave_rk_stage_fused(args["u0"], src, args["stage"], args["acc"], d, a, b, lattice=lattice,
                                         acc_in=args["acc_in"])
            else:
                plan.apply(src, d)
                if lattice is None:
                    plan.wave_rk_stage(args["u0"], src, args["stage"], args["acc"], d, a, b, acc_in=args["acc_in"])
                else:
                    plan.wave_rk_stage_halo(args["u0"], src, args["stage"], args["acc"], d, a, b, *lattice,
                                            acc_in=args["acc_in"])
            torch.cuda.synchronize()
            res.append([t.cpu().numpy() for t in (u, stage, acc)])
        for name, x, y in zip(("u", "stage", "acc"), res[0], res[1]):
            assert np.array_equal(x, y), (form, name, int(np.sum(x != y)))


@pytest.mark.parametrize("dtype,tol", [(0, 1e-12), (1, 1e-5)])
def test_fused_rk4_periodic_closed_form(cuda, dtype, tol):
    """RK4 with fused stages on a periodic block against the discrete closed form (ERK4 applied to the
    scheme's modified wavenumber, oracle.wave)."""
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd.wave import WaveRK4
    n, steps = 24, 4
    wl = synth.wave192(n=n)
    h = wl.blocks[0].h[0]
    dt = 0.25 * h
    rk = WaveRK4([dict(n=b.n, ng=b.ng, h=b.h, boundary=b.boundary) for b in wl.blocks], P.Scheme.named(SCHEME),
                 dt, dtype=dtype, fused=True)
    rk.load(wl.data)
    rk.run(steps)
    got = rk.u.double().cpu().numpy().reshape(5, n, n, n)   # one periodic block, no ghosts
    amp = W.mode_evolution(S.named(SCHEME), synth.WAVE_K, h, dt, steps)
    x = np.arange(n) * h
    for f in range(5):
        ref = W.mode_field(amp[f], synth.WAVE_K, x, x, x)
        assert np.max(np.abs(got[f] - ref)) <= tol * np.max(np.abs(ref)), f


def test_fused_rk4_lattice_equals_unfused_and_oracle(cuda):
    """RK4 on a 2x2x2 block lattice (closures, ghost refresh in the epilogue): fused steps equal the
    unfused ones bit for bit, and the stepped oracle at 1e-12."""
    import torch
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd.wave import WaveRK4
    nb, ng, steps = 12, 4, 3
    wl = synth.wave192(n=24, blocks_per_dim=2, ng=ng)
    h = wl.blocks[0].h[0]
    dt = 0.25 * h
    blocks = [dict(n=b.n, ng=b.ng, h=b.h, boundary=b.boundary) for b in wl.blocks]
    ref_rk = WaveRK4(blocks, P.Scheme.named(SCHEME), dt, lattice=(2, 2, 2))
    rk = WaveRK4(blocks, P.Scheme.named(SCHEME), dt, lattice=(2, 2, 2), fused=True)
    ref_rk.load(wl.data)
    rk.load(wl.data)
    for s in range(steps):
        ref_rk.run(1)
        rk.run(1)
        torch.cuda.synchronize()
        assert torch.equal(rk.u, ref_rk.u), s
    got = rk.u.cpu().numpy()
    st = [[wl.field_view(b, f).copy() for f in range(5)] for b in range(8)]
    W.rk4_blocks(S.named(SCHEME), st, nb, ng, h, dt, steps, lattice=(2, 2, 2))
    ref = np.concatenate([a.ravel() for blk in st for a in blk])
    sl = (slice(None),) + (slice(ng, ng + nb),) * 3
    g = got.reshape(8, 5, nb + 2 * ng, nb + 2 * ng, nb + 2 * ng)
    r = ref.reshape(8, 5, nb + 2 * ng, nb + 2 * ng, nb + 2 * ng)
    for f in range(5):
        assert np.max(np.abs(g[:, f][sl] - r[:, f][sl])) <= 1e-12 * np.max(np.abs(r[:, f][sl])), f


def test_fused_rk4_graph_replay_and_tuned_schedule(cuda):
    """A captured fused step replays like the eager one, also after the plan's schedule is autotuned
    (the fused passes follow the tuned partitions), and still equals the unfused step."""
    import torch
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd.wave import WaveRK4
    wl = synth.wave192(n=48)
    h = wl.blocks[0].h[0]
    blocks = [dict(n=b.n, ng=b.ng, h=b.h, boundary=b.boundary) for b in wl.blocks]
    eager = WaveRK4(blocks, P.Scheme.named(SCHEME), 0.25 * h, fused=True)
    graph = WaveRK4(blocks, P.Scheme.named(SCHEME), 0.25 * h, fused=True)
    plain = WaveRK4(blocks, P.Scheme.named(SCHEME), 0.25 * h)
    plain.load(wl.data)
    plain.plan.autotune(plain.u, plain.d)
    sched = plain.plan.get_schedule()
    fl = sched["flags"]
    for rk in (eager, graph):           # the same partitions and launch shape (same rounding)
        for N, x, parts in sched["classes"]:
            rk.plan.set_schedule(N, bool(x), parts, persistent=bool(fl & 1), split_x=bool(fl & 2),
                                 xcd=bool(fl & 4), concurrent=bool(fl & 8))
    for rk in (eager, graph, plain):
        rk.load(wl.data)
    graph.capture()
    graph.load(wl.data)
    for rep in range(3):
        eager.run(1)
        graph.run(1)
        plain.run(1)
        torch.cuda.synchronize()
        assert torch.equal(eager.u, graph.u), rep
        assert torch.equal(eager.u, plain.u), rep


def test_fused_stage_rejections(cuda):
    """Host checks of cfd_wave_rk_stage_fused, made before any launch."""
    import torch
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd import _lib
    from paper_2302_14858_amd.wave import wave_ops
    sch = P.Scheme.named(SCHEME)
    blocks = [dict(n=(12, 12, 12), ng=4, h=(0.1, 0.1, 0.1), boundary=(synth.CLOSURE,) * 3) for _ in range(8)]
    plan = P.Plan(blocks, 5, wave_ops(sch))
    nin, nout = plan.sizes()
    u, s, acc = (torch.zeros(nin, dtype=torch.float64, device="cuda") for _ in range(3))
    w = torch.zeros(nout, dtype=torch.float64, device="cuda")

    def status(fn):
        with pytest.raises(P.CfdError) as ei:
            fn()
        return ei.value.status

    # stage or acc aliasing src, stage aliasing acc or u0, work aliasing a state buffer
    assert status(lambda: plan.wave_rk_stage_fused(u, s, s, acc, w, 0.1, 0.1)) == _lib.CFD_EINVAL
    assert status(lambda: plan.wave_rk_stage_fused(u, s, acc, s, w, 0.1, 0.1)) == _lib.CFD_EINVAL
    assert status(lambda: plan.wave_rk_stage_fused(u, s, acc, acc, w, 0.1, 0.1)) == _lib.CFD_EINVAL
    assert status(lambda: plan.wave_rk_stage_fused(u, s, u, acc, w, 0.1, 0.1)) == _lib.CFD_EINVAL
    assert status(lambda: plan.wave_rk_stage_fused(u, s, acc, u, acc, 0.1, 0.1, acc_in=u)) == _lib.CFD_EINVAL
    # lattices that do not match the blocks
    assert status(lambda: plan.wave_rk_stage_fused(u, u, s, acc, w, 0.1, 0.1, lattice=(2, 2, 1))) == _lib.CFD_EINVAL
    assert status(lambda: plan.wave_rk_stage_fused(u, u, s, acc, w, 0.1, 0.1, lattice=(8, 1, 0))) == _lib.CFD_EINVAL
    # not the wave system's operators
    other = P.Plan(blocks, 5, [(sch, 0, 1), (sch, 1, 1), (sch, 2, 1), (sch, 0, 2), (sch, 1, 3), (sch, 1, 4)])
    assert status(lambda: other.wave_rk_stage_fused(u, u, s, acc, w, 0.1, 0.1)) == _lib.CFD_EINVAL
    # off while the hybrid closure iteration is on, back when it is off again
    plan.set_iteration(2, 2, 2, 2)
    assert status(lambda: plan.wave_rk_stage_fused(u, u, s, acc, w, 0.1, 0.1)) == _lib.CFD_EUNSUPPORTED
    plan.set_iteration(0)
    plan.wave_rk_stage_fused(u, u, s, acc, w, 0.1, 0.1, lattice=(2, 2, 2), acc_in=u)
    torch.cuda.synchronize()
    # the dense mixed-precision path has no fused stage
    pb = [dict(n=(32, 32, 32), ng=4, h=(0.1, 0.1, 0.1), boundary=(synth.PERIODIC,) * 3)]
    dense = P.Plan(pb, 5, wave_ops(sch), dtype=P.CFD_MIXED_BF16)
    ni, no = dense.sizes()
    x = [torch.zeros(ni, dtype=torch.float32, device="cuda") for _ in range(3)]
    y = torch.zeros(no, dtype=torch.float32, device="cuda")
    assert status(lambda: dense.wave_rk_stage_fused(x[0], x[0], x[1], x[2], y, 0.1, 0.1)) == _lib.CFD_EUNSUPPORTED
