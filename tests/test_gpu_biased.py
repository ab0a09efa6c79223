"""GPU parity of the biased (upwind) compact schemes (Sec. ssec:domdec_drp).

Left-biased, right-biased and upwind operators (Eqs. closure_left_X and
biasderapproxadv) on closure and periodic lines, every direction, FP64 and
FP32, against oracle/biased.py on the same seeded inputs; every output node is
compared (NaN-prefilled output).  Bar: relative max-norm error per (block,
operator, field) <= 1e-12 in FP64, <= 1e-5 in FP32.
"""
import numpy as np
import pytest

import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("name", ["(1)V1", "(1)V2", "(1)V3", "(1)V4", "(1)X1", "(1)X2", "(1)X3"])
def test_biased_closure_blocks(cuda, name, dtype):
    """Both biases and the upwind pair along x, y, z on uneven closure blocks (ragged line counts,
    lengths 7..48), velocity = field 1 (sign changes inside the blocks)."""
    from oracle import biased as OB
    ng = OB.required_ghosts(name)
    wl = synth.batch64(nblocks=6, nfields=3, sizes=(7, 16, 23, 48), ng=ng, seed=21)
    ops = []
    for d in range(3):
        ops += [(name + "-", d), (name + "+", d, 2), (name, d, -1, 1)]
    plan = H.make_plan(wl, ops, dtype=dtype)
    err = H.full_parity(plan, wl, ops, dtype)
    assert err <= H.tol_for(dtype), err


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("name", ["(1)V2", "(1)X1", "(1)X2", "(1)X3"])
def test_biased_periodic_lines(cuda, name, dtype):
    """Cyclic biased systems closed by their wrap value, a different line length per direction
    (including lines shorter than the stencil, which wrap onto themselves)."""
    wl = synth.periodic_box(n=(64, 5, 9), nfields=2, seed=22)
    ops = []
    for d in range(3):
        ops += [(name + "-", d), (name + "+", d), (name, d, 0, 1)]
    plan = H.make_plan(wl, ops, dtype=dtype)
    err = H.full_parity(plan, wl, ops, dtype)
    assert err <= H.tol_for(dtype), err


def test_biased_with_centred_operators_and_graph(cuda):
    """One plan mixing centred (banded kernel) and upwind (biased kernel) operators; the captured
    graph replays the eager result bit for bit."""
    import torch
    wl = synth.batch64(nblocks=5, nfields=4, ng=5, seed=23)
    ops = [("(1)QP_O8[1]", 0), ("(2)QP_O8[1]", 1), ("(1)X2", 0, -1, 0), ("(1)X2", 1, 3, 1), ("(1)X2", 2, -1, 2)]
    plan = H.make_plan(wl, ops)
    err = H.full_parity(plan, wl, ops)
    assert err <= H.ERR_F64, err
    _, nout = plan.sizes()
    x = torch.from_numpy(wl.data).cuda()
    y0 = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.apply(x, y0)
    y1 = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.capture_graph(x, y1)
    for _ in range(3):
        plan.launch_graph()
        torch.cuda.synchronize()
        assert torch.equal(y0, y1)
        y1.fill_(float("nan"))
        torch.cuda.synchronize()


def test_biased_concurrent_classes_match_sequential(cuda):
    """The biased kernel classes (x and y/z lines, several partition lengths) launched on forked
    streams give the sequential launches' output bit for bit, eagerly and as a replayed graph; a
    plan of only biased operators autotunes just that flag and keeps the result."""
    import torch
    import paper_2302_14858_amd as P
    wl = synth.batch64(nblocks=6, nfields=3, sizes=(16, 24, 48), ng=5, seed=25)
    ops = [("(1)X2", d, -1, d) for d in range(3)]
    plan = H.make_plan(wl, ops)
    _, nout = plan.sizes()
    x = torch.from_numpy(wl.data).cuda()
    ys = []
    for conc in (False, True):
        plan.set_schedule(concurrent=conc)
        y = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
        plan.apply(x, y)
        torch.cuda.synchronize()
        ys.append(y)
    assert torch.equal(ys[0], ys[1])
    y1 = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.capture_graph(x, y1)
    for _ in range(3):
        plan.launch_graph()
        torch.cuda.synchronize()
        assert torch.equal(ys[0], y1)
        y1.fill_(float("nan"))
        torch.cuda.synchronize()
    y2 = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.autotune(x, y2)
    y2.fill_(float("nan"))
    plan.apply(x, y2)
    torch.cuda.synchronize()
    assert torch.equal(ys[0], y2)
    assert plan.get_schedule()["concurrent"] in (False, True)
    err = H.full_parity(plan, wl, ops)
    assert err <= H.ERR_F64, err


def test_upwind_sign_selection_on_constant_velocity(cuda):
    """With c = +1 everywhere the upwind pair equals the left-biased operator bit for bit, with
    c = -1 minus the right-biased one (the kernel's min/max weights are exact)."""
    import torch
    wl = synth.batch64(nblocks=3, nfields=3, ng=4, seed=24)
    for b in range(len(wl.blocks)):
        wl.field_view(b, 1)[...] = 1.0
        wl.field_view(b, 2)[...] = -1.0
    ops = [("(1)X2-", 1, 0), ("(1)X2", 1, 0, 1), ("(1)X2+", 1, 0), ("(1)X2", 1, 0, 2)]
    plan = H.make_plan(wl, ops)
    _, nout = plan.sizes()
    x = torch.from_numpy(wl.data).cuda()
    y = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.apply(x, y)
    torch.cuda.synchronize()
    g = H.unpack(wl, ops, y.cpu().numpy(), plan.offsets()[1])
    for b in range(len(wl.blocks)):
        assert np.array_equal(g[b][0][0], g[b][1][0])
        assert np.array_equal(-g[b][2][0], g[b][3][0])


def test_biased_plan_validation(cuda):
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd import _lib
    wl = synth.batch64(nblocks=2, nfields=2, ng=3, seed=25)
    bd = H.block_dicts(wl)
    x2 = P.Scheme.named("(1)X2")
    with pytest.raises(P.CfdError) as e:                 # X2 needs 4 ghost layers
        P.Plan(bd, 2, [(x2, 0, -1, 1)])
    assert e.value.status == _lib.CFD_EGHOST
    x1 = P.Scheme.named("(1)X1")
    with pytest.raises(P.CfdError) as e:                 # upwind pair without a velocity field
        P.Plan(bd, 2, [(x1, 0, -1, -1)])
    assert e.value.status == _lib.CFD_EINVAL
    with pytest.raises(P.CfdError) as e:                 # velocity index out of range
        P.Plan(bd, 2, [(x1, 0, -1, 2)])
    assert e.value.status == _lib.CFD_EINVAL
    with pytest.raises(P.CfdError) as e:                 # a centred scheme reads no velocity
        P.Plan(bd, 2, [(P.Scheme.named("(1)Q1_3[1]"), 0, -1, 1)])
    assert e.value.status == _lib.CFD_EINVAL
    with pytest.raises(P.CfdError) as e:
        P.Plan(bd, 2, [(P.Scheme.named("(1)X1-"), 0)], dtype=P.CFD_MIXED_BF16)
    assert e.value.status == _lib.CFD_EUNSUPPORTED
    plan = P.Plan(bd, 2, [(P.Scheme.named("(1)X1-"), 0)])
    wlat = synth.lattice(n=(8, 8, 8), lat=(2, 1, 1), ng=4, nfields=1)
    p2 = P.Plan(H.block_dicts(wlat), 1, [(P.Scheme.named("(1)X2-"), 0)])
    p2.set_iteration(1, 2, 1, 1)                          # iterated biased closures are supported
    wlong = synth.lattice(n=(80, 4, 4), lat=(2, 1, 1), ng=4, nfields=1)
    with pytest.raises(P.CfdError) as e:                 # ... on lines of at most 64 nodes
        p3 = P.Plan(H.block_dicts(wlong), 1, [(P.Scheme.named("(1)X2-"), 0)])
        p3.set_iteration(1, 2, 1, 1)
    assert e.value.status == _lib.CFD_EUNSUPPORTED
    del plan


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("name", ["(1)V3s", "(1)X2s"])
def test_symmetrised_biased(cuda, name, dtype):
    """The mean of both biases, along x, y, z: closure blocks (lengths 7..48, the partitioned kernel),
    a periodic box, and lines of 80 nodes (the sweep kernel), against the oracle."""
    for wl in (synth.batch64(nblocks=5, nfields=2, sizes=(7, 16, 48), ng=5, seed=26),
               synth.periodic_box(n=(64, 5, 9), nfields=2, seed=27),
               synth.batch64(nblocks=2, nfields=1, sizes=(80,), ng=5, seed=28)):
        ops = [(name, d) for d in range(3)]
        plan = H.make_plan(wl, ops, dtype=dtype)
        err = H.full_parity(plan, wl, ops, dtype)
        assert err <= H.tol_for(dtype), (wl.name, err)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("M", [1, 2, 3])
def test_w_schemes_embedded_second_derivative(cuda, M, dtype):
    """W_M (Tab. ccuw_deg_one_col): both biases, the upwind pair and the symmetrised mean along x, y, z,
    each interior row taking the compact (2)P1_M second derivative that a line pass leaves in the plan
    scratch before the biased launches: closure blocks (lengths 7..48, the partitioned kernel; N_g =
    M + 2 and one more), a periodic box (line lengths the periodic line kernel takes for the embedded
    pass: partitions of 8..32 rows), and lines of 80 nodes (the sweep kernel), against the oracle."""
    from oracle import biased as OB
    name = f"(1)W{M}"
    ng = OB.required_ghosts(name)
    for wl in (synth.batch64(nblocks=5, nfields=3, sizes=(7, 16, 23, 48), ng=ng, seed=31 + M),
               synth.batch64(nblocks=3, nfields=2, sizes=(9, 16), ng=ng + 1, seed=34 + M),
               synth.periodic_box(n=(64, 8, 12), nfields=2, seed=37 + M),
               synth.batch64(nblocks=2, nfields=2, sizes=(80, 12), ng=ng, seed=40 + M)):
        ops = []
        for d in range(3):
            ops += [(name + "-", d), (name + "+", d, 1), (name, d, -1, 1), (name + "s", d)]
        plan = H.make_plan(wl, ops, dtype=dtype)
        err = H.full_parity(plan, wl, ops, dtype)
        assert err <= H.tol_for(dtype), (wl.name, err)


def test_w_scheme_in_a_mixed_plan_and_graph(cuda):
    """W operators beside centred and X operators in one plan (the embedded pass shares the launch
    groups of the centred passes; the biased launches follow them), autotuned; the captured graph
    replays the eager result bit for bit, and cfd_plan_set_iteration refuses the plan."""
    import torch
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd import _lib
    wl = synth.batch64(nblocks=5, nfields=4, ng=5, seed=44)
    ops = [("(1)QP_O8[1]", 0), ("(2)QP_O8[1]", 1), ("(1)W2-", 0, 2), ("(1)W3", 1, -1, 0), ("(1)X2+", 2),
           ("(1)W1s", 2, 3)]
    plan = H.make_plan(wl, ops)
    err = H.full_parity(plan, wl, ops)
    assert err <= H.ERR_F64, err
    _, nout = plan.sizes()
    x = torch.from_numpy(wl.data).cuda()
    y0 = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.autotune(x, y0)
    y0.fill_(float("nan"))
    plan.apply(x, y0)
    torch.cuda.synchronize()
    assert not torch.isnan(y0).any()
    y1 = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    plan.capture_graph(x, y1)
    for _ in range(3):
        plan.launch_graph()
        torch.cuda.synchronize()
        assert torch.equal(y0, y1)
        y1.fill_(float("nan"))
        torch.cuda.synchronize()
    with pytest.raises(P.CfdError) as e:
        plan.set_iteration(1, 5, 1, 1)
    assert e.value.status == _lib.CFD_EUNSUPPORTED



@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("M", [1, 2, 3])
def test_u_schemes_with_sampled_second_derivative(cuda, M, dtype):
    """U_M (Tab. ucd_slow, closure of Tab. ucd_slow_closure) reading f'' from another field of the
    block on every row, the closure row included: both biases, the upwind pair and the symmetrised
    mean along x, y, z on closure blocks (lengths 7..48 and 80, both kernels) and a periodic box.  The
    f'' field is independent data, so every term of the rows is exercised."""
    from oracle import biased as OB
    name = f"(1)U{M}"
    ng = OB.required_ghosts(name)
    for wl in (synth.batch64(nblocks=5, nfields=3, sizes=(7, 16, 23, 48), ng=ng, seed=51 + M),
               synth.periodic_box(n=(64, 5, 9), nfields=3, seed=54 + M),
               synth.batch64(nblocks=2, nfields=3, sizes=(80, 12), ng=ng, seed=57 + M)):
        ops = []
        for d in range(3):
            ops += [(name + "-", d, 0, -1, -1, 2), (name + "+", d, 1, -1, -1, 2), (name, d, 0, 1, -1, 2),
                    (name + "s", d, 2, -1, -1, 0)]
        plan = H.make_plan(wl, ops, dtype=dtype)
        err = H.full_parity(plan, wl, ops, dtype)
        assert err <= H.tol_for(dtype), (wl.name, err)


def test_u_scheme_validation(cuda):
    """A U operator needs a single field and the field of its sampled f''; other schemes refuse an
    aux_field; the hybrid iteration is refused for plans holding U operators."""
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd import _lib
    wl = synth.lattice(n=(16, 16, 16), lat=(2, 1, 1), ng=4, nfields=2)
    blocks = H.block_dicts(wl)
    u = P.Scheme.named("(1)U2-")
    for ops in ([(u, 0)], [(u, 0, 0)], [(u, 0, 0, -1, -1, 2)], [(u, 0, -1, -1, -1, 1)],
                [(P.Scheme.named("(1)X2-"), 0, 0, -1, -1, 1)]):
        with pytest.raises(P.CfdError) as e:
            P.Plan(blocks, 2, ops)
        assert e.value.status == _lib.CFD_EINVAL
    plan = P.Plan(blocks, 2, [(u, 0, 0, -1, -1, 1)])
    with pytest.raises(P.CfdError) as e:
        plan.set_iteration(1, 2, 1, 1)
    assert e.value.status == _lib.CFD_EUNSUPPORTED


@pytest.mark.parametrize("seed", range(4))
def test_u_w_seeded_sweep(cuda, seed):
    """Seeded sweep: random block extents (7..64), ghost widths, schemes among U_1..U_3 and W_1..W_3,
    biases (-, +, s, upwind), directions, field selections and dtypes, against the oracle."""
    from oracle import biased as OB
    rng = np.random.default_rng(900 + seed)
    kind = ["U", "W"][seed % 2]
    M = int(rng.integers(1, 4))
    name = f"(1){kind}{M}"
    ng = OB.required_ghosts(name) + int(rng.integers(0, 2))
    sizes = tuple(int(v) for v in rng.choice([7, 9, 13, 16, 20, 31, 40, 64], size=3, replace=False))
    wl = synth.batch64(nblocks=int(rng.integers(2, 5)), nfields=3, sizes=sizes, ng=ng, seed=950 + seed)
    dtype = int(rng.integers(0, 2))
    ops = []
    for d in range(3):
        suf = ["-", "+", "s", ""][int(rng.integers(0, 4))]
        f = int(rng.integers(0, 3))
        aux = (f + 1) % 3 if kind == "U" else -1
        vel = (f + 2) % 3 if suf == "" else -1
        if kind == "W" and rng.random() < 0.5 and suf != "":
            ops.append((name + suf, d))                      # every field
        else:
            ops.append((name + suf, d, f, vel, -1, aux))
    plan = H.make_plan(wl, ops, dtype=dtype)
    err = H.full_parity(plan, wl, ops, dtype)
    assert err <= H.tol_for(dtype), (name, ops, sizes, ng, dtype, err)
