"""The C ABI without a GPU: exported symbols, scheme construction on the host,
validation and error paths.  No kernel is launched here."""
import ctypes
import re
import os

import numpy as np
import pytest

import paper_2302_14858_amd as P
from paper_2302_14858_amd import _lib
from oracle import schemes as OS

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "cfd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cfd_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_abi_version():
    assert P.cfd_abi_version() == 3


NAMES = ["(1)P1_1", "(2)P1_1", "(1)P1_2", "(2)P1_2", "(1)P1_3", "(2)P1_3", "(1)Q1_3[1]", "(2)Q1_3[1]",
         "(1)Q1_3[4pi/5]", "(2)Q1_3[4pi/5]", "(1)QP_O8[1]", "(2)QP_O8[1]", "(1)Q1_3[1]:E", "(2)QP_O8[1]:E",
         "(1)E3", "(2)E4"]


@pytest.mark.parametrize("name", NAMES)
def test_registry_matches_oracle_construction(name):
    """The library's binary128 construction and the oracle's exact/mpmath one agree to round-off."""
    g = P.Scheme.named(name).get()
    o = OS.named(name)
    lhs = np.zeros(5)
    lhs[2 - o.nl:3 + o.nl] = o.lhs_floats()
    rhs = np.zeros(11)
    rhs[5 - o.M:6 + o.M] = o.rhs_floats()
    assert np.max(np.abs(lhs - g["lhs"])) <= 2e-16
    assert np.max(np.abs(rhs - g["rhs"])) <= 4e-16 * max(1, np.max(np.abs(rhs)))
    mc, rows = o.closure_floats()
    for j, r in enumerate(rows):
        c = np.zeros(11)
        c[5 - mc:6 + mc] = r
        assert np.max(np.abs(c - np.array(g["closure"][j]))) <= 4e-16 * max(1, np.max(np.abs(c)))
    assert P.Scheme.named(name).required_ghosts() == OS.required_ghosts(o, False)
    assert P.Scheme.named(name).required_ghosts(P.CFD_BOUNDARY_PERIODIC) == 0


def test_design_general_scheme():
    """cfd_scheme_design reproduces the registry entry it generalises."""
    a = P.Scheme.design(1, 6, 1, 3, 1.0, 4, True).get()
    b = P.Scheme.named("(1)Q1_3[1]").get()
    assert np.allclose(a["lhs"], b["lhs"], atol=1e-16) and np.allclose(a["rhs"], b["rhs"], atol=1e-16)


def test_create_from_paper_table():
    """(1)P1_2 with its closure typed from Tab. pade_deg_one is accepted."""
    s = P.Scheme.create(1, 6, [1 / 3, 1, 1 / 3], [-1 / 36, -28 / 36, 0, 28 / 36, 1 / 36],
                        [[v / 300 for v in (1, -11, 59, -239, 0, 239, -59, 11, -1)]])
    g = s.get()
    assert g["nl"] == 1 and g["mc"] == 4
    assert s.required_ghosts() == 4


def test_create_rejects_inconsistent_coefficients():
    with pytest.raises(P.CfdError) as e:
        P.Scheme.create(1, 6, [1 / 3, 1, 1 / 3], [-1 / 36, -28 / 36, 0, 28 / 36, 1.01 / 36],
                        [[v / 300 for v in (1, -11, 59, -239, 0, 239, -59, 11, -1)]])
    assert e.value.status == _lib.CFD_EINVAL
    with pytest.raises(P.CfdError):
        P.Scheme.create(1, 6, [1 / 3, 0.9, 1 / 3], [-1 / 36, -28 / 36, 0, 28 / 36, 1 / 36], [[0.0] * 9])


def test_unknown_name():
    with pytest.raises(P.CfdError) as e:
        P.Scheme.named("(1)Z9")
    assert e.value.status == _lib.CFD_EINVAL
    assert "unknown" in str(e.value)


def _blk(n=(16, 16, 16), ng=4, boundary=(0, 0, 0)):
    return dict(n=n, ng=ng, h=(0.1, 0.1, 0.1), boundary=boundary)


def test_plan_ghost_width_checked():
    s = P.Scheme.named("(1)QP_O8[1]")      # needs 5 ghost layers
    with pytest.raises(P.CfdError) as e:
        P.Plan([_blk(ng=4)], 1, [(s, 0)])
    assert e.value.status == _lib.CFD_EGHOST


def test_plan_short_line_rejected():
    s = P.Scheme.named("(1)QP_O8[1]")
    with pytest.raises(P.CfdError) as e:
        P.Plan([_blk(n=(4, 16, 16), ng=5)], 1, [(s, 0)])
    assert e.value.status == _lib.CFD_ESHAPE


def test_plan_bad_arguments():
    s = P.Scheme.named("(1)Q1_3[1]")
    with pytest.raises(P.CfdError) as e:
        P.Plan([_blk()], 1, [(s, 3)])
    assert e.value.status == _lib.CFD_EINVAL
    with pytest.raises(P.CfdError) as e:
        P.Plan([_blk()], 2, [(s, 0, 5)])
    assert e.value.status == _lib.CFD_EINVAL
    with pytest.raises(P.CfdError) as e:
        P.Plan([dict(n=(16, 16, 16), ng=4, h=(0.0, 0.1, 0.1), boundary=(0, 0, 0))], 1, [(s, 0)])
    assert e.value.status == _lib.CFD_EINVAL


def test_plan_second_derivative_operands_checked():
    """Host validation before any device call: a U scheme needs one field and the field of its
    sampled f''; an aux_field on any other scheme is refused; a W scheme's embedded (2)P1_M needs
    closure lines of 3 nodes and periodic lines as long as its stencil."""
    u = P.Scheme.named("(1)U2-")
    for ops in ([(u, 0)], [(u, 0, 0)], [(u, 0, 0, -1, -1, 3)], [(u, 0, -1, -1, -1, 1)],
                [(P.Scheme.named("(1)W2-"), 0, 0, -1, -1, 1)], [(P.Scheme.named("(1)Q1_3[1]"), 0, -1, -1, -1, 0)]):
        with pytest.raises(P.CfdError) as e:
            P.Plan([_blk()], 2, ops)
        assert e.value.status == _lib.CFD_EINVAL, ops
    w = P.Scheme.named("(1)W3+")
    with pytest.raises(P.CfdError) as e:
        P.Plan([_blk(n=(2, 16, 16), ng=5)], 1, [(w, 0)])
    assert e.value.status == _lib.CFD_ESHAPE
    with pytest.raises(P.CfdError) as e:
        P.Plan([_blk(n=(4, 16, 16), ng=0, boundary=(1, 1, 1))], 1, [(w, 0)])
    assert e.value.status == _lib.CFD_ESHAPE
    with pytest.raises(P.CfdError) as e:
        P.Plan([_blk(ng=4)], 1, [(w, 0)])
    assert e.value.status == _lib.CFD_EGHOST


def test_valid_plan_needs_a_device_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    s = P.Scheme.named("(1)Q1_3[1]")
    with pytest.raises(P.CfdError) as e:
        P.Plan([_blk()], 1, [(s, 0)])
    assert e.value.status == _lib.CFD_EDEVICE


def test_stage_kernels_validate_arguments():
    L = _lib.lib()
    assert L.cfd_axpby(0, -1, 1.0, None, 1.0, None, None) == _lib.CFD_EINVAL
    assert L.cfd_xpcy(7, 0, None, 1.0, None, None, None) == _lib.CFD_EINVAL
    assert L.cfd_axpby(0, 0, 1.0, None, 1.0, None, None) == _lib.CFD_OK   # empty is a no-op


def test_mixed_dense_plan_limits():
    """The dense mixed-precision path takes periodic lines of 32..256 nodes, multiples of 32."""
    s = P.Scheme.named("(1)Q1_3[1]")
    for n, bnd in [((64, 64, 64), (0, 0, 0)), ((40, 64, 64), (1, 1, 1)), ((288, 32, 32), (1, 1, 1))]:
        with pytest.raises(P.CfdError) as e:
            P.Plan([dict(n=n, ng=4, h=(0.1, 0.1, 0.1), boundary=bnd)], 1, [(s, 0)], dtype=P.CFD_MIXED_BF16)
        assert e.value.status == _lib.CFD_EUNSUPPORTED


def test_schedule_calls_validate_arguments():
    L = _lib.lib()
    flags = ctypes.c_int(-1)
    assert L.cfd_plan_get_flags(None, ctypes.byref(flags)) == _lib.CFD_EINVAL
    assert L.cfd_plan_set_schedule(None, 0, 0, 0, _lib.CFD_SCHED_CONCURRENT) == _lib.CFD_EINVAL
    assert L.cfd_plan_get_schedule(None, None, None, None, None, None, None, 0) == _lib.CFD_EINVAL


def test_create_rejects_biased_stencils():
    """The line kernels evaluate the interior RHS in centred form (Eq. sch_cent_om): a biased stencil
    that satisfies the Taylor conditions, e.g. the backward difference (-1, 1, 0) for d = 1, is refused
    rather than silently differentiated with its mirrored half."""
    with pytest.raises(P.CfdError) as e:
        P.Scheme.create(1, 1, [1.0], [-1.0, 1.0, 0.0])
    assert e.value.status == _lib.CFD_EUNSUPPORTED
    with pytest.raises(P.CfdError) as e:   # asymmetric implicit stencil
        P.Scheme.create(1, 2, [0.2, 1, 0.3], [-0.75, 0.0, 0.75], [[-0.5, 0.0, 0.5]])
    assert e.value.status in (_lib.CFD_EUNSUPPORTED, _lib.CFD_EINVAL)


def test_create_rejects_nonpositive_symbol():
    """alpha_1 = 0.6: the symbol 1 + 1.2 cos t vanishes inside [0, pi] (singular periodic system)."""
    a = 0.6
    with pytest.raises(P.CfdError) as e:
        P.Scheme.create(1, 2, [a, 1, a], [-(1 + 2 * a) / 2, 0.0, (1 + 2 * a) / 2], [[-0.5, 0.0, 0.5]])
    assert e.value.status == _lib.CFD_ESINGULAR
    # alpha_1 = 0.49 stays positive and is accepted
    a = 0.49
    P.Scheme.create(1, 2, [a, 1, a], [-(1 + 2 * a) / 2, 0.0, (1 + 2 * a) / 2], [[-0.5, 0.0, 0.5]])


def test_debug_alloc_hook_is_harmless_without_device():
    P.cfd_debug_fail_alloc(0)
    P.cfd_debug_fail_alloc(-1)


BIASED = ["(1)V1", "(1)V2", "(1)V3", "(1)V4", "(1)X1", "(1)X2", "(1)X3", "(1)W1", "(1)W2", "(1)W3",
          "(1)U1", "(1)U2", "(1)U3"]


@pytest.mark.parametrize("name", BIASED)
@pytest.mark.parametrize("suffix,bias", [("-", -1), ("+", 1), ("", 0), ("s", 2)])
def test_biased_registry_matches_oracle(name, suffix, bias):
    """Biased schemes: the library's binary128 construction (xi from the Taylor-residual
    series) and the oracle's exact one (xi from the complex error series) agree to round-off."""
    from oracle import biased as OB
    g = P.Scheme.named(name + suffix).get_biased()
    s, c = OB.named(name)
    assert g["bias"] == bias
    assert g["order"] == s.order
    assert abs(g["alpha"] - float(s.lhs.get(-1))) <= 2e-16
    a = np.array([float(s.rhs[0].get(m)) for m in range(-5, 6)])
    cc = np.array([float(c.rhs[0].get(m)) for m in range(-5, 7)])
    assert float(c.lhs.get(1)) == float(s.lhs.get(-1))
    assert np.max(np.abs(a - g["a"])) <= 4e-16 * np.max(np.abs(a))
    assert np.max(np.abs(cc - g["c"])) <= 8e-16 * np.max(np.abs(cc))
    sch = P.Scheme.named(name + suffix)
    assert sch.required_ghosts() == OB.required_ghosts(name)
    assert sch.required_ghosts(P.CFD_BOUNDARY_PERIODIC) == 0
    e = sch.get_embedded()
    if name[3] == "W":
        assert e["M"] == int(name[4:]) and e["alpha2"] == float(s.rhs[1].get(0))
    elif name[3] == "U":
        assert e["M"] == 0 and e["alpha2"] == float(s.rhs[1].get(0)) == -float(c.rhs[1].get(0))
    else:
        assert e == {"alpha2": 0.0, "M": 0}


def test_biased_design_ranges_and_lambda():
    from oracle import biased as OB
    from fractions import Fraction
    for fam, M in (("V", 0), ("V", 5), ("X", 0), ("X", 4), ("W", 0), ("W", 4), ("U", 0), ("U", 4), ("U", 5)):
        with pytest.raises(P.CfdError) as e:
            P.Scheme.design_biased(fam, M)
        assert e.value.status == _lib.CFD_EUNSUPPORTED
    with pytest.raises(P.CfdError) as e:
        P.Scheme.design_biased("Q", 2)
    assert e.value.status == _lib.CFD_EINVAL
    with pytest.raises(P.CfdError):
        P.Scheme.design_biased("X", 2, 0.5, 3)
    assert P.Scheme.design_biased("X", 2, 0.0, 2).get_biased()["bias"] == 2
    # a lambda other than the printed one: both constructions follow it
    g = P.Scheme.design_biased("X", 2, 0.5, -1).get_biased()
    s = OB.xscheme(2, Fraction(1, 2))
    xi, c = OB.xi_closure(s)
    assert abs(g["alpha"] - float(s.lhs.get(-1))) <= 2e-16
    a = np.array([float(s.rhs[0].get(m)) for m in range(-5, 6)])
    cc = np.array([float(c.rhs[0].get(m)) for m in range(-5, 7)])
    assert np.max(np.abs(a - g["a"])) <= 4e-16 * np.max(np.abs(a))
    assert np.max(np.abs(cc - g["c"])) <= 8e-16 * np.max(np.abs(cc))
    # W with another lambda: the library and the oracle's construction follow it
    g = P.Scheme.design_biased("W", 2, 0.5, 1).get_biased()
    s = OB.wscheme(2, Fraction(1, 2))
    _, c = OB.xi_closure(OB.with_explicit_second(s, OB.embedded_second(2).closure[0]))
    a = np.array([float(s.rhs[0].get(m)) for m in range(-5, 6)])
    cc = np.array([float(c.rhs[0].get(m)) for m in range(-5, 7)])
    assert g["bias"] == 1 and abs(g["alpha"] - float(s.lhs.get(-1))) <= 2e-16
    assert np.max(np.abs(a - g["a"])) <= 4e-16 * np.max(np.abs(a))
    assert np.max(np.abs(cc - g["c"])) <= 8e-16 * np.max(np.abs(cc))
    assert P.Scheme.design_biased("W", 2, 0.5, 1).get_embedded()["alpha2"] == float(s.rhs[1].get(0))
    with pytest.raises(P.CfdError) as e:
        P.Scheme.named("(1)Q1_3[1]").get_embedded()
    assert e.value.status == _lib.CFD_EINVAL
    with pytest.raises(P.CfdError):
        P.Scheme.named("(1)X2*")
    with pytest.raises(P.CfdError):
        P.Scheme.named("(2)X2")


@pytest.mark.parametrize("dr,L,R,classes", [
    (1, 0, 1, [(0, 1, 2), (2, 0, 0)]),        # the worked example of Sec. 2 (d_I = (0, 2))
    (1, 1, 0, [(0, 2, 2), (2, 0, 0)]),        # U_2 of Eq. defChenSchemes
    (1, 1, 1, [(0, 2, 2)]),                   # Pade (1)P1_2
    (2, 1, 1, [(0, 3, 3)]),                   # fully determined second-degree tridiagonal, M = 3
    (1, 2, 2, [(0, 2, 2)]),                   # classical pentadiagonal O(8) (Sec. 2)
])
def test_taylor_scheme_matches_oracle(dr, L, R, classes):
    g = P.cfd_taylor_scheme(dr, L, R, classes)
    lhs, rhs, q = OS.determined_scheme(dr, (L, R), classes)
    assert g["order"] == q
    assert np.max(np.abs(np.array([float(v) for v in lhs.coef]) - g["lhs"])) <= 4e-16
    for st, got in zip(rhs, g["rhs"]):
        ref = np.array([float(v) for v in st.coef])
        assert np.max(np.abs(ref - got)) <= 8e-16 * max(1.0, np.max(np.abs(ref)))


def test_taylor_scheme_rejects_bad_extents():
    with pytest.raises(P.CfdError) as e:
        P.cfd_taylor_scheme(1, 9, 9, [(0, 9, 9)])
    assert e.value.status == _lib.CFD_EINVAL


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5])
def test_dissipation_stencil_matches_oracle(r):
    """The library's Kreiss-Oliger stencil (binomial form) equals the oracle's repeated
    differences (Eq. dissdef) on a unit impulse, scaled by h^-1."""
    from oracle import dissipation as ODS
    sigma = 0.04 * r
    g = P.Scheme.dissipation(r, sigma).get()
    assert g["nl"] == 0 and g["m"] == r and g["d"] == 2 * r
    N = 2 * r + 1
    imp = np.zeros(N + 2 * r)
    imp[r + N // 2] = 1.0
    q = ODS.ko_line(imp, r, 1.0, r, sigma)
    ref = np.zeros(11)
    for m in range(-r, r + 1):
        ref[5 - m] = q[N // 2 + m]
    assert np.max(np.abs(ref - g["rhs"])) <= 1e-15 * max(1.0, np.max(np.abs(ref)))
    assert P.Scheme.dissipation(r, sigma).required_ghosts() == r


def test_dissipation_rejects_bad_arguments():
    for r, s in ((0, 0.1), (6, 0.1)):
        with pytest.raises(P.CfdError) as e:
            P.Scheme.dissipation(r, s)
        assert e.value.status == _lib.CFD_EUNSUPPORTED
    for s in (-0.1, float("nan"), float("inf")):
        with pytest.raises(P.CfdError) as e:
            P.Scheme.dissipation(4, s)
        assert e.value.status == _lib.CFD_EINVAL
