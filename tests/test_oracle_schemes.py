"""Pins of the oracle's scheme construction against what the paper prints.

Every expected value comes from tests/golden/paper_tables.json (typed from
the paper's tables) or from a closed form; none comes from the GPU library.
"""
import json
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from oracle import schemes as S

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def F(s):
    return Fraction(s)


def test_worked_example_exact():
    """Sec. 2 worked example: d_r = 1 with d_I = (0, 2) is fully determined and O(dx^5)."""
    g = GOLD["worked_example"]
    lhs, rhs, q = S.determined_scheme(1, (0, 1), [(0, 1, 2), (2, 0, 0)])
    assert lhs.coef == [F(v) for v in g["alpha1"]]
    assert rhs[0].coef == [F(v) for v in g["alpha0"]]
    assert rhs[1].coef == [F(g["alpha2_0"])]
    assert q == g["order"]


@pytest.mark.parametrize("name", list(k for k in GOLD["pade"] if k != "cite"))
def test_pade_tables_exact(name):
    g = GOLD["pade"][name]
    s = S.named(name)
    assert s.lhs.coef == [F(v) for v in g["lhs"]]
    assert s.rhs[0].coef == [F(v) for v in g["rhs"]]
    ser = S.eps_series(s, max(int(k) for k in g["eps"]) + 1, exact=True)
    for power, val in g["eps"].items():
        assert ser[int(power)] == (F(val), 0)
    # no lower powers
    for j in range(int(min(g["eps"], key=int))):
        assert ser[j] == (0, 0)


@pytest.mark.parametrize("name", list(k for k in GOLD["pade_closures"] if k != "cite"))
def test_matched_closures_exact(name):
    """The closure rule of Sec. 2.4 regenerates the printed matched closures."""
    g = GOLD["pade_closures"][name]
    s = S.named(name)
    assert s.closure[0].coef == [F(v) for v in g["closure"]]
    cl = S.Scheme("cl", s.dr, s.order, S.Stencil(s.dr, 0, 0, [Fraction(1)]), [s.closure[0]])
    ser = S.eps_series(cl, max(int(k) for k in g["eps"]) + 1, exact=True)
    for power, val in g["eps"].items():
        assert ser[int(power)] == (F(val), 0)


@pytest.mark.parametrize("name", list(k for k in GOLD["explicit"] if k != "cite"))
def test_explicit_tables_exact(name):
    g = GOLD["explicit"][name]
    s = S.named(name)
    assert s.rhs[0].coef == [F(v) for v in g["rhs"]]
    ser = S.eps_series(s, max(int(k) for k in g["eps"]) + 1, exact=True)
    for power, val in g["eps"].items():
        assert ser[int(power)] == (F(val), 0)


def _close_to_printed(value, printed: str):
    """Equal to the printed number within half a unit of its last printed digit."""
    p = printed.lstrip("-")
    mant = p.split("e")[0]
    digits = len(mant.replace(".", "").lstrip("0"))
    ref = float(printed)
    if ref == 0:
        return abs(value) < 1e-12
    ulp = 10 ** (np.floor(np.log10(abs(ref))) - digits + 1)
    return abs(float(value) - ref) <= 0.5 * ulp * 1.0000001


@pytest.mark.parametrize("name", list(k for k in GOLD["tuned"] if k != "cite"))
def test_tuned_tables_to_printed_digits(name):
    """Spectral tuning (Eqs. optfunc, gammacut) regenerates Tabs. num_deg_one/two."""
    g = GOLD["tuned"][name]
    s = S.named(name)
    assert _close_to_printed(s.lhs.get(1), g["lhs1"])
    assert _close_to_printed(s.lhs.get(-1), g["lhs1"])
    for m, v in enumerate(g["rhs_pos"]):
        assert _close_to_printed(s.rhs[0].get(m), v), (m, s.rhs[0].get(m), v)
    for m, v in enumerate(g["closure_pos"]):
        assert _close_to_printed(s.closure[0].get(m), v), (m, s.closure[0].get(m), v)
    ser = S.eps_series(s, 7)
    assert _close_to_printed(ser[6][0], g["eps6"])


@pytest.mark.parametrize("name", ["(1)Q1_3[1]", "(2)Q1_3[1]", "(1)QP_O8[1]", "(2)QP_O8[1]"])
def test_tuned_scheme_is_constrained_minimum(name):
    """Brute force: moving along the Taylor null space raises the objective of Eq. optfunc."""
    s = S.named(name)
    eta_c = 1
    with mp.workdps(30):
        def eps_of(delta):
            t = S.Scheme("t", s.dr, s.order, S.Stencil(s.dr, s.lhs.L, s.lhs.R, list(s.lhs.coef)),
                         [S.Stencil(0, s.rhs[0].L, s.rhs[0].R, list(s.rhs[0].coef))])
            # null-space direction: perturb alpha_1 symmetrically and re-solve the Taylor rows for the RHS
            nl, M = s.nl, s.M
            t.lhs.coef[nl + 1] += delta
            t.lhs.coef[nl - 1] += delta
            layout = [("I", 0, n) for n in range(-M, M + 1)]
            rows, b = [], []
            for l in range(s.order + s.dr):
                rows.append([S._mpf(v) for v in S.taylor_row(layout, l)])
                b.append(sum(S._mpf(t.lhs.get(j)) * (S._mpf(j) ** (l - s.dr) if l - s.dr > 0 else (1 if l == s.dr else 0))
                             / mp.factorial(l - s.dr) if l >= s.dr else 0 for j in range(-nl, nl + 1)))
            x, _ = mp.qr_solve(mp.matrix(rows), mp.matrix(b))
            t.rhs[0].coef = [x[i] for i in range(2 * M + 1)]
            return mp.quad(lambda e: abs(S.spectral_error(t, e)) ** 2, [0, eta_c])
        e0 = eps_of(0)
        for d in (1e-3, -1e-3, 1e-2, -1e-2):
            assert eps_of(d) > e0


def _rational_null_space(rows):
    """Basis of the null space of a rational matrix (list of rows of Fractions), by exact RREF."""
    A = [list(r) for r in rows]
    n = len(A[0])
    piv_cols, r = [], 0
    for c in range(n):
        p = next((i for i in range(r, len(A)) if A[i][c] != 0), None)
        if p is None:
            continue
        A[r], A[p] = A[p], A[r]
        pv = A[r][c]
        A[r] = [v / pv for v in A[r]]
        for i in range(len(A)):
            if i != r and A[i][c] != 0:
                f = A[i][c]
                A[i] = [a - f * b for a, b in zip(A[i], A[r])]
        piv_cols.append(c)
        r += 1
        if r == len(A):
            break
    free = [c for c in range(n) if c not in piv_cols]
    basis = []
    for fcol in free:
        z = [F(0)] * n
        z[fcol] = F(1)
        for i, pc in enumerate(piv_cols):
            z[pc] = -A[i][fcol]
        basis.append(z)
    return basis


@pytest.mark.parametrize("name", ["(1)Q1_3[1]", "(2)Q1_3[1]", "(1)QP_O8[1]", "(2)QP_O8[1]",
                                  "(1)Q1_3[4pi/5]"])
def test_tuned_scheme_is_minimum_along_every_null_direction(name):
    """Eq. optfunc at the tuned scheme against every direction that keeps the constraints (the
    normalisation and the Taylor rows of Eq. Tcons, no symmetry imposed): the exact rational null
    space of the constraint rows, each basis vector and two mixed directions.  Along each the
    objective has zero slope and positive curvature, so every perturbation raises it."""
    s = S.named(name)
    eta_c = mp.mpf(1) if name.endswith("[1]") else 4 * mp.pi / 5
    nl, M = s.nl, s.M
    layout = S._unknown_layout((s.dr, nl, nl), [(0, M, M)])
    rows = [S._normalisation_row(layout, s.dr)] + [S.taylor_row(layout, l) for l in range(s.order + s.dr)]
    Z = _rational_null_space(rows)
    # the constraint rows are independent: the free directions are what they leave over
    assert len(Z) == len(layout) - len(rows) >= 1
    # each constraint holds exactly along each direction
    for z in Z:
        for r in rows:
            assert sum(a * b for a, b in zip(r, z)) == 0
    dirs = list(Z)
    if len(Z) >= 2:
        dirs.append([a + b for a, b in zip(Z[0], Z[1])])
        dirs.append([a - 2 * b for a, b in zip(Z[0], Z[1])])
    with mp.workdps(30):
        c0 = [S._mpf(v) for v in s.lhs.coef] + [S._mpf(v) for v in s.rhs[0].coef]

        def J(c):
            lhs, rhs = S._unpack(layout, c, (s.dr, nl, nl), [(0, M, M)])
            t = S.Scheme("t", s.dr, s.order, lhs, rhs)
            return mp.quad(lambda e: abs(S.spectral_error(t, e)) ** 2, [0, eta_c])

        j0 = J(c0)
        for z in dirs:
            zn = [S._mpf(v) for v in z]
            scale = mp.sqrt(mp.fsum(v * v for v in zn))
            zn = [v / scale for v in zn]
            for delta in (mp.mpf("1e-3"), mp.mpf("1e-2")):
                jp = J([a + delta * b for a, b in zip(c0, zn)])
                jm = J([a - delta * b for a, b in zip(c0, zn)])
                curv = jp + jm - 2 * j0
                assert jp > j0 and jm > j0
                assert curv > 0
                assert abs(jp - jm) < 1e-12 * curv, (name, float(jp - jm), float(curv))


@pytest.mark.parametrize("name,need", [("(1)P1_1", 3), ("(2)P1_2", 4), ("(1)P1_3", 5), ("(1)Q1_3[1]", 4),
                                       ("(2)Q1_3[4pi/5]", 4), ("(1)QP_O8[1]", 5), ("(2)QP_O8[1]", 5),
                                       ("(1)Q1_3[1]:E", 3), ("(2)QP_O8[1]:E", 4), ("(1)E3", 3), ("(2)E4", 4)])
def test_required_ghosts_follow_the_closure_rule(name, need):
    """Ghost layers from the reach of the closure rows (Sec. 2.4, Eq. sch_cent_om): a matched closure
    of a scheme of formal order 2p has half-width p + 1, so N_g >= p + 1; the order-only closure has
    half-width p (N_g >= p); an explicit E_M reaches M.  Periodic lines need none."""
    s = S.named(name)
    p = s.order // 2
    if s.nl == 0:
        rule = s.M
    elif name.endswith(":E"):
        rule = p
    else:
        rule = p + 1
    assert rule == need
    assert S.required_ghosts(s, False) == need
    assert S.required_ghosts(s, True) == 0


def test_phi_estimate_table():
    """Tab. phi_estimate from Eq. adv_ppw_estimate with the oracle's error constants."""
    g = GOLD["phi_estimate"]
    NT = g["N_T"]
    for name, row in g["rows"].items():
        s = S.named(name)
        C6 = abs(float(S.eps_series(s, 7)[6][0]))
        if "/" in row["C6"]:
            assert abs(C6 - float(F(row["C6"]))) < 1e-15
        else:
            assert _close_to_printed(C6, row["C6"])
        for eps_phi, expect in zip(g["eps_phi"], row["N_nu"]):
            nu = 2 * np.pi * (2 * np.pi * NT * C6 / eps_phi) ** (1.0 / 6)
            assert int(np.ceil(nu)) == expect


@pytest.mark.parametrize("name", ["(1)P1_2", "(1)Q1_3[1]", "(2)Q1_3[1]", "(1)QP_O8[1]", "(2)QP_O8[1]"])
def test_modified_wavenumber_series_matches_direct(name):
    """The eps series (Eq. relmodnormwavnum) agrees with Eq. fdpwerrdef evaluated directly."""
    s = S.named(name)
    with mp.workdps(40):
        ser = S.eps_series(s, s.order + 12)
        eta = mp.mpf("0.05")
        direct = S.modified_wavenumber_power(s, eta) / (1j * eta) ** s.dr - 1
        approx = sum(ser[j][0] * eta ** j for j in range(len(ser)))
        assert abs(direct - approx) < 1e-25


@pytest.mark.parametrize("name", ["(1)QP_O8[1]", "(2)QP_O8[1]"])
def test_penta_interior_symbol_positive(name):
    """The pentadiagonal D_L symbol 1 + 2a1 cos t + 2a2 cos 2t stays positive (no-pivot LU is safe)."""
    s = S.named(name)
    a1, a2 = float(s.lhs.get(1)), float(s.lhs.get(2))
    t = np.linspace(0, np.pi, 2001)
    assert np.min(1 + 2 * a1 * np.cos(t) + 2 * a2 * np.cos(2 * t)) > 0.05
