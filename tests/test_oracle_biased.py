"""Pins of the biased-scheme oracle (oracle/biased.py) against the paper.

Every printed tuple of Tabs. ucd_slow, ucd_fast, ucd_slow_closure,
ucd_fast_closure, ccux_deg_one_col and ccuw_deg_one_col is reproduced exactly (fixtures in
tests/golden/biased_tables.json, typed from the paper); the line operator is
pinned by polynomial exactness on every row, the closed form of Eq.
fdpwerrdef on periodic lines, the mirror symmetry between the two biases, the
dispersion preserved by the closures, and the grid-convergence order.
"""
import json
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from oracle import biased as B
from oracle import schemes as S

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "biased_tables.json")))


def _fr(v):
    return Fraction(v)


def _eps(s, n):
    return S.eps_series(s, n, exact=True)


@pytest.mark.parametrize("kind,table", [("U", "ucd_slow"), ("V", "ucd_fast")])
@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_ucd_tables_exact(kind, table, M):
    g = GOLD[table][str(M)]
    s = B.ucd(kind, M)
    assert s.order == g["order"]
    assert [s.lhs.get(n) for n in (-1, 0)] == [_fr(v) for v in g["a1"]]
    assert [s.rhs[0].get(n) for n in range(-M, M + 1)] == [_fr(v) for v in g["a0"]]
    if kind == "U":
        assert s.rhs[1].dK == 2 and s.rhs[1].get(0) == _fr(g["a2"])
    else:
        assert len(s.rhs) == 1
    ser = _eps(s, g["order"] + 2)
    for j in range(g["order"]):
        assert ser[j] == (0, 0), (j, ser[j])            # formal order: eps starts at eta^order
    for j, re, im in g["eps"]:
        assert ser[j] == (_fr(re), _fr(im)), (j, ser[j])


@pytest.mark.parametrize("kind,table", [("U", "ucd_slow_closure"), ("V", "ucd_fast_closure")])
@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_xi_tables_exact(kind, table, M):
    xi, _ = B.xi_closure(B.ucd(kind, M))
    assert xi == _fr(GOLD[table][str(M)])


@pytest.mark.parametrize("M", [1, 2, 3])
def test_ccux_table_exact(M):
    g = GOLD["ccux"][str(M)]
    assert B.X_LAMBDA[M] == _fr(g["sigma"])
    s = B.xscheme(M)
    assert s.order == 2 * M + 2
    assert [s.lhs.get(n) for n in (-1, 0)] == [_fr(v) for v in g["a1"]]
    W = M + 2
    assert (s.rhs[0].L, s.rhs[0].R) == (W, W)
    assert [s.rhs[0].get(n) for n in range(-W, W + 1)] == [_fr(v) for v in g["a0"]]
    ser = _eps(s, s.order + 2)
    for j in range(s.order):
        assert ser[j] == (0, 0)
    for j, re, im in g["eps"]:
        assert ser[j] == (_fr(re), _fr(im))
    _, c = B.xi_closure(s)
    assert [c.lhs.get(n) for n in (0, 1)] == [_fr(v) for v in g["closure_a1"]]
    assert (c.rhs[0].L, c.rhs[0].R) == (W, W + 1)
    assert [c.rhs[0].get(n) for n in range(-W, W + 2)] == [_fr(v) for v in g["closure_a0"]]


@pytest.mark.parametrize("M", [1, 2, 3])
def test_ccuw_table_exact(M):
    """Tab. ccuw_deg_one_col: W^-_M as the lambda = sigma combination with its f'' term; Wtilde^-_M
    as that row with f'' from the explicit closure of (2)P1_M; Wbar^-_M as the xi-closure of Wtilde;
    eps of the interior with the compact (2)P1_M second derivative."""
    g = GOLD["ccuw"][str(M)]
    assert B.W_LAMBDA[M] == _fr(g["sigma"])
    s, wb, wt = B.w_rows(M)
    assert s.order == 2 * M + 2
    assert [s.lhs.get(n) for n in (-1, 0)] == [_fr(v) for v in g["a1"]]
    W = M + 1
    assert (s.rhs[0].L, s.rhs[0].R) == (W, W)
    assert [s.rhs[0].get(n) for n in range(-W, W + 1)] == [_fr(v) for v in g["a0"]]
    assert s.rhs[1].dK == 2 and s.rhs[1].get(0) == _fr(g["a2"])
    assert [wt.lhs.get(n) for n in (-1, 0)] == [_fr(v) for v in g["tilde_a1"]]
    assert (wt.rhs[0].L, wt.rhs[0].R) == (M + 2, M + 2)
    assert [wt.rhs[0].get(n) for n in range(-(M + 2), M + 3)] == [_fr(v) for v in g["tilde_a0"]]
    assert [wb.lhs.get(n) for n in (0, 1)] == [_fr(v) for v in g["closure_a1"]]
    assert (wb.rhs[0].L, wb.rhs[0].R) == (M + 2, M + 3)
    assert [wb.rhs[0].get(n) for n in range(-(M + 2), M + 4)] == [_fr(v) for v in g["closure_a0"]]
    ser = B.w_eps_series(M, s.order + 2)
    for j in range(s.order):
        assert ser[j] == (0, 0)
    for j, re, im in g["eps"]:
        assert ser[j] == (_fr(re), _fr(im))


@pytest.mark.parametrize("M", [1, 2, 3])
@pytest.mark.parametrize("bias", [-1, 1])
def test_w_line_end_rows_are_the_printed_closures(M, bias):
    """The W line operator (interior rows with f'' from the (2)P1_M line solve) has, as the
    right side of its end rows, exactly the printed Wbar (closed end) and Wtilde (other end):
    A D = B row by row, A the bidiagonal left side."""
    g = GOLD["ccuw"][str(M)]
    name, N = f"(1)W{M}", 17
    ng = B.required_ghosts(name)
    D = B.line_matrix(name, bias, N, ng, False)
    al = float(_fr(g["a1"][0]))
    wbar = np.array([float(_fr(v)) for v in g["closure_a0"]])
    wtil = np.array([float(_fr(v)) for v in g["tilde_a0"]])
    if bias < 0:
        closed = D[0] + al * D[1]                 # x_0 + alpha x_1 = Wbar . f
        other = D[N - 1] + al * D[N - 2]          # alpha x_{N-2} + x_{N-1} = Wtilde . f
        ref_c = np.zeros(N + 2 * ng)
        ref_c[ng - (M + 2): ng + M + 4] = wbar
        ref_o = np.zeros(N + 2 * ng)
        ref_o[ng + N - 1 - (M + 2): ng + N + M + 2] = wtil
    else:                                         # mirror image: offsets reversed, signs flipped
        closed = D[N - 1] + al * D[N - 2]
        other = D[0] + al * D[1]
        ref_c = np.zeros(N + 2 * ng)
        ref_c[ng + N - 1 - (M + 3): ng + N + M + 2] = -wbar[::-1]
        ref_o = np.zeros(N + 2 * ng)
        ref_o[ng - (M + 2): ng + M + 3] = -wtil[::-1]
    assert np.max(np.abs(closed - ref_c)) < 1e-13
    assert np.max(np.abs(other - ref_o)) < 1e-13


def test_explicit_derivative_stencils_match_tab_diss_scheme():
    for q, row in GOLD["diss_scheme"].items():
        if q.startswith("_"):
            continue
        assert B.explicit_deriv(int(q)) == row


@pytest.mark.parametrize("name", ["(1)V1", "(1)V2", "(1)V3", "(1)V4", "(1)X1", "(1)X2", "(1)X3"])
def test_mirror_conjugates_eps_and_closure_keeps_dispersion(name):
    """Right bias = complex conjugate error (captions of Tabs. ucd_slow, ucd_fast,
    ucd_slow_closure); the closure keeps Re eta~ of the interior exactly (the
    correction only adds an imaginary part)."""
    s, c = B.named(name)
    n = s.order + 3
    a, b = _eps(s, n), _eps(B.mirror(s), n)
    assert all(x[0] == y[0] and x[1] == -y[1] for x, y in zip(a, b))
    with mp.workdps(40):
        for eta in np.linspace(0.05, 3.1, 23):
            wi = S.modified_wavenumber_power(s, eta) / 1j
            wc = S.modified_wavenumber_power(c, eta) / 1j
            assert abs(mp.re(wi) - mp.re(wc)) < mp.mpf(10) ** -30
    # closure and interior agree in eps up to (and including) the matched imaginary term
    q = B.correction_order(s.order)
    ec = _eps(c, q)
    assert ec[: q] == a[: q]


def _poly_line(deg, N, ng, h, x0=0.37):
    x = (np.arange(N + 2 * ng) - ng) * h + x0
    t = x / (N * h)                       # O(1)-scaled polynomial
    coef = np.arange(1, deg + 2) * 0.1 + 1
    f = sum(c * t ** j for j, c in enumerate(coef))
    df = sum((j * c * t ** (j - 1) for j, c in enumerate(coef) if j), np.zeros_like(t)) / (N * h)
    return f, df[ng:ng + N]


@pytest.mark.parametrize("name", ["(1)V2", "(1)V4", "(1)X1", "(1)X2", "(1)X3", "(1)W1", "(1)W2", "(1)W3"])
@pytest.mark.parametrize("bias", [-1, 1])
def test_polynomial_exactness_every_row(name, bias):
    s, _ = B.named(name)
    ng, N, h = B.required_ghosts(name), 19, 0.1
    D = B.line_matrix(name, bias, N, ng, False)
    worst = 0.0
    for deg in range(s.order + 1):
        f, df = _poly_line(deg, N, ng, h)
        rel = np.max(np.abs(D @ f / h - df)) / max(1.0, np.max(np.abs(df)))
        assert rel < 1e-11, deg
        worst = max(worst, rel)
    f, df = _poly_line(s.order + 1, N, ng, h)
    rel = np.max(np.abs(D @ f / h - df)) / np.max(np.abs(df))
    assert rel > 100 * max(worst, 1e-15)                      # order is not higher than stated


@pytest.mark.parametrize("name", ["(1)V3", "(1)X1", "(1)X2", "(1)X3", "(1)W1", "(1)W3"])
@pytest.mark.parametrize("bias", [-1, 1])
def test_periodic_closed_form(name, bias):
    """On a periodic line a Fourier mode is an eigenvector with eigenvalue
    i eta~(eta)/h (Eq. fdpwerrdef): D sin(theta) = (Re eta~ cos theta - Im eta~ sin theta)/h.
    For W, eta~ is that of the interior row with the compact (2)P1_M second derivative."""
    s, _ = B.named(name)
    if name[3] == "W":
        s = B.w_compact_scheme(int(name[4:]))
    if bias > 0:
        s = B.mirror(s)
    N = 48
    h = 2 * np.pi / N
    x = np.arange(N) * h
    for k, ph in ((1, 0.3), (5, 1.1), (11, 2.0), (20, 0.7)):
        th = k * x + ph
        g = np.concatenate([np.zeros(0), np.sin(th)])
        D = B.line_matrix(name, bias, N, 0, True)
        got = D @ g / h
        with mp.workdps(30):
            et = complex(S.modified_wavenumber_power(s, k * h) / 1j)
        ref = (et.real * np.cos(th) - et.imag * np.sin(th)) / h
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref)), k


@pytest.mark.parametrize("name", ["(1)V2", "(1)X2", "(1)W2"])
@pytest.mark.parametrize("periodic", [False, True])
def test_biases_are_mirror_images(name, periodic):
    """D+[f](x_k) = -D-[f reversed](x_{N-1-k}): the right-biased operator is the
    reflection of the left-biased one, closure rows included."""
    ng, N, h = B.required_ghosts(name), 23, 0.05
    rng = np.random.default_rng(7)
    g = rng.standard_normal(N + 2 * ng)
    Dl = B.line_matrix(name, -1, N, ng, periodic)
    Dr = B.line_matrix(name, +1, N, ng, periodic)
    assert np.max(np.abs(Dr @ g + (Dl @ g[::-1])[::-1])) < 1e-12


@pytest.mark.parametrize("name,order", [("(1)V2", 5), ("(1)X1", 4), ("(1)X2", 6), ("(1)W1", 4), ("(1)W2", 6)])
def test_convergence_order_closure_lines(name, order):
    errs = []
    Ns = [32, 64, 128]
    ng = B.required_ghosts(name)
    for N in Ns:
        h = 1.0 / N
        x = (np.arange(N + 2 * ng) - ng + 0.5) * h
        f = np.exp(np.sin(2 * np.pi * x) + 0.5 * x)
        df = (2 * np.pi * np.cos(2 * np.pi * x) + 0.5) * f
        e = 0.0
        for bias in (-1, 1):
            D = B.line_matrix(name, bias, N, ng, False)
            e = max(e, np.max(np.abs(D @ f / h - df[ng:ng + N])))
        errs.append(e)
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert slopes[-1] > order - 0.6, slopes


def test_upwind_selects_by_sign():
    """c > 0 everywhere gives c times the left-biased derivative, c < 0 the
    right-biased one; a mixed-sign c picks per node (Eq. biasderapproxadv)."""
    name, ng = "(1)X2", 4
    rng = np.random.default_rng(3)
    n = (9, 7, 6)
    f = rng.standard_normal(tuple(e + 2 * ng for e in n[::-1]))
    for d in range(3):
        dl = B.apply_block(name, -1, f, ng, 0.1, d)
        dr = B.apply_block(name, +1, f, ng, 0.1, d)
        cpos = rng.uniform(0.5, 2.0, dl.shape)
        assert np.allclose(B.upwind_block(name, f, cpos, ng, 0.1, d), cpos * dl, rtol=0, atol=1e-13)
        assert np.allclose(B.upwind_block(name, f, -cpos, ng, 0.1, d), -cpos * dr, rtol=0, atol=1e-13)
        assert np.all(B.upwind_block(name, f, np.zeros_like(cpos), ng, 0.1, d) == 0)
        mix = cpos * np.where(rng.random(dl.shape) < 0.5, -1, 1)
        got = B.upwind_block(name, f, mix, ng, 0.1, d)
        assert np.allclose(got, np.where(mix > 0, mix * dl, mix * dr), rtol=0, atol=1e-13)


def test_block_directions_match_lines():
    name, ng = "(1)X1", 3
    rng = np.random.default_rng(5)
    n = (10, 8, 7)
    f = rng.standard_normal(tuple(e + 2 * ng for e in n[::-1]))
    for d in range(3):
        out = B.apply_block(name, -1, f, ng, 0.2, d)
        D = B.line_matrix(name, -1, n[d], ng, False)
        z, y, x = 2, 3, 4
        idx = [z + ng, y + ng, x + ng]
        idx[2 - d] = slice(None)
        line = f[tuple(idx)]
        ref = D @ line / 0.2
        oi = [z, y, x]
        oi[2 - d] = slice(None)
        assert np.allclose(out[tuple(oi)], ref, rtol=0, atol=1e-12)


def test_ghost_requirement_rule():
    """N_g >= M + 2 for X_M (after Eq. closure_left_X); V_M needs M + 1 (its
    closure correction reaches one node further than its interior)."""
    for M in (1, 2, 3):
        assert B.required_ghosts(f"(1)X{M}") == M + 2
    for M in (1, 2, 3, 4):
        assert B.required_ghosts(f"(1)V{M}") == M + 1
    for M in (1, 2, 3):                 # W_M: its closure and the embedded (2)P1_M closure
        assert B.required_ghosts(f"(1)W{M}") == M + 2
    with pytest.raises(ValueError):
        B.line_matrix("(1)X2", -1, 12, 3, False)


@pytest.mark.parametrize("name", ["(1)V2", "(1)X2", "(1)X3"])
def test_symmetrised_is_non_dissipative_on_periodic_lines(name):
    """The mean of both biases (the symmetrisation of the decomposition study) keeps only the real
    part of the modified wavenumber: D sin(theta) = Re eta~ cos(theta) / h, with no sin component (the
    right bias's Im eta~ is the left one's, negated)."""
    s, _ = B.named(name)
    N, ng = 40, 0
    h = 2 * np.pi / N
    x = np.arange(N) * h
    for k, ph in ((1, 0.2), (7, 1.3), (15, 0.4)):
        th = k * x + ph
        f = np.broadcast_to(np.sin(th)[None, None, :], (2, 3, N)).copy()
        got = B.symmetrised_block(name, f, ng, h, 0, periodic=True)
        with mp.workdps(30):
            et = complex(S.modified_wavenumber_power(s, k * h) / 1j)
        ref = et.real * np.cos(th) / h
        assert np.max(np.abs(got - ref[None, None, :])) < 1e-12 * np.max(np.abs(ref)), k
        assert abs(et.imag) > 1e-6 or k == 1   # the biases themselves dissipate


@pytest.mark.parametrize("name", ["(1)V2", "(1)X1", "(1)X2"])
@pytest.mark.parametrize("bias", [-1, 1])
def test_iterated_biased_closure_converges_to_the_global_scheme(name, bias):
    """Eq. iter_left_X (and its mirror): passing one end value per iteration across a periodic tiling
    converges to the global periodic biased operator, the error shrinking by about |alpha|^N_B per
    iteration (the end value's influence decays as (-alpha)^k along the sub-domain)."""
    ng, NB, NS = B.iterated_ghosts(name), 12, 6
    NM = NB * NS
    h = 2 * np.pi / NM
    x = (np.arange(NM) + 0.5) * h
    f = np.sin(3 * x + 0.4) + 0.3 * np.cos(7 * x)
    blocks = np.stack([f[(np.arange(-ng, NB + ng) + I * NB) % NM] for I in range(NS)])
    its = B.iterate_1d(name, bias, blocks, ng, h, 8)
    glob = B.line_matrix(name, bias, NM, 0, True) @ f / h
    err = [np.max(np.abs(it.reshape(-1) - glob)) for it in its]
    s, _ = B.named(name)
    rate = abs(float(s.lhs.get(-1))) ** NB
    for i in range(1, 8):
        assert err[i + 1] <= 2.0 * rate * err[i] + 1e-13 * np.max(np.abs(glob)), (i, err)
    assert err[8] < 1e-12 * np.max(np.abs(glob))
    assert err[1] < 1e-2 * err[0]


def test_biased_iteration_converges_faster_than_centred():
    """The decomposition study's remark: under iteration the biased schemes converge more rapidly
    than the centred ones (here X_2^- against P_2^1 on the paper's g, N_M = 128, N_B = 16)."""
    import synth
    from oracle import iterate as IT
    from oracle import lines as OL
    from oracle import schemes as OS
    NM, NB = 128, 16
    h = 2 * np.pi / NM
    xg = (np.arange(NM) + 0.5) * h
    g = synth.paper_g(xg)
    ng = 4
    blocks = np.stack([synth.paper_g((I * NB + np.arange(-ng, NB + ng) + 0.5) * h) for I in range(NM // NB)])
    gb = B.line_matrix("(1)X2", -1, NM, 0, True) @ g / h
    eb = [IT.modal_rms_error(gb, it.reshape(-1))[0] for it in B.iterate_1d("(1)X2", -1, blocks, ng, h, 2)]
    sc = OS.named("(1)P1_2")
    gc = OL.apply_line(sc, g, 0, h, periodic=True)
    ec = [IT.modal_rms_error(gc, it.reshape(-1))[0] for it in IT.iterate_1d(sc, blocks, ng, h, 2)]
    assert eb[1] / eb[0] < 0.1 * (ec[1] / ec[0]), (eb, ec)


@pytest.mark.parametrize("M", [1, 2, 3])
@pytest.mark.parametrize("bias", [-1, 1])
def test_u_line_operator_with_sampled_second_derivative(M, bias):
    """U_M as a line operator on (f, f''): exact on polynomials up to its formal order 2M+2 on every
    row, closure row included (its f'' term is the mirror's, -alpha^(2)_0), and not beyond; the
    closure row's f'' weight is the interior's negated."""
    name = f"(1)U{M}"
    s, c = B.named(name)
    assert c.rhs[1].dK == 2 and c.rhs[1].get(0) == -s.rhs[1].get(0)
    ng, N, h = B.required_ghosts(name), 19, 0.1
    D, D2 = B.line_matrices(name, bias, N, ng, False)
    x = (np.arange(N + 2 * ng) - ng) * h + 0.37
    worst = 0.0
    for deg in range(s.order + 2):
        t = x / (N * h)
        coef = np.arange(1, deg + 2) * 0.1 + 1
        f = sum(cf * t ** j for j, cf in enumerate(coef))
        df = sum((j * cf * t ** (j - 1) for j, cf in enumerate(coef) if j), np.zeros_like(t)) / (N * h)
        d2f = sum((j * (j - 1) * cf * t ** (j - 2) for j, cf in enumerate(coef) if j > 1), np.zeros_like(t)) / (N * h) ** 2
        got = D @ f / h + h * (D2 @ d2f[ng:ng + N])
        rel = np.max(np.abs(got - df[ng:ng + N])) / max(1.0, np.max(np.abs(df)))
        if deg <= s.order:
            assert rel < 1e-11, deg
            worst = max(worst, rel)
        else:                                                 # order is not higher than stated
            assert rel > 10 * max(worst, 1e-15)
    with pytest.raises(ValueError):
        B.line_matrix(name, bias, N, ng, False)


@pytest.mark.parametrize("M", [1, 3])
@pytest.mark.parametrize("bias", [-1, 1])
def test_u_periodic_closed_form(M, bias):
    """On a periodic line, with f'' sampled exactly, a Fourier mode is an eigenvector with the
    eigenvalue of U_M's symbol (Eq. fdpwerrdef with the f'' class)."""
    name = f"(1)U{M}"
    s, _ = B.named(name)
    if bias > 0:
        s = B.mirror(s)
    N = 48
    h = 2 * np.pi / N
    x = np.arange(N) * h
    D, D2 = B.line_matrices(name, bias, N, 0, True)
    for k, ph in ((1, 0.3), (7, 1.1), (19, 2.0)):
        th = k * x + ph
        got = D @ np.sin(th) / h + h * (D2 @ (-k * k * np.sin(th)))
        with mp.workdps(30):
            et = complex(S.modified_wavenumber_power(s, k * h) / 1j)
        ref = (et.real * np.cos(th) - et.imag * np.sin(th)) / h
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref)), k
