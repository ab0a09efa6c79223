"""Pins of the oracle's FP64 line operator (block closure and periodic).

Checked against what the mathematics fixes: the modified wavenumber on
Fourier modes (Eq. fdpwerrdef), exactness on polynomials up to the formal
order (Eq. Tcons), a dense assembly of Eqs. diff_mat_subL/R solved with
partial pivoting, the embedded operator of Eq. iter_scheme (i = 0) on a
periodic tiling, the grid-convergence order, and the decay of the closure's
influence into the block interior.
"""
import numpy as np
import pytest

import mpmath as mp

from oracle import lines as L
from oracle import schemes as S

SCHEMES = ["(1)P1_2", "(2)P1_2", "(1)Q1_3[1]", "(2)Q1_3[1]", "(1)QP_O8[1]", "(2)QP_O8[1]", "(1)Q1_3[1]:E",
           "(1)E3"]


def eta_tilde_power(s, eta):
    return complex(S.modified_wavenumber_power(s, eta))


@pytest.mark.parametrize("name", SCHEMES)
@pytest.mark.parametrize("N", [16, 48])
def test_periodic_closed_form(name, N):
    s = S.named(name)
    h = 2 * np.pi / N
    x = np.arange(N) * h
    for k in (1, 3, N // 3):
        phi = 0.3 * k
        y = L.apply_line(s, np.sin(k * x + phi), 0, h, periodic=True)
        lam = eta_tilde_power(s, k * h)     # (i eta~)^d
        if s.dr == 1:
            expect = (lam.imag / h) * np.cos(k * x + phi)
        else:
            expect = (lam.real / h ** 2) * np.sin(k * x + phi)
        assert np.max(np.abs(y - expect)) <= 1e-12 * max(1.0, np.max(np.abs(expect)))


@pytest.mark.parametrize("name", SCHEMES)
def test_polynomial_exactness_closure_block(name):
    """Every row (closure and interior) is exact up to degree order + d - 1."""
    s = S.named(name)
    ng = S.required_ghosts(s, False)
    N, h = 21, 0.37
    x = (np.arange(-ng, N + ng) + 0.5) * h - 2.0   # cell-centred, not symmetric about 0
    top = s.order + s.dr - 1
    for deg in range(top + 1):
        f = ((x - 0.1) / 3) ** deg
        y = L.apply_line(s, f, ng, h)
        xi = x[ng:ng + N]
        if deg < s.dr:
            ex = np.zeros(N)
        else:
            c = np.prod([deg - i for i in range(s.dr)])
            ex = c * ((xi - 0.1) / 3) ** (deg - s.dr) / 3 ** s.dr
        assert np.max(np.abs(y - ex)) <= 1e-10 * max(1.0, np.max(np.abs(ex))), deg
    f = ((x - 0.1) / 3) ** (top + 1)
    y = L.apply_line(s, f, ng, h)
    c = np.prod([top + 1 - i for i in range(s.dr)])
    ex = c * ((x[ng:ng + N] - 0.1) / 3) ** (top + 1 - s.dr) / 3 ** s.dr
    assert np.max(np.abs(y - ex)) > 1e-9   # and not beyond: the order is exactly what is claimed


def dense_block_operator(s, N, ng, h):
    """h^-d D_L^-1 D_R restricted to the interior rows (Eqs. diff_mat_subL/R)."""
    W = N + 2 * ng
    DL = np.eye(W)
    DR = np.zeros((W, W))
    nl = s.nl
    nc = len(s.closure) if nl > 0 else 0
    mc, crow = s.closure_floats()
    a = s.rhs_floats()
    al = s.lhs_floats()
    sgn = (-1) ** s.dr
    for k in range(N):
        r = ng + k
        if k < nc:
            DR[r, r - mc:r + mc + 1] = crow[k]
        elif k >= N - nc:
            DR[r, r - mc:r + mc + 1] = [sgn * v for v in crow[N - 1 - k][::-1]]
        else:
            DR[r, r - s.M:r + s.M + 1] = a
            DL[r, r - nl:r + nl + 1] = al
    for r in list(range(ng)) + list(range(ng + N, W)):
        DR[r, r] = 1.0          # ghost rows: identity (they are not outputs)
    D = np.linalg.solve(DL, DR) / h ** s.dr
    return D[ng:ng + N, :]


@pytest.mark.parametrize("name", SCHEMES)
@pytest.mark.parametrize("N", [12, 29])
def test_dense_assembly(name, N):
    s = S.named(name)
    ng = S.required_ghosts(s, False) + 1
    h = 0.05
    rng = np.random.default_rng(11)
    g = rng.standard_normal(N + 2 * ng)
    D = dense_block_operator(s, N, ng, h)
    y = L.apply_line(s, g, ng, h)
    ref = D @ g
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_embedded_operator_periodic_tiling():
    """[0]D = G diag(D) G on a periodic 1D tiling (Eqs. example_G, iter_scheme with i = 0)."""
    s = S.named("(1)Q1_3[1]")
    NM, NB = 32, 8
    ng = S.required_ghosts(s, False)
    NS = NM // NB
    W = NB + 2 * ng
    h = 2 * np.pi / NM
    G = np.zeros((NS * W, NS * W))
    for I in range(NS):
        for k in range(W):
            r = I * W + k
            loc = k - ng           # node index local to the sub-domain
            if 0 <= loc < NB:
                G[r, r] = 1.0
            elif loc < 0:
                J = (I - 1) % NS
                G[r, J * W + ng + NB + loc] = 1.0
            else:
                J = (I + 1) % NS
                G[r, J * W + ng + loc - NB] = 1.0
    Dsub = np.zeros((W, W))
    Dsub[ng:ng + NB, :] = dense_block_operator(s, NB, ng, h)
    Dbig = G @ np.kron(np.eye(NS), Dsub) @ G
    xg = (np.arange(NM) + 0.5) * h
    fglob = np.exp(np.sin(2 * xg)) * 0.05
    F = np.zeros(NS * W)
    for I in range(NS):
        F[I * W + ng:I * W + ng + NB] = fglob[I * NB:(I + 1) * NB]
    ref = Dbig @ F
    # oracle: fill ghosts from the neighbours, then one block solve per sub-domain
    out = np.zeros(NS * W)
    for I in range(NS):
        idx = (np.arange(-ng, NB + ng) + I * NB) % NM
        out[I * W + ng:I * W + ng + NB] = L.apply_line(s, fglob[idx], ng, h)
    for I in range(NS):
        sl = slice(I * W + ng, I * W + ng + NB)
        assert np.max(np.abs(out[sl] - ref[sl])) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("name,slope", [("(1)Q1_3[1]", 6), ("(2)Q1_3[1]", 6), ("(1)QP_O8[1]", 8),
                                        ("(2)QP_O8[1]", 8)])
def test_convergence_order_closure_block(name, slope):
    """Error against the exact derivative of g (Eq. test_grid_conv_g) converges at the formal order."""
    s = S.named(name)
    ng = S.required_ghosts(s, False)
    A, Sg, N1, x0 = 0.05, 1.0, 2, 0.2

    def g(x, d):
        u = -Sg * np.sin(N1 * (x - x0))
        e = A * np.exp(u)
        if d == 0:
            return e
        du = -Sg * N1 * np.cos(N1 * (x - x0))
        if d == 1:
            return e * du
        d2u = Sg * N1 ** 2 * np.sin(N1 * (x - x0))
        return e * (du ** 2 + d2u)

    errs = []
    Ns = [8, 16, 32]          # before round-off sets in for the 8th-order schemes
    for N in Ns:
        h = 1.0 / N           # block [0, 1], cell-centred
        x = (np.arange(-ng, N + ng) + 0.5) * h
        y = L.apply_line(s, g(x, 0), ng, h)
        errs.append(np.max(np.abs(y - g(x[ng:ng + N], s.dr))))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) > slope - 0.7, rates


def test_closure_influence_decays_into_interior():
    """Block result minus global periodic result decays geometrically away from the block ends."""
    s = S.named("(1)Q1_3[1]")
    ng = S.required_ghosts(s, False)
    NM = 128
    h = 2 * np.pi / NM
    x = np.arange(NM) * h
    f = np.sin(3 * x) + 0.3 * np.cos(7 * x + 1)
    glob = L.apply_line(s, f, 0, h, periodic=True)
    NB = 64
    idx = np.arange(-ng, NB + ng) % NM
    blk = L.apply_line(s, f[idx], ng, h)
    d = np.abs(blk - glob[:NB])
    assert d[NB // 2] < 1e-6 * d[1]
    alpha = float(s.lhs.get(1))
    rho = abs((-1 + np.sqrt(1 - 4 * alpha ** 2)) / (2 * alpha))
    # decay rate between rows 4 and 16 close to the stable root of the symbol
    rate = (d[16] / d[4]) ** (1 / 12)
    assert abs(rate - rho) < 0.05


@pytest.mark.parametrize("name", ["(1)Q1_3[1]", "(2)QP_O8[1]"])
def test_block_apply_matches_lines_each_direction(name):
    """The 3D driver gathers every line of the requested direction (checked by a polynomial in that axis)."""
    s = S.named(name)
    ng = S.required_ghosts(s, False)
    n = (9, 11, 13)
    h = 0.1
    coords = [(np.arange(-ng, n[a] + ng) + 0.5) * h for a in range(3)]
    Z, Y, X = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    for d, C in enumerate((X, Y, Z)):
        f = C ** 3 + 0.5 * X * Y * Z           # the cross term is linear along each axis
        out = L.apply_block(s, f, ng, h, d)
        inner = (slice(ng, -ng),) * 3
        Cin, Xi, Yi, Zi = C[inner], X[inner], Y[inner], Z[inner]
        other = {0: Yi * Zi, 1: Xi * Zi, 2: Xi * Yi}[d]
        if s.dr == 1:
            ex = 3 * Cin ** 2 + 0.5 * other
        else:
            ex = 6 * Cin
        assert np.max(np.abs(out - ex)) < 1e-9 * np.max(np.abs(ex))
