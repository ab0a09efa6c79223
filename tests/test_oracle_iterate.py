"""Pins of the oracle's hybrid closure iteration (Sec. ssec:domdec_iter, Eq. iter_center_P).

* The dense embedded operator [i]D of Eq. iter_scheme, built from the matrices the paper
  defines (G of Eq. example_G, D_L and D_R of Eqs. diff_mat_subL/R for i = 0, and the iterated
  D_L, D_R of Eq. diff_mat_subMR with the selectors E^c and Z^c), applied to a periodic 1D tiling,
  equals the oracle's line-by-line iterates for i = 0..4.
* The iterates converge to the global periodic operator (the overlapping sub-domain systems then
  agree on every shared node): the gap shrinks geometrically and is at round-off after 40 steps.
* Iterate 0 is the block-closure derivative.
"""
import numpy as np
import pytest

import synth
from oracle import iterate as IT
from oracle import lines as L
from oracle import schemes as S

SCHEMES = ["(1)Q1_3[1]", "(2)Q1_3[1]", "(1)P1_2", "(2)P1_2"]


def _tiling(fglob, NB, ng):
    NM = fglob.size
    NS = NM // NB
    return np.stack([fglob[(np.arange(-ng, NB + ng) + I * NB) % NM] for I in range(NS)])


def _G(NS, NB, ng):
    """Eq. example_G: keep each sub-domain's interior, fill its ghosts from the neighbours."""
    W = NB + 2 * ng
    G = np.zeros((NS * W, NS * W))
    for I in range(NS):
        for k in range(W):
            r = I * W + k
            loc = k - ng
            if 0 <= loc < NB:
                G[r, r] = 1.0
            elif loc < 0:
                G[r, ((I - 1) % NS) * W + ng + NB + loc] = 1.0
            else:
                G[r, ((I + 1) % NS) * W + ng + loc - NB] = 1.0
    return G


def _D0(s, NB, ng, h):
    """[0]D on one sub-domain: h^-d D_L^-1 D_R of Eqs. diff_mat_subL/R (ghost rows identity)."""
    W = NB + 2 * ng
    DL = np.eye(W)
    DR = np.zeros((W, W))
    mc, crow = s.closure_floats()
    a, al, M = s.rhs_floats(), s.lhs_floats(), s.M
    sgn = (-1) ** s.dr
    for k in range(NB):
        r = ng + k
        if k == 0:
            DR[r, r - mc:r + mc + 1] = crow[0]
        elif k == NB - 1:
            DR[r, r - mc:r + mc + 1] = [sgn * v for v in crow[0][::-1]]
        else:
            DR[r, r - M:r + M + 1] = a
            DL[r, r - 1:r + 2] = al
    D = np.zeros((W, W))
    D[ng:ng + NB] = (np.linalg.solve(DL, DR) / h ** s.dr)[ng:ng + NB]
    return D


def _iterated_matrices(s, NB, ng, c):
    """D_L, D_R of Eq. diff_mat_subMR (N_c = k^c_- identity rows at each end, "1" rows at
    k^c_+-, interior rows in between), and the selectors Z^c_- Z^c_+ and E^c_- + E^c_+."""
    W = NB + 2 * ng
    kcm, kcp = ng - c, ng + NB - 1 + c          # k^c_-, k^c_+ in local indices
    a, al, M = s.rhs_floats(), s.lhs_floats(), s.M
    DL = np.eye(W)
    DR = np.zeros((W, W))
    DR[kcm, kcm] = 1.0
    DR[kcp, kcp] = 1.0
    for r in range(kcm + 1, kcp):
        DL[r, r - 1:r + 2] = al
        DR[r, r - M:r + M + 1] = a
    Z = np.zeros((W, W))
    E = np.zeros((W, W))
    for r in range(W):
        if kcm < r < kcp:
            Z[r, r] = 1.0
        if r in (kcm, kcp):
            E[r, r] = 1.0
    return DL, DR, Z, E


@pytest.mark.parametrize("name", SCHEMES)
@pytest.mark.parametrize("NM,NB", [(32, 8), (48, 16)])
def test_iterates_equal_dense_embedded_operator(name, NM, NB):
    s = S.named(name)
    c = 2
    ng = IT.required_ghosts_iterated(s, c)
    NS = NM // NB
    W = NB + 2 * ng
    h = 2 * np.pi / NM
    xg = (np.arange(NM) + 0.5) * h
    fglob = np.exp(np.sin(2 * xg)) * 0.05 + 0.01 * np.cos(5 * xg + 0.3)
    blocks = _tiling(fglob, NB, ng)
    F = blocks.reshape(-1)
    G = _G(NS, NB, ng)
    D0 = _D0(s, NB, ng, h)
    Di = G @ np.kron(np.eye(NS), D0) @ G                       # [0]D
    DL, DR, Z, E = _iterated_matrices(s, NB, ng, c)
    bDLinv = np.kron(np.eye(NS), np.linalg.inv(DL))
    bZDR = np.kron(np.eye(NS), Z @ DR) / h ** s.dr
    bE = np.kron(np.eye(NS), E)
    iters = IT.iterate_1d(s, blocks, ng, h, 4, c)
    for i in range(5):
        if i > 0:
            Di = G @ (bDLinv @ (bZDR + bE @ Di))               # Eq. iter_scheme
        ref = (Di @ F).reshape(NS, W)[:, ng:ng + NB]
        assert np.max(np.abs(iters[i] - ref)) <= 1e-12 * np.max(np.abs(ref)), i


@pytest.mark.parametrize("name", SCHEMES)
def test_iterates_converge_to_global_periodic_operator(name):
    s = S.named(name)
    ng = IT.required_ghosts_iterated(s)
    NM, NB = 96, 16
    h = 2 * np.pi / NM
    x = np.arange(NM) * h
    f = np.sin(3 * x) + 0.4 * np.cos(11 * x + 1.0) + 0.1 * np.sin(23 * x + 0.2)
    glob = L.apply_line(s, f, 0, h, periodic=True).reshape(NM // NB, NB)
    its = IT.iterate_1d(s, _tiling(f, NB, ng), ng, h, 40)
    gaps = [np.max(np.abs(it - glob)) for it in its]
    scale = np.max(np.abs(glob))
    assert gaps[0] > 1e-8 * scale                    # the closure differs from the global scheme
    assert gaps[40] <= 1e-13 * scale
    # geometric decrease until round-off: a contraction factor of at most 0.25 per iteration
    for i in range(40):
        if gaps[i] > 1e-13 * scale:
            assert gaps[i + 1] < 0.25 * gaps[i], (i, gaps[i], gaps[i + 1])


def test_iterate_zero_is_block_closure():
    s = S.named("(1)Q1_3[1]")
    ng = IT.required_ghosts_iterated(s)
    rng = np.random.default_rng(5)
    blocks = rng.standard_normal((3, 12 + 2 * ng, 4))
    it0 = IT.iterate_1d(s, blocks, ng, 0.1, 0)[0]
    for I in range(3):
        for j in range(4):
            assert np.array_equal(it0[I, :, j], L.apply_line(s, blocks[I, :, j], ng, 0.1))


def test_lattice_driver_matches_1d():
    """The 3D lattice driver gathers the rows of blocks along each direction in order."""
    s = S.named("(1)Q1_3[1]")
    ng = IT.required_ghosts_iterated(s)
    n, lat = 8, (3, 2, 2)
    h = 2 * np.pi / (n * 3)
    NG = [n * lat[d] for d in range(3)]
    rng = np.random.default_rng(7)
    glob = rng.standard_normal((NG[2], NG[1], NG[0]))
    fields = {}
    for kz in range(lat[2]):
        for ky in range(lat[1]):
            for kx in range(lat[0]):
                iz = (np.arange(-ng, n + ng) + kz * n) % NG[2]
                iy = (np.arange(-ng, n + ng) + ky * n) % NG[1]
                ix = (np.arange(-ng, n + ng) + kx * n) % NG[0]
                fields[(kx, ky, kz)] = glob[np.ix_(iz, iy, ix)]
    res = IT.iterate_lattice(s, fields, lat, ng, h, 0, 2)
    # the x-row of blocks at (ky, kz) = (1, 0), interior line y = 3, z = 5
    row = np.stack([fields[(kx, 1, 0)][ng + 5, ng + 3, :] for kx in range(3)])
    ref = IT.iterate_1d(s, row, ng, h, 2)[-1]
    for kx in range(3):
        assert np.array_equal(res[(kx, 1, 0)][5, 3, :], ref[kx])


# --- the decomposition error metric (Eq. err_met_rms_sp) and the decomposition study (Sec. 2.5) ---

def test_modal_rms_error_closed_forms():
    """Equal inputs give zero; an added delta cos(3x) moves the two coefficients n = +-3 by delta/2
    each, so over the 4 selected modes eps_A = delta / (2 sqrt 2); a phase shift phi of the 3x wave
    gives eps_theta = phi / sqrt 2."""
    N = 64
    x = 2 * np.pi * np.arange(N) / N
    base = np.cos(3 * x) + 0.5 * np.sin(5 * x)
    assert IT.modal_rms_error(base, base) == (0.0, 0.0)
    d = 1e-3
    ea, et = IT.modal_rms_error(base, base + d * np.cos(3 * x))
    assert abs(ea - d / (2 * np.sqrt(2))) < 1e-15 and et < 1e-13
    phi = 0.05
    ea, et = IT.modal_rms_error(base, np.cos(3 * x + phi) + 0.5 * np.sin(5 * x))
    assert abs(et - phi / np.sqrt(2)) < 1e-12


def _decomp_errors(name, fn, NB, iters=3):
    s = S.named(name)
    NM, ng = 128, 4
    wl = synth.decomp_line(fn, NM=NM, NB=NB, ng=ng)
    h = wl.blocks[0].h[0]
    xg = (np.arange(NM) + 0.5) * h
    glob = L.apply_line(s, fn(xg), 0, h, periodic=True)
    blocks = np.stack([wl.field_view(b, 0)[ng, ng, :] for b in range(len(wl.blocks))])
    its = IT.iterate_1d(s, blocks, ng, h, iters)
    return [IT.modal_rms_error(glob, it.reshape(-1)) for it in its]


@pytest.mark.parametrize("name,fn", [("(1)P1_2", synth.paper_g), ("(1)Q1_3[1]", synth.paper_g),
                                     ("(2)P1_2", synth.paper_h), ("(2)Q1_3[1]", synth.paper_h)])
def test_decomposition_study_trends(name, fn):
    """The trends the decomposition figures report, on the paper's g and h at N_M = 128, N_g = 4: the
    iterated closures approach the global scheme (both errors fall with every iteration, by two orders
    of magnitude or more after three), and for the first degree the larger sub-domains (N_B = 32) give
    the smaller error at every iteration."""
    e16 = _decomp_errors(name, fn, 16)
    e32 = _decomp_errors(name, fn, 32)
    for e in (e16, e32):
        for i in range(3):
            assert e[i + 1][0] < e[i][0] and e[i + 1][1] < e[i][1], (name, i, e)
        assert e[3][0] < 1e-2 * e[0][0]
    if name.startswith("(1)"):
        for i in range(4):
            assert e32[i][0] < e16[i][0], (name, i)
