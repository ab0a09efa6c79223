"""Oracle: hybrid iteration of the block closures (Sec. ssec:domdec_iter).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may use it; the product library never does.

What it computes (arXiv 2302.14858, Eq. iter_center_P and its matrix form
Eq. iter_scheme): sub-domains tile a periodic line.  Iterate [0] is the
block-closure derivative of Eq. sch_cent_om.  For i > 0 each sub-domain solves
the interior implicit rows of the scheme on the extended row range
k^c_- + 1 .. k^c_+ - 1, where k^c_- = k*_- - c and k^c_+ = k*_+ + c, with the
derivative at k^c_- and k^c_+ fixed to the previous iterate there.  Those two
nodes lie in the ghost layer: their values are the previous iterate of the
neighbouring sub-domains at the same global nodes (node N_B - c of the left
neighbour, node c - 1 of the right one).  The paper takes c = 2 for centred
tridiagonal schemes; the definition is written for implicit half-width 1, and
only that case is implemented here.

Every line is an independent tridiagonal system; it is solved with the Thomas
algorithm (Gaussian elimination without pivoting) in FP64, vectorised over the
lines with numpy.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

from . import lines as OL
from .schemes import Scheme, required_ghosts


def required_ghosts_iterated(s: Scheme, c: int = 2) -> int:
    """Ghost layers the iteration needs: the block closure's, and the interior
    stencil on the first extended row k*_- - c + 1 (reach M + c - 1)."""
    return max(required_ghosts(s, False), s.M + c - 1)


def _thomas(lo, di, up, r):
    """Solve the tridiagonal systems lo x_{k-1} + di x_k + up x_{k+1} = r_k along axis 0
    (constant coefficients, r of shape (n, ...))."""
    n = r.shape[0]
    cp = np.empty(n)
    dp = np.empty_like(r)
    cp[0] = up / di
    dp[0] = r[0] / di
    for k in range(1, n):
        m = di - lo * cp[k - 1]
        cp[k] = up / m
        dp[k] = (r[k] - lo * dp[k - 1]) / m
    x = np.empty_like(r)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def extended_solve(s: Scheme, g, ng: int, h: float, e_minus, e_plus, c: int = 2):
    """One iterate on one sub-domain: lines along axis 0 of g (N_B + 2 ng nodes, ghosts
    included), end values e_minus (at node -c) and e_plus (at node N_B - 1 + c) of shape
    g.shape[1:].  Returns the derivative on the N_B interior nodes."""
    if s.nl != 1:
        raise ValueError("the hybrid iteration is defined for tridiagonal schemes")
    if ng < required_ghosts_iterated(s, c):
        raise ValueError("not enough ghost layers for the iteration")
    g = np.asarray(g, dtype=np.float64)
    NB = g.shape[0] - 2 * ng
    a = s.rhs_floats()
    M = s.M
    al = s.lhs_floats()          # (alpha_-1, 1, alpha_1)
    hinv = 1.0 / h ** s.dr
    rows = np.arange(-c + 1, NB + c - 1)          # k^c_- + 1 .. k^c_+ - 1
    r = np.zeros((rows.size,) + g.shape[1:])
    for i, k in enumerate(rows):
        acc = np.zeros(g.shape[1:])
        for m in range(-M, M + 1):
            acc = acc + a[m + M] * g[ng + k + m]
        r[i] = hinv * acc
    r[0] = r[0] - al[0] * e_minus
    r[-1] = r[-1] - al[2] * e_plus
    x = _thomas(al[0], al[1], al[2], r)
    return x[c - 1:c - 1 + NB]


def iterate_1d(s: Scheme, blocks, ng: int, h: float, iters: int, c: int = 2):
    """Iterates [0] .. [iters] on a periodic tiling of sub-domains along axis 0.

    blocks: array (NS, N_B + 2 ng, ...): sub-domain I (in order along the line) with its
    ghost layers filled from its neighbours.  Returns the list of iterates, each of shape
    (NS, N_B, ...)."""
    blocks = np.asarray(blocks, dtype=np.float64)
    NS = blocks.shape[0]
    NB = blocks.shape[1] - 2 * ng
    lines = blocks.reshape(NS, blocks.shape[1], -1)
    x0 = np.stack([np.stack([OL.apply_line(s, lines[I, :, j], ng, h) for j in range(lines.shape[2])], axis=1)
                   for I in range(NS)])
    out = [x0.reshape((NS, NB) + blocks.shape[2:])]
    prev = x0
    for _ in range(iters):
        cur = np.empty_like(prev)
        for I in range(NS):
            em = prev[(I - 1) % NS, NB - c]
            ep = prev[(I + 1) % NS, c - 1]
            cur[I] = extended_solve(s, lines[I], ng, h, em, ep, c)
        out.append(cur.reshape((NS, NB) + blocks.shape[2:]))
        prev = cur
    return out


def iterate_lattice(s: Scheme, fields: Dict[Tuple[int, int, int], np.ndarray], lattice, ng: int, h: float,
                    direction: int, iters: int, c: int = 2):
    """The iteration along one direction of a periodic lattice of equal blocks.

    fields: block (kx, ky, kz) -> one field [z][y][x] with ng ghost layers, filled from the
    neighbours.  Returns block -> interior derivative [z][y][x] after `iters` iterations."""
    axis = 2 - direction                     # [z][y][x] storage
    nlat = lattice[direction]
    out = {}
    # group the blocks into rows of the lattice along `direction`
    rows = {}
    for key in fields:
        other = tuple(v for d, v in enumerate(key) if d != direction)
        rows.setdefault(other, {})[key[direction]] = key
    for other, members in rows.items():
        keys = [members[i] for i in range(nlat)]
        stack = np.stack([np.moveaxis(fields[k], axis, 0) for k in keys])   # (NS, NB+2ng, a, b)
        inner = [slice(ng, -ng)] * 2
        stack = stack[(slice(None), slice(None)) + tuple(inner)]             # lines of interior nodes only
        res = iterate_1d(s, stack, ng, h, iters, c)[-1]                       # (NS, NB, a, b)
        for i, k in enumerate(keys):
            out[k] = np.moveaxis(res[i], 0, axis)
    return out


def modal_rms_error(global_vals, decomposed_vals, a_cut: float = 1e-8):
    """RMS amplitude and phase errors of Eq. err_met_rms_sp between two derivative approximants
    sampled on one periodic line (global scheme first): the Fourier coefficients a_n = FFT / N of
    both, over the modes whose amplitude relative to the global coefficients' largest is at least
    a_cut (reading: the printed set keeps the modes at or above the cut, which is what its footnote
    describes), eps_A = rms |a_n - b_n| and eps_theta = rms of arg a_n - arg b_n (wrapped to
    (-pi, pi]).  Returns (eps_A, eps_theta)."""
    a = np.fft.fft(np.asarray(global_vals, dtype=np.float64)) / len(global_vals)
    b = np.fft.fft(np.asarray(decomposed_vals, dtype=np.float64)) / len(decomposed_vals)
    sel = np.abs(a) >= a_cut * np.max(np.abs(a))
    eps_a = np.sqrt(np.mean(np.abs(a[sel] - b[sel]) ** 2))
    dth = np.angle(a[sel]) - np.angle(b[sel])
    dth = (dth + np.pi) % (2 * np.pi) - np.pi
    return float(eps_a), float(np.sqrt(np.mean(dth ** 2)))
