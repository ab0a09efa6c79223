"""Oracle: biased (upwind) compact schemes and their line operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import this
module; only ``tests/`` and the benchmark's CPU-baseline leg use it.

Written from Daszuta, arXiv 2302.14858, Sec. ssec:domdec_drp:

* ``ucd``: the left-biased first-degree schemes U^-_M (order 2M+2, with the
  f'' sample; as a line operator, ``line_matrices`` / ``apply_block_hermite``,
  it takes the sampled f'' as data on every row, closure row included) and
  V^-_M (order 2M+1, alpha^(2)_0 = 0) of
  Eq. defChenSchemes, fixed by Taylor matching (Eq. Tcons) on the ansatz of
  Eq. mdAnsatz with alpha^(1) on nodes k-1, k and alpha^(0) on k-M .. k+M.
* ``mirror``: the right-biased scheme of a left-biased one,
  alpha+(1)_m = alpha-(1)_{-m}, alpha+(0)_m = -alpha-(0)_{-m},
  alpha+(2)_0 = -alpha-(2)_0 (the rule stated with Eq. defChenSchemes).
* ``xi_closure``: the closure at k*_- of a left-biased scheme: the
  right-biased mirror plus xi dx^q alpha^(1) . f^(q) over its two implicit
  nodes, f^(q) taken from the centred explicit approximant (q)E_{q/2}
  (Tab. diss_scheme), with q the even order just above the scheme's formal
  order p.  xi is fixed by matching the lowest imaginary coefficient of the
  relative wavenumber error (Eqs. ucd_slow_closure_chi, ucd_fast_closure_chi
  and the matching conditions after them).  Reading: the printed derivative
  degree "2M+2" of Eq. ucd_slow_closure_chi gives an eta power that cannot
  reach the eta^{2M+3} term it is meant to match; the correction of order
  2M+4 reproduces every xi of Tab. ucd_slow_closure, so that is the one used.
* ``xscheme``: X^-_M, the combination lambda U^-_M + (1 - lambda) V^-_{M+1}
  of Eq. LCslowfast with the f'' sample replaced by the explicit (2)E_{M+2}
  (Tab. misc_explicit), and its xi-closure; lambda is the sigma printed in
  Tab. ccux_deg_one_col.
* ``wscheme`` / ``w_rows``: W^-_M, the same combination with lambda the sigma
  of Tab. ccuw_deg_one_col, keeping the f'' term, which is now the centred
  tridiagonal Pade second derivative (2)P1_M solved on the line with its
  matched explicit closure (Tabs. pade_deg_two, the compact approximant the
  text names for W; its caption's "(1)P" can only be the second-degree
  scheme).  At k*_+ that f'' is the closure's explicit value, which turns the
  interior row into the printed Wtilde^-_M; at k*_- the closure Wbar^-_M is
  the xi-closure of that explicit row (mirror at k*_-, where f'' is again the
  closure's).  ``w_eps_series``: the interior error with the compact f''.
* ``line_matrix`` / ``apply_block``: the banded system of Eq. closure_left_X
  (left bias, closure row at k*_-) and its mirror image (right bias, closure
  row at k*_+), or the circulant system on periodic lines, assembled densely
  and solved with numpy (LU with partial pivoting): f~ = h^-1 A^-1 B f.
* ``symmetrised_block``: the mean of both biases' derivatives (the
  symmetrisation of biased schemes in the decomposition study, Sec. 2.5).
* ``upwind_block``: the shift-advection term c d f of Eq. biasderapproxadv,
  with c a field sampled on the grid (the shift component, Sec. ssec:z4c):
  c > 0 takes the left-biased scheme (Im eta~ <= 0), c < 0 the right-biased
  one.  Reading: the printed weight 1/2 (|c| - c) of the second set would
  give |c| D~ = -c D~ for c < 0, the wrong sign for c d f; the selection by
  the sign of c that the text states is used,
  c D~ -> 1/2 (c - |c|) D~[right-biased] + 1/2 (c + |c|) D~[left-biased].

Arithmetic: the coefficients are exact rationals; the line operator is FP64.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb
from typing import Dict, List, Tuple

import numpy as np

from . import lines as L
from . import schemes as S
from .schemes import Scheme, Stencil, determined_scheme, eps_series


# ---------------------------------------------------------------------------
# Scheme construction
# ---------------------------------------------------------------------------

def _stencil_from_map(dK: int, m: Dict[int, Fraction]) -> Stencil:
    lo, hi = min(m), max(m)
    return Stencil(dK, -lo, hi, [m.get(n, Fraction(0)) for n in range(lo, hi + 1)])


def ucd(kind: str, M: int) -> Scheme:
    """U^-_M (kind 'U') or V^-_M (kind 'V') of Eq. defChenSchemes, exact."""
    ext = [(0, M, M)] + ([(2, 0, 0)] if kind == "U" else [])
    lhs, rhs, q = determined_scheme(1, (1, 0), ext)
    return Scheme(f"(1){kind}{M}-", 1, q, lhs, rhs, [])


def mirror(s: Scheme, name: str = "") -> Scheme:
    """Right-biased image of a first-degree biased scheme (and vice versa)."""
    lhs = Stencil(s.lhs.dK, s.lhs.R, s.lhs.L, [s.lhs.get(-n) for n in range(-s.lhs.R, s.lhs.L + 1)])
    rhs = [Stencil(r.dK, r.R, r.L, [(-1) ** (r.dK + 1) * r.get(-n) for n in range(-r.R, r.L + 1)])
           for r in s.rhs]
    return Scheme(name or s.name, s.dr, s.order, lhs, rhs, [])


def explicit_deriv(q: int) -> List[int]:
    """(q)E_{q/2}: dx^q f^(q)_k ~ sum_{n=-q/2}^{q/2} (-1)^(q/2-n) C(q, n+q/2) f_{k+n}
    (the repeated forward/backward differences of Tab. diss_scheme / Eq. dissdef)."""
    h = q // 2
    return [(-1) ** (h - n) * comb(q, n + h) for n in range(-h, h + 1)]


def correction_order(p: int) -> int:
    """Even derivative order of the closure correction: the first even number above p."""
    return p + 2 - (p % 2)


def _closure_with(s_minus: Scheme, xi: Fraction) -> Scheme:
    base = mirror(s_minus)
    q = correction_order(s_minus.order)
    h = q // 2
    e = explicit_deriv(q)
    r0: Dict[int, Fraction] = {}
    for n in base.rhs[0].offsets():
        r0[n] = r0.get(n, Fraction(0)) + base.rhs[0].get(n)
    for j in base.lhs.offsets():
        for t in range(-h, h + 1):
            r0[j + t] = r0.get(j + t, Fraction(0)) + xi * base.lhs.get(j) * e[t + h]
    return Scheme(s_minus.name + ":closure", 1, s_minus.order, base.lhs,
                  [_stencil_from_map(0, r0)] + base.rhs[1:], [])


def _im_coef(s: Scheme, j: int) -> Fraction:
    return eps_series(s, j + 1, exact=True)[j][1]


def xi_closure(s_minus: Scheme) -> Tuple[Fraction, Scheme]:
    """(xi, closure row at k*_-) for a left-biased scheme.

    The imaginary coefficient of eta^(q-1) in the closure's relative error is
    affine in xi; xi makes it equal to the interior scheme's."""
    q = correction_order(s_minus.order)
    target = _im_coef(s_minus, q - 1)
    c0 = _im_coef(_closure_with(s_minus, Fraction(0)), q - 1)
    c1 = _im_coef(_closure_with(s_minus, Fraction(1)), q - 1) - c0
    xi = (target - c0) / c1
    return xi, _closure_with(s_minus, xi)


# sigma of Tab. ccux_deg_one_col
X_LAMBDA = {1: Fraction(37, 100), 2: Fraction(86, 100), 3: Fraction(146, 100)}


def xscheme(M: int, lam: Fraction = None) -> Scheme:
    """X^-_M: lambda U^-_M + (1 - lambda) V^-_{M+1} with f'' -> (2)E_{M+2} (Eq. LCslowfast)."""
    if lam is None:
        lam = X_LAMBDA[M]
    u, v = ucd("U", M), ucd("V", M + 1)
    _, e2rhs, _ = determined_scheme(2, (0, 0), [(0, M + 2, M + 2)])
    a2 = u.rhs[1].get(0)
    lhs = Stencil(1, 1, 0, [lam * u.lhs.get(n) + (1 - lam) * v.lhs.get(n) for n in (-1, 0)])
    r0: Dict[int, Fraction] = {}
    for st, w in ((u.rhs[0], lam), (v.rhs[0], 1 - lam), (e2rhs[0], lam * a2)):
        for n in st.offsets():
            r0[n] = r0.get(n, Fraction(0)) + w * st.get(n)
    return Scheme(f"(1)X{M}-", 1, u.order, lhs, [_stencil_from_map(0, r0)], [])


# sigma of Tab. ccuw_deg_one_col
W_LAMBDA = {1: Fraction(38, 100), 2: Fraction(71, 100), 3: Fraction(95, 100)}


def wscheme(M: int, lam: Fraction = None) -> Scheme:
    """W^-_M: lambda U^-_M + (1 - lambda) V^-_{M+1} (Eq. LCslowfast), the f'' term kept
    (rhs[1], derivative class 2) for the embedded second derivative."""
    if lam is None:
        lam = W_LAMBDA[M]
    u, v = ucd("U", M), ucd("V", M + 1)
    lhs = Stencil(1, 1, 0, [lam * u.lhs.get(n) + (1 - lam) * v.lhs.get(n) for n in (-1, 0)])
    r0: Dict[int, Fraction] = {}
    for st, w in ((u.rhs[0], lam), (v.rhs[0], 1 - lam)):
        for n in st.offsets():
            r0[n] = r0.get(n, Fraction(0)) + w * st.get(n)
    a2 = lam * u.rhs[1].get(0)
    return Scheme(f"(1)W{M}-", 1, u.order, lhs, [_stencil_from_map(0, r0), Stencil(2, 0, 0, [a2])], [])


def embedded_second(M: int) -> Scheme:
    """The second derivative W_M embeds: (2)P1_M with its matched explicit closure."""
    return S.named(f"(2)P1_{M}")


def with_explicit_second(s: Scheme, e2: Stencil) -> Scheme:
    """The row of s with its f'' sample replaced by the explicit dx^2 f'' ~ e2 . f."""
    a2 = s.rhs[1].get(0)
    r0: Dict[int, Fraction] = {}
    for st, w in ((s.rhs[0], Fraction(1)), (e2, a2)):
        for n in st.offsets():
            r0[n] = r0.get(n, Fraction(0)) + w * st.get(n)
    return Scheme(s.name + ":explicit", 1, s.order, s.lhs, [_stencil_from_map(0, r0)], [])


def w_rows(M: int) -> Tuple[Scheme, Scheme, Scheme]:
    """(W^-_M interior, Wbar^-_M at k*_-, Wtilde^-_M at k*_+)."""
    s = wscheme(M)
    wt = with_explicit_second(s, embedded_second(M).closure[0])
    _, wb = xi_closure(wt)
    return s, wb, wt


def _conv(a: Stencil, b: Stencil, dK: int) -> Dict[int, Fraction]:
    out: Dict[int, Fraction] = {}
    for i in a.offsets():
        for j in b.offsets():
            out[i + j] = out.get(i + j, Fraction(0)) + Fraction(a.get(i)) * Fraction(b.get(j))
    return out


def w_compact_scheme(M: int) -> Scheme:
    """The interior W^-_M with its compact f'' as one scheme on f alone (periodic lines).

    With A2 f''~ = h^-2 B2 f the row is A1 . f~' = h^-1 (B0 . f + a2 (B2 / A2) . f), i.e. the
    scheme (A1 * A2) . f~' = h^-1 (B0 * A2 + a2 B2) . f with * the convolution of stencils."""
    s, P = wscheme(M), embedded_second(M)
    a2 = s.rhs[1].get(0)
    lhs = _conv(s.lhs, P.lhs, 1)
    r = _conv(s.rhs[0], P.lhs, 0)
    for n in P.rhs[0].offsets():
        r[n] = r.get(n, Fraction(0)) + a2 * P.rhs[0].get(n)
    lo, hi = min(lhs), max(lhs)
    return Scheme(f"(1)W{M}-:compact", 1, s.order,
                  Stencil(1, -lo, hi, [lhs.get(n, Fraction(0)) for n in range(lo, hi + 1)]),
                  [_stencil_from_map(0, r)], [])


def w_eps_series(M: int, nterms: int):
    """Relative wavenumber error series of the interior W^-_M with its compact f''."""
    return S.eps_series(w_compact_scheme(M), nterms, exact=True)


@lru_cache(maxsize=None)
def named(name: str) -> Tuple[Scheme, Scheme]:
    """(left-biased interior scheme, its closure row at k*_-) for "(1)V{M}", "(1)U{M}" (M = 1..4),
    "(1)X{M}" or "(1)W{M}" (M = 1..3).  U carries the sampled f'' term in rhs[1] of both rows
    (a Hermite-type input, see ``line_matrices``); W carries its f'' term in rhs[1] of the interior
    row, filled by the embedded second derivative."""
    if not name.startswith("(1)"):
        raise KeyError(name)
    kind, M = name[3], int(name[4:])
    if kind == "V" and 1 <= M <= 4:
        s = ucd("V", M)
    elif kind == "U" and 1 <= M <= 4:
        s = ucd("U", M)
    elif kind == "X" and M in X_LAMBDA:
        s = xscheme(M)
    elif kind == "W" and M in W_LAMBDA:
        s, wb, _ = w_rows(M)
        return s, wb
    else:
        raise KeyError(name)
    return s, xi_closure(s)[1]


def required_ghosts(name: str) -> int:
    """Reach past a block end of the rows of both biases (N_g >= M + 2 for X_M,
    after Eq. closure_left_X).  Left bias: the closure row k*_- reaches its
    left half-width, interior row k*_- + 1 its left half-width - 1, interior
    row k*_+ its right half-width; the right bias is the mirror image.  W also
    needs what its embedded second derivative's closure reaches."""
    s, c = named(name)
    need = max(c.rhs[0].L, s.rhs[0].L - 1, s.rhs[0].R)
    if name[3] == "W":
        need = max(need, S.required_ghosts(embedded_second(int(name[4:])), False))
    return need


# ---------------------------------------------------------------------------
# Line operator (Eq. closure_left_X and its mirror; periodic circulant)
# ---------------------------------------------------------------------------

def _f(v) -> float:
    return float(v)


@lru_cache(maxsize=None)
def line_matrix(name: str, bias: int, N: int, ng: int, periodic: bool) -> np.ndarray:
    """Dense D with f~ = h^-1 D g for one line, g holding the N + 2 ng samples
    (g[ng + k] is interior node k).  bias = -1: left-biased rows with the closure
    at k*_-; bias = +1: the mirror image (closure at k*_+)."""
    if name[3] == "U":
        raise ValueError(f"{name} needs the sampled f'' (line_matrices)")
    return line_matrices(name, bias, N, ng, periodic)[0]


@lru_cache(maxsize=None)
def line_matrices(name: str, bias: int, N: int, ng: int, periodic: bool):
    """(D, D2): f~ = h^-1 D g + h D2 s for one line, s the sampled f'' on the N interior nodes
    (D2 is None unless the scheme samples f'', i.e. U_M: every row of Eq. defChenSchemes, closure
    row included, carries its alpha^(2)_0 dx^2 f''_k)."""
    s, c = named(name)
    if bias > 0:
        s, c = mirror(s), mirror(c)
    A = np.zeros((N, N))
    B = np.zeros((N, N + 2 * ng))
    E2 = None
    C2 = np.zeros((N, N)) if name[3] == "U" else None
    if len(s.rhs) > 1 and C2 is None:
        # W: the f'' term of every interior row from the embedded second derivative
        # (unit spacing), dense over the same samples
        P = embedded_second(int(name[4:]))
        E2 = np.zeros((N, N + 2 * ng))
        for j in range(N + 2 * ng):
            if periodic and not (ng <= j < ng + N):
                continue
            e = np.zeros(N + 2 * ng)
            e[j] = 1.0
            if periodic:
                e[:ng] = e[N:N + ng]
                e[ng + N:] = e[ng:2 * ng]
            E2[:, j] = L.apply_line(P, e, ng, 1.0, periodic)
        a2 = _f(s.rhs[1].get(0))

    def put(row, lhs, rhs, wrap):
        for n in lhs.offsets():
            col = row + n
            if wrap:
                col %= N
            A[row, col] += _f(lhs.get(n))
        for n in rhs.offsets():
            col = row + n
            if wrap:
                col %= N
            elif not (-ng <= col < N + ng):
                raise ValueError(f"{name}: row {row} reaches node {col}, outside {ng} ghost layers")
            B[row, ng + col] += _f(rhs.get(n))

    for k in range(N):
        closure_row = (not periodic) and ((bias < 0 and k == 0) or (bias > 0 and k == N - 1))
        if closure_row:
            put(k, c.lhs, c.rhs[0], False)
            if C2 is not None:
                C2[k, k] = _f(c.rhs[1].get(0))
        else:
            put(k, s.lhs, s.rhs[0], periodic)
            if E2 is not None:
                B[k] += a2 * E2[k]
            if C2 is not None:
                C2[k, k] = _f(s.rhs[1].get(0))
    if C2 is None:
        return np.linalg.solve(A, B), None
    return np.linalg.solve(A, B), np.linalg.solve(A, C2)


def apply_block(name: str, bias: int, f: np.ndarray, ng: int, h: float, direction: int,
                periodic: bool = False) -> np.ndarray:
    """Biased first derivative along ``direction`` of one block-field [z][y][x]
    (ng ghosts on every side); returns the interior [z][y][x]."""
    f = np.asarray(f, dtype=np.float64)
    nz, ny, nx = (e - 2 * ng for e in f.shape)
    n = (nx, ny, nz)
    N = n[direction]
    D = line_matrix(name, bias, N, ng, periodic)
    ax = 2 - direction
    g = np.moveaxis(f, ax, -1)                      # line nodes last
    sl = [slice(ng, ng + e) for e in (nz, ny, nx)]
    del sl[ax]
    g = g[tuple(sl)]                                # interior of the other two directions
    if periodic:
        # ghosts are not read: wrap the interior samples
        gi = g[..., ng:ng + N]
        gg = np.concatenate([gi[..., N - ng:] if ng else gi[..., :0], gi, gi[..., :ng]], axis=-1)
        out = gg @ D.T / h
    else:
        out = g @ D.T / h
    return np.moveaxis(out, -1, ax)


def apply_block_hermite(name: str, bias: int, f: np.ndarray, f2: np.ndarray, ng: int, h: float, direction: int,
                        periodic: bool = False) -> np.ndarray:
    """U_M: the biased first derivative along ``direction`` of one block-field [z][y][x] (ng ghosts)
    given the sampled second derivative f2 of the same field along that direction on the interior
    [z][y][x]."""
    f = np.asarray(f, dtype=np.float64)
    nz, ny, nx = (e - 2 * ng for e in f.shape)
    N = (nx, ny, nz)[direction]
    D, D2 = line_matrices(name, bias, N, ng, periodic)
    ax = 2 - direction
    g = np.moveaxis(f, ax, -1)
    sl = [slice(ng, ng + e) for e in (nz, ny, nx)]
    del sl[ax]
    g = g[tuple(sl)]
    if periodic:
        gi = g[..., ng:ng + N]
        g = np.concatenate([gi[..., N - ng:] if ng else gi[..., :0], gi, gi[..., :ng]], axis=-1)
    s2 = np.moveaxis(np.asarray(f2, dtype=np.float64), ax, -1)
    out = g @ D.T / h + (s2 @ D2.T) * h
    return np.moveaxis(out, -1, ax)


def _one_bias(name, bias, f, ng, h, direction, periodic, f2):
    if f2 is not None:
        return apply_block_hermite(name, bias, f, f2, ng, h, direction, periodic)
    return apply_block(name, bias, f, ng, h, direction, periodic)


def upwind_block(name: str, f: np.ndarray, c: np.ndarray, ng: int, h: float, direction: int,
                 periodic: bool = False, f2: np.ndarray = None) -> np.ndarray:
    """c d_dir f with upwind selection (Eq. biasderapproxadv, read as stated in
    the module header): c > 0 takes the left-biased scheme, c < 0 the
    right-biased one; c is the interior [z][y][x] of the velocity field
    (f2: the sampled f'' of U_M)."""
    dl = _one_bias(name, -1, f, ng, h, direction, periodic, f2)
    dr = _one_bias(name, +1, f, ng, h, direction, periodic, f2)
    c = np.asarray(c, dtype=np.float64)
    return 0.5 * (c - np.abs(c)) * dr + 0.5 * (c + np.abs(c)) * dl


def symmetrised_block(name: str, f: np.ndarray, ng: int, h: float, direction: int,
                      periodic: bool = False, f2: np.ndarray = None) -> np.ndarray:
    """The symmetrised biased derivative: the mean of the left- and right-biased results
    (the symmetrisation of biased schemes in the decomposition study of Sec. 2.5)."""
    return 0.5 * (_one_bias(name, -1, f, ng, h, direction, periodic, f2) +
                  _one_bias(name, +1, f, ng, h, direction, periodic, f2))


def iterated_ghosts(name: str) -> int:
    """Ghost layers the iteration needs: the closure's, and the interior rows that now also run on the
    first (left bias) or last (right bias) node, reaching the interior stencil's full half-width."""
    s, _ = named(name)
    return max(required_ghosts(name), s.rhs[0].L, s.rhs[0].R)


def iterate_1d(name: str, bias: int, blocks, ng: int, h: float, iters: int):
    """Iterates [0] .. [iters] of a biased scheme on a periodic tiling of sub-domains (Eq.
    iter_left_X for the left bias, its mirror image for the right one).

    [0] is the block-closure derivative (Eq. closure_left_X).  For i > 0 every row of the
    sub-domain takes the interior scheme, and the value at k^c = k*_- - 1 (left bias; k*_+ + 1 for the
    right bias), a ghost node, is fixed to the previous iterate there: the last node of the left
    neighbour (the first node of the right neighbour).  blocks: (NS, N_B + 2 ng) samples, ghosts
    filled from the neighbours, optionally with trailing axes of independent lines.  Returns the list
    of iterates, each (NS, N_B, ...)."""
    blocks = np.asarray(blocks, dtype=np.float64)
    NS, NB = blocks.shape[0], blocks.shape[1] - 2 * ng
    s, _ = named(name)
    if bias > 0:
        s = mirror(s)
    D0 = line_matrix(name, bias, NB, ng, False)
    out = [np.stack([np.tensordot(D0, blocks[I], axes=(1, 0)) / h for I in range(NS)])]
    # interior right-hand sides of every row, and the one implicit neighbour's weight
    r = np.zeros((NS, NB) + blocks.shape[2:])
    for m in s.rhs[0].offsets():
        r += _f(s.rhs[0].get(m)) * blocks[:, ng + m: ng + m + NB]
    r /= h
    side = -1 if bias < 0 else 1
    a = _f(s.lhs.get(side))
    for _ in range(iters):
        prev = out[-1]
        cur = np.empty_like(prev)
        for I in range(NS):
            if bias < 0:
                x = prev[(I - 1) % NS, NB - 1]
                for k in range(NB):
                    x = r[I, k] - a * x
                    cur[I, k] = x
            else:
                x = prev[(I + 1) % NS, 0]
                for k in range(NB - 1, -1, -1):
                    x = r[I, k] - a * x
                    cur[I, k] = x
        out.append(cur)
    return out
