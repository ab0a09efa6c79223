"""Oracle: compact finite-difference scheme construction, written from the paper.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import this
module; only ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark use it.

Everything here follows Daszuta, "Spectrally-tuned compact finite-difference
schemes with domain decomposition" (arXiv 2302.14858):

* the coefficient tuples alpha^(d_K) and the multi-derivative ansatz
  (Sec. 2, Eqs. coeffTupDefn, fcnTupDefn, mdAnsatz);
* Taylor matching with the normalisation alpha^(d_r)_0 = 1 (Eq. Tcons);
* the modified wavenumber and the spectral error functional
  (Sec. 2.1, Eqs. phase_tup, fdpwerrdef, sp_error, optfunc) with the cut-off
  weight of Eq. gammacut;
* the relative error of the normalised wavenumber and its series
  (Eqs. relmodnormwavnum, errrelmodwavcent);
* the matched explicit closure of Sec. 2.4 (Eq. errelmodwavecentmatch and the
  two conditions that follow it).

Arithmetic: exact rationals (``fractions.Fraction``) when a scheme is fully
determined by Taylor matching; ``mpmath`` at ``DPS`` decimal digits when it is
tuned.  The paper uses a CAS at arbitrary precision plus IPOPT; the objective
of Eq. optfunc is a quadratic form in the coefficients and the constraints are
linear, so the minimiser is the solution of the KKT linear system, which is
what :func:`tune` solves.  No symmetry of the coefficients is imposed: for the
centred schemes it comes out of the minimisation, as the paper remarks.

Reading of the closure conditions: the paper states the matching conditions
as "C_0 = d^{2p}/d eta^{2p} eps[closure] at 0" and "0 = d^{2p+1}/d eta^{2p+1}
eps[closure] at 0".  C_0 is defined as the coefficient of eta^{2p} in the
series of Eq. errrelmodwavcent, so the first condition is read as equality of
series coefficients (the derivative would carry a factor (2p)!).  With this
reading the closures printed in Tabs. pade_deg_one, pade_deg_two, num_deg_one
and num_deg_two are reproduced (see tests/test_oracle_schemes.py).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from functools import lru_cache
from math import factorial
from typing import Dict, List, Optional, Sequence, Tuple

import mpmath as mp

DPS = 60  # decimal digits for the tuned (non-rational) schemes


# ---------------------------------------------------------------------------
# Scheme record
# ---------------------------------------------------------------------------

@dataclass
class Stencil:
    """A coefficient tuple alpha^(d_K) = (alpha_n), n = -L..R (Eq. coeffTupDefn)."""

    dK: int                      # derivative class d_K of the samples it multiplies
    L: int
    R: int
    coef: List = field(default_factory=list)   # index n + L

    def get(self, n):
        if -self.L <= n <= self.R:
            return self.coef[n + self.L]
        return 0

    def offsets(self):
        return range(-self.L, self.R + 1)


@dataclass
class Scheme:
    """An implicit (or explicit) scheme of Eq. mdAnsatz with d_I = (0,) unless stated.

    ``lhs`` is alpha^(d_r); ``rhs`` is the list of alpha^(d_I).
    ``closure`` lists the explicit stencils used on the rows nearest a block
    end (row k*_- first, then k*_- + 1, ...); the right end uses the mirror
    image.  ``order`` is the formal order of accuracy.
    """

    name: str
    dr: int
    order: int
    lhs: Stencil
    rhs: List[Stencil]
    closure: List[Stencil] = field(default_factory=list)

    # convenience views for the single-RHS-class (d_I = (0,)) case
    @property
    def nl(self) -> int:
        return max(self.lhs.L, self.lhs.R)

    @property
    def M(self) -> int:
        r = self.rhs[0]
        return max(r.L, r.R)

    def lhs_floats(self) -> List[float]:
        return [float(self.lhs.get(n)) for n in range(-self.nl, self.nl + 1)]

    def rhs_floats(self) -> List[float]:
        return [float(self.rhs[0].get(n)) for n in range(-self.M, self.M + 1)]

    def closure_floats(self) -> Tuple[int, List[List[float]]]:
        if not self.closure:
            return 0, []
        mc = max(max(c.L, c.R) for c in self.closure)
        rows = [[float(c.get(n)) for n in range(-mc, mc + 1)] for c in self.closure]
        return mc, rows


# ---------------------------------------------------------------------------
# Taylor constraints (Eq. Tcons substituted into Eq. mdAnsatz)
# ---------------------------------------------------------------------------

def _unknown_layout(lhs_ext: Tuple[int, int], rhs_ext: Sequence[Tuple[int, int, int]]):
    """Order the unknowns: alpha^(d_r)_{-L..R} then each alpha^(d_I)_{-L..R}.

    Returns a list of (side, dK, n) with side 'r' for the left-hand side
    (unknown derivative d_r) and 'I' for the known samples.
    """
    layout = []
    dr, L, R = lhs_ext
    for n in range(-L, R + 1):
        layout.append(("r", dr, n))
    for dK, L, R in rhs_ext:
        for n in range(-L, R + 1):
            layout.append(("I", dK, n))
    return layout


def taylor_row(layout, l, one=Fraction(1)):
    """Coefficient row of the l-th Taylor condition.

    Substituting f^(dK)_{k+n} = sum_l (n dx)^l / l! f^(dK+l)_k into
    Eq. mdAnsatz and collecting dx^l f^(l)_k gives

        sum_I sum_n alpha^(d_I)_n n^(l-d_I)/(l-d_I)!  -  sum_n alpha^(d_r)_n n^(l-d_r)/(l-d_r)!  = 0.
    """
    row = []
    for side, dK, n in layout:
        p = l - dK
        if p < 0:
            row.append(0 * one)
            continue
        v = one * (n ** p) / factorial(p)   # 0**0 == 1
        row.append(v if side == "I" else -v)
    return row


def _normalisation_row(layout, dr, one=Fraction(1)):
    return [one if (side == "r" and n == 0) else 0 * one for side, dK, n in layout]


def _solve_exact(A: List[List[Fraction]], b: List[Fraction]) -> List[Fraction]:
    """Gauss-Jordan elimination over the rationals (square, non-singular)."""
    n = len(A)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for c in range(n):
        p = next((r for r in range(c, n) if M[r][c] != 0), None)
        if p is None:
            raise ValueError("singular Taylor system")
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [vr - f * vc for vr, vc in zip(M[r], M[c])]
    return [M[i][n] for i in range(n)]


def _unpack(layout, x, lhs_ext, rhs_ext) -> Tuple[Stencil, List[Stencil]]:
    dr, L, R = lhs_ext
    lhs = Stencil(dr, L, R, [])
    rhs = [Stencil(dK, Lk, Rk, []) for dK, Lk, Rk in rhs_ext]
    for (side, dK, n), v in zip(layout, x):
        if side == "r":
            lhs.coef.append(v)
        else:
            for s in rhs:
                if s.dK == dK:
                    s.coef.append(v)
    return lhs, rhs


def determined_scheme(dr: int, lhs_LR: Tuple[int, int], rhs_ext: Sequence[Tuple[int, int, int]]):
    """Fully determined scheme: C_S = C_T + 1 (Sec. 2, after Eq. Tcons).

    ``rhs_ext`` lists (d_I, L, R).  Returns (lhs, rhs, order) with exact
    rational coefficients; ``order`` is the formal order obtained.
    """
    lhs_ext = (dr, lhs_LR[0], lhs_LR[1])
    layout = _unknown_layout(lhs_ext, rhs_ext)
    nunk = len(layout)
    rows = [_normalisation_row(layout, dr)]
    rhs_vec = [Fraction(1)]
    l = 0
    while len(rows) < nunk:
        rows.append(taylor_row(layout, l))
        rhs_vec.append(Fraction(0))
        l += 1
    x = _solve_exact(rows, rhs_vec)
    lhs, rhs = _unpack(layout, x, lhs_ext, rhs_ext)
    # formal order: first Taylor row that is violated, minus d_r
    q = l
    while sum(a * b for a, b in zip(taylor_row(layout, q), x)) == 0:
        q += 1
    return lhs, rhs, q - dr


# ---------------------------------------------------------------------------
# Modified wavenumber and spectral error (Eqs. phase_tup, fdpwerrdef, sp_error)
# ---------------------------------------------------------------------------

def _mpf(v):
    """mpmath number from an int, Fraction or mpf."""
    if isinstance(v, Fraction):
        return mp.mpf(v.numerator) / v.denominator
    return mp.mpf(v)


def _E_dot(st: Stencil, eta):
    """alpha^(d_K) . E^(d_K)(eta) with E_m = exp(i m eta) (Eq. phase_tup)."""
    return mp.fsum(_mpf(st.get(n)) * mp.expj(n * eta) for n in st.offsets())


def modified_wavenumber_power(s: Scheme, eta):
    """(i eta~)^{d_r} of Eq. fdpwerrdef (complex)."""
    eta = mp.mpf(eta)
    num = mp.fsum((1j * eta) ** r.dK * _E_dot(r, eta) for r in s.rhs)
    return num / _E_dot(s.lhs, eta)


def spectral_error(s: Scheme, eta):
    """e~(eta) of Eq. sp_error."""
    eta = mp.mpf(eta)
    return mp.fsum((1j * eta) ** r.dK * _E_dot(r, eta) for r in s.rhs) - (1j * eta) ** s.dr * _E_dot(s.lhs, eta)


# ---------------------------------------------------------------------------
# Series of the relative error eps(eta) = eta~^d/eta^d - 1 (Eq. relmodnormwavnum)
# ---------------------------------------------------------------------------

def eps_series(s: Scheme, nterms: int, exact: bool = False):
    """Power-series coefficients c_j of eps(eta) = sum_j c_j eta^j, j < nterms.

    (i eta~)^d = N(eta)/Dn(eta) with N = sum_I (i eta)^{d_I} alpha^(d_I).E and
    Dn = alpha^(d_r).E; eps = N / ((i eta)^d Dn) - 1.  The series are formed
    from exp(i n eta) = sum_j (i n eta)^j / j! and divided term by term.
    Coefficients are complex in general (biased schemes); returned as
    (real, imag) pairs of Fractions when ``exact`` else mpmath numbers.
    """
    one = Fraction(1) if exact else mp.mpf(1)
    conv = (lambda v: Fraction(v)) if exact else _mpf
    J = nterms + s.dr + 2

    # complex numbers as (re, im) pairs to stay exact
    def cmul(a, b):
        return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])

    ipow = [(one, 0 * one), (0 * one, one), (-one, 0 * one), (0 * one, -one)]

    def series_E(st: Stencil, shift: int):
        # sum_n alpha_n exp(i n eta) * (i eta)^shift, as coefficients of eta^j
        out = [(0 * one, 0 * one) for _ in range(J)]
        for j in range(J):
            if j - shift < 0:
                continue
            jj = j - shift
            acc = 0 * one
            for n in st.offsets():
                acc += conv(st.get(n)) * (n ** jj) / factorial(jj)   # 0**0 == 1
            # (i)^jj from exp expansion times (i)^shift
            c = cmul(ipow[jj % 4], ipow[shift % 4])
            out[j] = (out[j][0] + acc * c[0], out[j][1] + acc * c[1])
        return out

    N = [(0 * one, 0 * one) for _ in range(J)]
    for r in s.rhs:
        t = series_E(r, r.dK)
        N = [(a[0] + b[0], a[1] + b[1]) for a, b in zip(N, t)]
    # divide N by (i eta)^d: shift down by d and multiply by i^{-d}
    d = s.dr
    inv_id = ipow[(-d) % 4]
    Nd = [cmul(N[j + d], inv_id) for j in range(J - d)]
    Dn = series_E(s.lhs, 0)[: J - d]

    # power-series division Q = Nd / Dn
    def cdiv(a, b):
        den = b[0] * b[0] + b[1] * b[1]
        return ((a[0] * b[0] + a[1] * b[1]) / den, (a[1] * b[0] - a[0] * b[1]) / den)

    Q = []
    for j in range(nterms):
        acc = Nd[j]
        for i in range(1, j + 1):
            t = cmul(Dn[i], Q[j - i])
            acc = (acc[0] - t[0], acc[1] - t[1])
        Q.append(cdiv(acc, Dn[0]))
    Q[0] = (Q[0][0] - one, Q[0][1])
    return Q


# ---------------------------------------------------------------------------
# Spectral tuning (Eqs. optfunc, gammacut): equality-constrained quadratic
# minimisation solved through its KKT system
# ---------------------------------------------------------------------------

def tune(dr: int, lhs_LR: Tuple[int, int], rhs_ext: Sequence[Tuple[int, int, int]],
         order: int, eta_c) -> Tuple[Stencil, List[Stencil]]:
    """min eps[e~; gamma(.; eta_c)] subject to alpha^(d_r)_0 = 1 and Taylor rows.

    Formal order ``order`` for derivative d_r requires the Taylor rows
    l = 0 .. order + d_r - 1 (Eq. Tcons).  The objective of Eq. optfunc is
    c^T H c with H_jk = int_0^{eta_c} Re(phi_j conj(phi_k)) d eta, where phi_j
    is the contribution of unknown j to e~(eta) (Eq. sp_error).
    """
    with mp.workdps(DPS):
        lhs_ext = (dr, lhs_LR[0], lhs_LR[1])
        layout = _unknown_layout(lhs_ext, rhs_ext)
        nunk = len(layout)
        cons = [[_mpf(v) for v in _normalisation_row(layout, dr)]]
        rhs_c = [mp.mpf(1)]
        for l in range(order + dr):
            cons.append([_mpf(v) for v in taylor_row(layout, l)])
            rhs_c.append(mp.mpf(0))
        eta_c = mp.mpf(eta_c)

        def phi(j, eta):
            side, dK, n = layout[j]
            v = (1j * eta) ** dK * mp.expj(n * eta)
            return v if side == "I" else -v

        H = mp.matrix(nunk, nunk)
        for j in range(nunk):
            for k in range(j, nunk):
                val = mp.quad(lambda e: mp.re(phi(j, e) * mp.conj(phi(k, e))), [0, eta_c])
                H[j, k] = val
                H[k, j] = val
        ncons = len(cons)
        K = mp.matrix(nunk + ncons, nunk + ncons)
        b = mp.matrix(nunk + ncons, 1)
        for j in range(nunk):
            for k in range(nunk):
                K[j, k] = 2 * H[j, k]
        for i, row in enumerate(cons):
            for j in range(nunk):
                K[nunk + i, j] = row[j]
                K[j, nunk + i] = row[j]
            b[nunk + i] = rhs_c[i]
        x = mp.lu_solve(K, b)
        coeffs = [x[j] for j in range(nunk)]
        lhs, rhs = _unpack(layout, coeffs, lhs_ext, rhs_ext)
        return lhs, rhs


# ---------------------------------------------------------------------------
# Explicit closures (Sec. 2.4)
# ---------------------------------------------------------------------------

def _lstsq_exact_or_mp(rows, rhs, exact):
    """Solve a consistent over-determined system with full column rank."""
    if exact:
        # normal equations over the rationals are exact
        n = len(rows[0])
        AtA = [[sum(r[i] * r[j] for r in rows) for j in range(n)] for i in range(n)]
        Atb = [sum(r[i] * b for r, b in zip(rows, rhs)) for i in range(n)]
        x = _solve_exact(AtA, Atb)
        res = max(abs(sum(a * b for a, b in zip(r, x)) - bb) for r, bb in zip(rows, rhs))
        if res != 0:
            raise ValueError("closure conditions are inconsistent")
        return x
    A = mp.matrix(rows)
    b = mp.matrix(rhs)
    x, res = mp.qr_solve(A, b)
    if res > mp.mpf(10) ** (-(DPS // 2)):
        raise ValueError("closure conditions are inconsistent (residual %s)" % res)
    return [x[i] for i in range(len(rows[0]))]


def explicit_closure(interior: Scheme, mc: int, matched: bool = True) -> Stencil:
    """Centred explicit closure of half-width mc for the interior scheme.

    ``matched=True`` builds C-bar_{p+1}[O(dx^{2p})] of Sec. 2.4: the Taylor rows
    that fix the formal order, the unit normalisation, the lowest error
    constant C_0 of the interior scheme (Eq. errrelmodwavcent) matched, and the
    next (odd) power of eta removed (Eq. errelmodwavecentmatch).
    ``matched=False`` builds the order-only closure C-bar_p (Taylor rows only).
    """
    d = interior.dr
    q = interior.order
    exact = all(isinstance(v, Fraction) for v in interior.lhs.coef)
    one = Fraction(1) if exact else mp.mpf(1)
    ctx = mp.workdps(DPS)
    ctx.__enter__()
    try:
        # unknowns: alpha-bar^(0)_n, n = -mc..mc; alpha-bar^(d)_0 = 1 (explicit)
        offs = list(range(-mc, mc + 1))

        def trow(l):
            return [one * (n ** l) / factorial(l) for n in offs]   # 0**0 == 1

        rows, rhs = [], []
        for l in range(q + d):
            rows.append(trow(l))
            rhs.append(one if l == d else 0 * one)
        if matched:
            ser = eps_series(interior, q + 1, exact=exact)
            C0 = ser[q][0]  # real for centred interior schemes
            # eps of an explicit stencil: coefficient of eta^q is i^q sum a_n n^{q+d}/(q+d)!
            iq = [(1, 0), (0, 1), (-1, 0), (0, -1)][q % 4]
            if iq[1] != 0:
                raise ValueError("odd formal order is not a centred scheme")
            rows.append([iq[0] * v for v in trow(q + d)])
            rhs.append(C0)
            rows.append(trow(q + d + 1))
            rhs.append(0 * one)
        x = _lstsq_exact_or_mp(rows, rhs, exact)
    finally:
        ctx.__exit__(None, None, None)
    return Stencil(0, mc, mc, x)


# ---------------------------------------------------------------------------
# Named schemes used by the workloads
# ---------------------------------------------------------------------------

def _centred(dr, nl, M, order=None, eta_c=None):
    rhs_ext = [(0, M, M)]
    if eta_c is None:
        lhs, rhs, q = determined_scheme(dr, (nl, nl), rhs_ext)
        return lhs, rhs, q
    lhs, rhs = tune(dr, (nl, nl), rhs_ext, order, eta_c)
    return lhs, rhs, order


def _eta(tag):
    return mp.mpf(1) if tag == "1" else 4 * mp.pi / 5


@lru_cache(maxsize=None)
def named(name: str) -> Scheme:
    """Schemes of the appendix tables by name, with their closures.

    Names: ``(d)P1_M`` (Pade, Tabs. pade_deg_one/two), ``(d)Q1_3[1]`` and
    ``(d)Q1_3[4pi/5]`` (Tabs. num_deg_one/two), ``(d)QP_O8[1]`` (pentadiagonal,
    formal order 8, M = 3, tuned with eta_c = 1 by the same procedure), ``(d)E_M``
    (explicit, Tab. misc_explicit).  A suffix ``:E`` replaces the matched
    closure with the order-only explicit closure C-bar_p.
    """
    base, _, variant = name.partition(":")
    dr = int(base[1])
    kind = base[3:]
    if kind.startswith("P1_"):
        M = int(kind[3:])
        lhs, rhs, q = _centred(dr, 1, M)
        ncl, mc_match = 1, q // 2 + 1
    elif kind.startswith("Q1_3["):
        tag = kind[5:-1]
        lhs, rhs, q = _centred(dr, 1, 3, 6, _eta(tag))
        ncl, mc_match = 1, 4
    elif kind.startswith("QP_O8["):
        tag = kind[6:-1]
        lhs, rhs, q = _centred(dr, 2, 3, 8, _eta(tag))
        ncl, mc_match = 2, 5
    elif kind.startswith("E"):
        M = int(kind[1:])
        lhs, rhs, q = _centred(dr, 0, M)
        return Scheme(name, dr, q, lhs, rhs, [])
    else:
        raise KeyError(name)
    s = Scheme(name, dr, q, lhs, rhs, [])
    if variant == "E":
        cl = explicit_closure(s, q // 2, matched=False)
    elif variant == "":
        cl = explicit_closure(s, mc_match, matched=True)
    else:
        raise KeyError(name)
    s.closure = [cl] * ncl
    return s


def required_ghosts(s: Scheme, periodic: bool) -> int:
    """Ghost layers a block needs for the closure prescription (Eq. sch_cent_om).

    Row k*_- + j (j < number of closure rows) reaches mc - j nodes past the
    block end; the first implicit row reaches M - nc.  Periodic lines need none.
    """
    if periodic:
        return 0
    if s.nl == 0:
        return s.M
    nc = len(s.closure)
    need = s.M - nc
    for j, c in enumerate(s.closure):
        need = max(need, max(c.L, c.R) - j)
    return need
