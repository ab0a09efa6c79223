"""Pins of the mixed-derivative oracle (oracle/mixed.py, Sec. ssec:z4c).

* Exactness: every row of D is exact for polynomials up to degree q + d - 1, so
  1/2 (D_i D_j + D_j D_i) of p(x_i) r(x_j) with both degrees within that bound is p' r'
  exactly, closure rows and edge ghosts included.
* Periodic closed form: a Fourier mode is an eigenvector of D along each axis with eigenvalue
  i eta~(k h)/h (Eq. fdpwerrdef), so D_x D_y sin(k.x + phi) = -(eta~_x/h)(eta~_y/h) sin(k.x + phi).
* Grid convergence of the closure composition at the formal order.
"""
import numpy as np
import pytest

from oracle import mixed as OM
from oracle import schemes as OS


def _grid(n, ng, h, x0):
    return [x0[a] + (np.arange(-ng, n[a] + ng) + 0.5) * h[a] for a in range(3)]


@pytest.mark.parametrize("name", ["(1)Q1_3[1]", "(1)P1_2", "(1)QP_O8[1]", "(1)E3"])
@pytest.mark.parametrize("di,dj", [(0, 1), (0, 2), (1, 2)])
def test_polynomial_exactness(name, di, dj):
    s = OS.named(name)
    ng = OS.required_ghosts(s, False)
    n, h = (11, 9, 8), (0.13, 0.11, 0.17)
    x = _grid(n, ng, h, (0.2, -0.1, 0.3))
    deg = min(3, s.order)                  # within every row's exactness, O(1) data
    coords = np.meshgrid(x[2], x[1], x[0], indexing="ij")      # z, y, x
    X = [coords[2], coords[1], coords[0]]
    p = 1 + 0.3 * X[di] + 0.2 * X[di] ** 2 + 0.1 * X[di] ** deg
    r = 0.5 - 0.4 * X[dj] + 0.25 * X[dj] ** 2 + 0.05 * X[dj] ** deg
    dp = 0.3 + 0.4 * X[di] + 0.1 * deg * X[di] ** (deg - 1)
    dr = -0.4 + 0.5 * X[dj] + 0.05 * deg * X[dj] ** (deg - 1)
    got = OM.mixed_block(s, p * r, ng, h, (0, 0, 0), di, dj)
    ref = (dp * dr)[ng:-ng, ng:-ng, ng:-ng]
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("name", ["(1)Q1_3[1]", "(1)QP_O8[1]"])
def test_periodic_closed_form(name):
    s = OS.named(name)
    n = (24, 20, 18)
    h = tuple(2 * np.pi / v for v in n)
    x = [np.arange(n[a]) * h[a] for a in range(3)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    k = (3, 5, 2)
    th = k[0] * X + k[1] * Y + k[2] * Z + 0.4
    f = np.pad(np.sin(th), 2)
    for di, dj in ((0, 1), (0, 2), (1, 2)):
        got = OM.mixed_block(s, f, 2, h, (1, 1, 1), di, dj)
        et = [complex(OS.modified_wavenumber_power(s, k[a] * h[a]) / 1j).real / h[a] for a in range(3)]
        ref = -et[di] * et[dj] * np.sin(th)
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_convergence_order_closure():
    s = OS.named("(1)Q1_3[1]")
    ng = 4
    errs = []
    for N in (12, 24, 48):
        hh = 1.0 / N
        n, h = (N, N, 4), (hh, hh, hh)
        x = _grid(n, ng, h, (0.0, 0.0, 0.0))
        Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
        f = np.sin(6 * X + 0.3) * np.sin(5 * Y + 0.1)
        ref = (30 * np.cos(6 * X + 0.3) * np.cos(5 * Y + 0.1))[ng:-ng, ng:-ng, ng:-ng]
        got = OM.mixed_block(s, f, ng, h, (0, 0, 0), 0, 1)
        errs.append(np.max(np.abs(got - ref)))
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert slopes[-1] > 5.3, slopes
