"""Pins of the Kreiss-Oliger oracle (oracle/dissipation.py, Eq. dissdef).

* The repeated differences reproduce the binomial stencils (2r)E_r printed in
  Tab. diss_scheme (applied to a unit impulse).
* On a periodic line a Fourier mode is an eigenvector: the symbol of
  (D_+)^r (D_-)^r is (2 cos(eta) - 2)^r / dx^(2r) = (-4 sin^2(eta/2))^r / dx^(2r), so
  Q^(2r) sin(theta) = -sigma sin^(2r)(eta/2) / dx * sin(theta), a closed form independent of
  the stencil (and non-positive: the operator dissipates).
* Block lines in every direction agree with the line operator.
"""
import json
import os

import numpy as np
import pytest

from oracle import dissipation as D

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "biased_tables.json")))


@pytest.mark.parametrize("r", [2, 3, 4, 5, 6])
def test_repeated_differences_reproduce_tab_diss_scheme(r):
    ng, N, h = r, 2 * r + 1, 1.0
    g = np.zeros(N + 2 * ng)
    g[ng + N // 2] = 1.0                     # unit impulse at the middle node
    sigma = 1.0
    q = D.ko_line(g, ng, h, r, sigma)
    # Q = -(-1)^r / 4^r * sigma * h^(2r-1) * D^(2r); D^(2r) of the impulse, read at node N//2 + m,
    # is the stencil entry for offset -m (symmetric)
    d2r = q / (-((-1) ** r) / 4 ** r * sigma)
    row = GOLD["diss_scheme"][str(2 * r)]
    got = [d2r[N // 2 + m] for m in range(-r, r + 1)]
    assert np.allclose(got, row, rtol=0, atol=1e-9 * max(abs(v) for v in row))


@pytest.mark.parametrize("r,sigma", [(2, 0.3), (3, 0.5), (4, 0.04), (5, 1.0)])
def test_periodic_closed_form(r, sigma):
    N = 40
    h = 2 * np.pi / N
    x = np.arange(N) * h
    for k, ph in ((1, 0.2), (7, 1.3), (19, 0.4), (20, 0.9)):
        th = k * x + ph
        got = D.ko_line(np.sin(th), 0, h, r, sigma, periodic=True)
        ref = -sigma * np.sin(k * h / 2) ** (2 * r) / h * np.sin(th)
        assert np.max(np.abs(got - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref))), k


def test_block_directions_match_lines():
    rng = np.random.default_rng(4)
    ng, n = 4, (9, 7, 6)
    f = rng.standard_normal(tuple(e + 2 * ng for e in n[::-1]))
    for d in range(3):
        out = D.ko_block(f, ng, 0.3, d, 4, 0.04)
        idx = [2 + ng, 3 + ng, 4 + ng]
        idx[2 - d] = slice(None)
        ref = D.ko_line(f[tuple(idx)], ng, 0.3, 4, 0.04)
        oi = [2, 3, 4]
        oi[2 - d] = slice(None)
        assert np.allclose(out[tuple(oi)], ref, rtol=0, atol=1e-14)


def test_needs_r_ghosts():
    with pytest.raises(ValueError):
        D.ko_line(np.zeros(10 + 6), 3, 1.0, 4, 1.0)
