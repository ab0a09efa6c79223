"""Oracle: Kreiss-Oliger dissipation, written from the paper.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import this
module; only ``tests/`` uses it.

Eq. dissdef of arXiv 2302.14858 (Sec. 3, advection tests; applied to every
field component in every direction in Sec. ssec:z4c):

    Q^(2r) = -(-1)^r / 2^(2r) * sigma * dx^(2r-1) * (D_+)^r (D_-)^r,
    D_+ f_i = (f_{i+1} - f_i) / dx,   D_- f_i = (f_i - f_{i-1}) / dx.

``ko_line`` applies the difference operators literally, r times each, on the
stored samples of a line (the block's ghost layers supply the r nodes each
side needs); no stencil is tabulated.  Periodic lines wrap instead.
"""
from __future__ import annotations

import numpy as np


def _dminus(v: np.ndarray, lo: int, h: float):
    """D_- on samples v of nodes lo, lo+1, ...: defined from node lo+1 on."""
    return (v[1:] - v[:-1]) / h, lo + 1


def _dplus(v: np.ndarray, lo: int, h: float):
    """D_+ on samples v of nodes lo, lo+1, ...: defined up to the last node but one."""
    return (v[1:] - v[:-1]) / h, lo


def ko_line(g: np.ndarray, ng: int, h: float, r: int, sigma: float, periodic: bool = False) -> np.ndarray:
    """Q^(2r) f on the N interior nodes of one line; g holds N + 2 ng samples
    (g[ng + k] is node k), or just the N interior samples when periodic."""
    g = np.asarray(g, dtype=np.float64)
    if periodic:
        N = g.size
        v = g[np.arange(-r, N + r) % N]
        lo = -r
    else:
        if ng < r:
            raise ValueError(f"Kreiss-Oliger of degree {2 * r} needs {r} ghost layers, line has {ng}")
        N = g.size - 2 * ng
        v = g[ng - r: ng + N + r]
        lo = -r
    for _ in range(r):
        v, lo = _dminus(v, lo, h)
    for _ in range(r):
        v, lo = _dplus(v, lo, h)
    assert lo == 0 and v.size == N, (lo, v.size, N)
    return -((-1) ** r) / 2 ** (2 * r) * sigma * h ** (2 * r - 1) * v


def ko_block(f: np.ndarray, ng: int, h: float, direction: int, r: int, sigma: float,
             periodic: bool = False) -> np.ndarray:
    """Q^(2r) along ``direction`` (0=x, 1=y, 2=z) of one block-field [z][y][x] with ng
    ghosts on every side; returns the interior [z][y][x]."""
    f = np.asarray(f, dtype=np.float64)
    nz, ny, nx = (e - 2 * ng for e in f.shape)
    ax = 2 - direction
    g = np.moveaxis(f, ax, -1)
    sl = [slice(ng, ng + e) for e in (nz, ny, nx)]
    del sl[ax]
    g = g[tuple(sl)]
    N = (nx, ny, nz)[direction]
    out = np.empty(g.shape[:-1] + (N,))
    for idx in np.ndindex(*g.shape[:-1]):
        line = g[idx]
        out[idx] = ko_line(line[ng:ng + N] if periodic else line, ng, h, r, sigma, periodic)
    return np.moveaxis(out, -1, ax)
