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
    """D_- along the last axis on samples of nodes lo, lo+1, ...: defined from node lo+1 on."""
    return (v[..., 1:] - v[..., :-1]) / h, lo + 1


def _dplus(v: np.ndarray, lo: int, h: float):
    """D_+ along the last axis on samples of nodes lo, lo+1, ...: defined up to the last node but one."""
    return (v[..., 1:] - v[..., :-1]) / h, lo


def _ko_lines(v: np.ndarray, N: int, h: float, r: int, sigma: float) -> np.ndarray:
    """Q^(2r) on lines stored along the last axis as nodes -r .. N+r-1."""
    lo = -r
    for _ in range(r):
        v, lo = _dminus(v, lo, h)
    for _ in range(r):
        v, lo = _dplus(v, lo, h)
    assert lo == 0 and v.shape[-1] == N, (lo, v.shape, N)
    return -((-1) ** r) / 2 ** (2 * r) * sigma * h ** (2 * r - 1) * v


def ko_line(g: np.ndarray, ng: int, h: float, r: int, sigma: float, periodic: bool = False) -> np.ndarray:
    """Q^(2r) f on the N interior nodes of one line; g holds N + 2 ng samples
    (g[ng + k] is node k), or just the N interior samples when periodic."""
    g = np.asarray(g, dtype=np.float64)
    if periodic:
        N = g.size
        return _ko_lines(g[np.arange(-r, N + r) % N], N, h, r, sigma)
    if ng < r:
        raise ValueError(f"Kreiss-Oliger of degree {2 * r} needs {r} ghost layers, line has {ng}")
    N = g.size - 2 * ng
    return _ko_lines(g[ng - r: ng + N + r], N, h, r, sigma)


def ko_block(f: np.ndarray, ng: int, h: float, direction: int, r: int, sigma: float,
             periodic: bool = False) -> np.ndarray:
    """Q^(2r) along ``direction`` (0=x, 1=y, 2=z) of one block-field [z][y][x] with ng
    ghosts on every side; returns the interior [z][y][x].  Every line of the block is
    differenced at once along the last axis."""
    f = np.asarray(f, dtype=np.float64)
    nz, ny, nx = (e - 2 * ng for e in f.shape)
    ax = 2 - direction
    g = np.moveaxis(f, ax, -1)
    sl = [slice(ng, ng + e) for e in (nz, ny, nx)]
    del sl[ax]
    g = g[tuple(sl)]
    N = (nx, ny, nz)[direction]
    if periodic:
        v = g[..., ng + (np.arange(-r, N + r) % N)]
    else:
        if ng < r:
            raise ValueError(f"Kreiss-Oliger of degree {2 * r} needs {r} ghost layers, block has {ng}")
        v = g[..., ng - r: ng + N + r]
    return np.moveaxis(_ko_lines(v, N, h, r, sigma), -1, ax)
