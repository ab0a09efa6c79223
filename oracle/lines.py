"""Oracle FP64 line operator (ctypes front end of ``oracle/lines.c``).

TEST INFRASTRUCTURE ONLY.  The block-closure system of Eq. sch_cent_om and
the periodic (circulant) system, solved line by line in plain C.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import build as _build
from .schemes import Scheme, required_ghosts

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_line.restype = ctypes.c_int
        L.orc_line.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               ctypes.c_int, _dp, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
        L.orc_block_dir.restype = ctypes.c_int
        L.orc_block_dir.argtypes = [ctypes.c_int] * 6 + [ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp,
                                                          ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, _dp,
                                                          _dp, _dp, ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _arr(v):
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    return a, a.ctypes.data_as(_dp)


class _Coefs:
    """FP64 views of a scheme's coefficient tuples, kept alive for the C call."""

    def __init__(self, s: Scheme):
        self.d = s.dr
        self.nl = s.nl
        self.M = s.M
        self.alpha, self.p_alpha = _arr(s.lhs_floats())
        self.a, self.p_a = _arr(s.rhs_floats())
        mc, rows = s.closure_floats()
        self.nc = len(rows) if s.nl > 0 else 0
        self.mc = mc
        self.cbar, self.p_cbar = _arr(np.array(rows, dtype=np.float64).ravel() if rows else [0.0])


def check_ghosts(s: Scheme, ng: int, periodic: bool):
    need = required_ghosts(s, periodic)
    if ng < need:
        raise ValueError(f"{s.name}: {ng} ghost layers given, {need} needed")


def apply_line(s: Scheme, g, ng: int, h: float, periodic: bool = False) -> np.ndarray:
    """Derivative on the N interior nodes of one line; g holds N + 2 ng values."""
    check_ghosts(s, ng, periodic)
    c = _Coefs(s)
    g, pg = _arr(g)
    N = g.size - 2 * ng
    x = np.empty(N)
    rc = lib().orc_line(N, ng, int(periodic), c.d, float(h), c.nl, c.p_alpha, c.M, c.p_a,
                        c.nc, c.mc, c.p_cbar, pg, x.ctypes.data_as(_dp))
    if rc:
        raise RuntimeError(f"orc_line failed ({rc})")
    return x


def apply_block(s: Scheme, f, ng: int, h: float, direction: int, periodic: bool = False,
                nthreads: int = 0, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Derivative along ``direction`` (0=x, 1=y, 2=z) of one block-field.

    ``f`` is [z][y][x] with ng ghost layers on every side; the result is the
    interior [z][y][x].
    """
    check_ghosts(s, ng, periodic)
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx = (e - 2 * ng for e in f.shape)
    n = (nx, ny, nz)
    nc = len(s.closure) if s.nl > 0 else 0
    if not periodic and n[direction] < 2 * nc + 1:
        raise ValueError("line too short for the closure rows")
    c = _Coefs(s)
    if out is None:
        out = np.empty((nz, ny, nx))
    rc = lib().orc_block_dir(nx, ny, nz, ng, direction, int(periodic), c.d, float(h), c.nl, c.p_alpha,
                             c.M, c.p_a, c.nc, c.mc, c.p_cbar, f.ctypes.data_as(_dp),
                             out.ctypes.data_as(_dp), int(nthreads))
    if rc:
        raise RuntimeError(f"orc_block_dir failed ({rc})")
    return out


def max_threads() -> int:
    return lib().orc_max_threads()
