"""Oracle: symmetrised mixed second derivatives, written from the paper.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import this
module; only ``tests/`` uses it.

Sec. ssec:z4c of arXiv 2302.14858: for i != j the mixed derivative is taken
as 1/2 (D_i[D_j[f]] + D_j[D_i[f]]) with D the first-degree compact operator
(block closure or periodic) of the scheme; for i = j the second-degree scheme
is used directly (that case is the ordinary operator, oracle.lines).

Reading: on a block with closures, D_i needs the values of D_j f on the N_g
ghost layers along i.  They are the operator D_j applied to the lines along j
that run through those ghost layers (the block's stored samples, edges
included), so the composition is taken on the block's own data: D_j f on the
block extended by N_g layers along i (interior along the other directions),
then D_i of that on the interior.  Along a periodic direction no extension is
needed (its lines wrap).
"""
from __future__ import annotations

import numpy as np

from . import lines as OL
from .schemes import Scheme


def _axis(direction: int) -> int:
    return 2 - direction   # arrays are [z][y][x]


def first_then(s: Scheme, f: np.ndarray, ng: int, h, periodic, dj: int, di: int) -> np.ndarray:
    """D_di[D_dj[f]] on the interior of one block-field f [z][y][x] (ng ghosts on every side).

    h and periodic are per direction (x, y, z)."""
    f = np.asarray(f, dtype=np.float64)
    ai, aj = _axis(di), _axis(dj)
    gi = 0 if periodic[di] else ng
    n_i = f.shape[ai] - 2 * ng
    # D_dj on the lines along dj through every node with i in [-gi, n_i + gi) and the third
    # direction interior: present those nodes to the block operator as its "interior" along i,
    # with ng zero layers either side (never read: these lines run along dj)
    ext = np.take(f, np.arange(ng - gi, ng + n_i + gi), axis=ai)
    pad = [(0, 0)] * 3
    pad[ai] = (ng, ng)
    fe = np.pad(ext, pad)
    g = OL.apply_block(s, fe, ng, h[dj], dj, periodic=bool(periodic[dj]))
    # g: [z][y][x] interior of fe: along i the extended range (n_i + 2 gi), others interior.
    # Re-pad to a block with ng ghosts on every side whose ghosts along i are the gi layers of g
    pad2 = [(ng, ng)] * 3
    pad2[ai] = (ng - gi, ng - gi)
    gp = np.pad(g, pad2)
    return OL.apply_block(s, gp, ng, h[di], di, periodic=bool(periodic[di]))


def mixed_block(s: Scheme, f: np.ndarray, ng: int, h, periodic, di: int, dj: int) -> np.ndarray:
    """1/2 (D_i[D_j f] + D_j[D_i f]) on the interior [z][y][x]."""
    if di == dj:
        raise ValueError("mixed derivative needs two different directions")
    return 0.5 * (first_then(s, f, ng, h, periodic, dj, di) + first_then(s, f, ng, h, periodic, di, dj))
