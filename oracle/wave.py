"""Oracle for the first-order wave system under classical RK4.

TEST INFRASTRUCTURE ONLY.

* ``mode_evolution``: the fully discrete evolution of one Fourier mode on a
  periodic grid in closed form.  A compact operator acts on exp(i k.x) as
  multiplication by i kappa_j with kappa_j = eta~(k_j h)/h (Eq. fdpwerrdef), so
  the semi-discrete system for the five complex amplitudes is a 5x5 matrix
  Lhat and one RK4 step multiplies by the stability polynomial
  R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 at z = dt Lhat (classical ERK4).
* ``rk4_blocks``: plain RK4 on a periodic lattice of blocks with ghost layers
  filled from the neighbours before every derivative (the communication step
  of Sec. 2.4) and the block-closure line operator of ``oracle.lines``.
"""
from __future__ import annotations

import numpy as np

from . import lines as L
from .schemes import Scheme, modified_wavenumber_power


def kappa(s: Scheme, k: int, h: float) -> float:
    """Discrete wavenumber of the first-derivative scheme for integer k."""
    lam = complex(modified_wavenumber_power(s, k * h))   # i eta~
    return lam.imag / h


def mode_evolution(s: Scheme, k, h: float, dt: float, nsteps: int) -> np.ndarray:
    """Complex amplitudes (phi, Pi, psi_x, psi_y, psi_z) after nsteps, starting
    from phi = sin(k.x), Pi = -w cos(k.x), psi_j = k_j cos(k.x), w = |k|."""
    w = float(np.sqrt(sum(v * v for v in k)))
    kx, ky, kz = (kappa(s, kj, h) for kj in k)
    Lh = np.zeros((5, 5), dtype=complex)
    Lh[0, 1] = 1.0
    Lh[1, 2], Lh[1, 3], Lh[1, 4] = 1j * kx, 1j * ky, 1j * kz
    Lh[2, 1], Lh[3, 1], Lh[4, 1] = 1j * kx, 1j * ky, 1j * kz
    z = dt * Lh
    I = np.eye(5)
    R = I + z + z @ z / 2 + z @ z @ z / 6 + z @ z @ z @ z / 24
    u0 = np.array([-1j, -w, k[0], k[1], k[2]], dtype=complex)
    return np.linalg.matrix_power(R, nsteps) @ u0


def mode_field(amp: complex, k, x, y, z) -> np.ndarray:
    """Re(amp * exp(i k.x)) on the tensor grid (z, y, x)."""
    ph = k[0] * x[None, None, :] + k[1] * y[None, :, None] + k[2] * z[:, None, None]
    return np.real(amp * np.exp(1j * ph))


def fill_ghosts(state, nb, ng, lattice):
    """state[b][f] arrays with ghosts; copy face ghosts from lattice neighbours (periodic)."""
    bx, by, bz = lattice
    for b in range(len(state)):
        kx, ky, kz = b % bx, (b // bx) % by, b // (bx * by)
        for f in range(len(state[b])):
            a = state[b][f]
            sl = slice(ng, ng + nb)
            xm = state[(kz * by + ky) * bx + (kx - 1) % bx][f]
            xp = state[(kz * by + ky) * bx + (kx + 1) % bx][f]
            a[sl, sl, :ng] = xm[sl, sl, nb:nb + ng]
            a[sl, sl, ng + nb:] = xp[sl, sl, ng:2 * ng]
            ym = state[(kz * by + (ky - 1) % by) * bx + kx][f]
            yp = state[(kz * by + (ky + 1) % by) * bx + kx][f]
            a[sl, :ng, sl] = ym[sl, nb:nb + ng, sl]
            a[sl, ng + nb:, sl] = yp[sl, ng:2 * ng, sl]
            zm = state[(((kz - 1) % bz) * by + ky) * bx + kx][f]
            zp = state[(((kz + 1) % bz) * by + ky) * bx + kx][f]
            a[:ng, sl, sl] = zm[nb:nb + ng, sl, sl]
            a[ng + nb:, sl, sl] = zp[ng:2 * ng, sl, sl]


def fill_ghosts_table(state, ng, nbr, shared=0):
    """Face ghosts by a neighbour table (Sec. 2.4: a block's ghost layers hold its neighbours' data).

    state[b][f]: arrays [z][y][x] with ng ghosts on every side (blocks may differ in extent);
    nbr[b][face] = block across face (x-, x+, y-, y+, z-, z+) or -1 (ghosts left as they are).
    Ghost layer l of the + face is the neighbour's interior layer l, of the - face its layer n - ng + l,
    at the same coordinates along the face; edges and corners are not touched.  Reads are taken from a
    copy made before any write, so a block may be its own neighbour.

    shared = 1: vertex-centred sampling (Eq. gridDisc, G_VC): neighbouring blocks share their extremal
    node, so the ghost layers continue past it: layer l of the + face is the neighbour's node 1 + l, of
    the - face its node n - 1 - ng + l."""
    src = [[a.copy() for a in blk] for blk in state]
    for b in range(len(state)):
        for face in range(6):
            q = nbr[b][face]
            if q < 0:
                continue
            d, side = face // 2, face % 2
            ax = 2 - d                          # array axis of direction d
            for f in range(len(state[b])):
                a, s_ = state[b][f], src[q][f]
                n_a = a.shape[ax] - 2 * ng
                n_q = s_.shape[ax] - 2 * ng
                idx_a = [slice(ng, a.shape[k] - ng) for k in range(3)]
                idx_s = [slice(ng, s_.shape[k] - ng) for k in range(3)]
                if side:
                    idx_a[ax] = slice(ng + n_a, 2 * ng + n_a)
                    idx_s[ax] = slice(ng + shared, 2 * ng + shared)
                else:
                    idx_a[ax] = slice(0, ng)
                    idx_s[ax] = slice(n_q - shared, n_q + ng - shared)
                a[tuple(idx_a)] = s_[tuple(idx_s)]


def shared_node_average(blocks, ng, nbr):
    """Vertex-centred tilings (Eq. gridDisc, G_VC; the averaging of shared nodes the sampling figure and
    the communication matrix's footnote call for): block b's last node along d and its + neighbour's
    first node are one point; both get the mean of the two values.  Directions x, y, z in turn, so a
    node shared by 4 (edge) or 8 (corner) blocks ends with the mean of all its copies.

    blocks[b]: list of arrays [z][y][x] with ng ghost layers on every side (ng = 0 for interior-only
    outputs); averaged in place over the face's interior nodes."""
    for d in range(3):
        ax = 2 - d
        for b in range(len(blocks)):
            q = nbr[b][2 * d + 1]
            if q < 0:
                continue
            for a, c in zip(blocks[b], blocks[q]):
                n_a = a.shape[ax] - 2 * ng
                ia = [slice(ng, a.shape[k] - ng) for k in range(3)]
                ic = [slice(ng, c.shape[k] - ng) for k in range(3)]
                ia[ax] = ng + n_a - 1
                ic[ax] = ng
                m = 0.5 * (a[tuple(ia)] + c[tuple(ic)])
                a[tuple(ia)] = m
                c[tuple(ic)] = m


def rhs_blocks(s: Scheme, state, nb, ng, h, periodic):
    out = []
    for b in range(len(state)):
        phi, Pi, px, py, pz = state[b]
        d = [L.apply_block(s, Pi, ng, h, 0, periodic), L.apply_block(s, Pi, ng, h, 1, periodic),
             L.apply_block(s, Pi, ng, h, 2, periodic)]
        div = (L.apply_block(s, px, ng, h, 0, periodic) + L.apply_block(s, py, ng, h, 1, periodic) +
               L.apply_block(s, pz, ng, h, 2, periodic))
        sl = (slice(ng, ng + nb),) * 3
        out.append([Pi[sl].copy(), div, d[0], d[1], d[2]])
    return out


def rk4_blocks(s: Scheme, state, nb, ng, h, dt, nsteps, lattice=None, periodic=False):
    """RK4 on blocks; state[b][f] includes ghosts and is advanced in place."""
    sl = (slice(ng, ng + nb),) * 3
    for _ in range(nsteps):
        if lattice:
            fill_ghosts(state, nb, ng, lattice)
        u0 = [[a.copy() for a in blk] for blk in state]
        acc = [[a[sl].copy() for a in blk] for blk in state]
        cur = state
        for a_c, b_c in ((dt / 2, dt / 6), (dt / 2, dt / 3), (dt, dt / 3), (None, dt / 6)):
            k = rhs_blocks(s, cur, nb, ng, h, periodic)
            for bi in range(len(state)):
                for f in range(5):
                    acc[bi][f] += b_c * k[bi][f]
            if a_c is not None:
                nxt = [[a.copy() for a in blk] for blk in u0]
                for bi in range(len(state)):
                    for f in range(5):
                        nxt[bi][f][sl] = u0[bi][f][sl] + a_c * k[bi][f]
                if lattice:
                    fill_ghosts(nxt, nb, ng, lattice)
                cur = nxt
        for bi in range(len(state)):
            for f in range(5):
                state[bi][f][sl] = acc[bi][f]
    if lattice:
        fill_ghosts(state, nb, ng, lattice)
    return state
