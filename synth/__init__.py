"""Seeded synthetic workloads shared by the GPU library's tests/benchmark and the oracle.

This module only samples analytic fields on block grids (ghost layers
included) and lays them out; it contains none of the compact finite-difference
arithmetic.  Every draw comes from ``numpy.random.default_rng(seed)``.

Workloads (shapes and structure follow the paper's test problems: sums of
plane waves on periodic grids, Sec. 2.1 and 3; smooth localized profiles plus
small-amplitude noise; uneven mesh blocks with ghost layers, Sec. 2.4):

* ``periodic32``  : periodic 32^3, h = 2 pi/32, one field, 8 modes, k in [1,12]^3.
* ``block128``    : one 128^3 block on [-1,1]^3 (cell-centred), Gaussian pulse
                    plus 64 noise modes with N(0, 1e-3^2) amplitudes, k in [0,40]^3.
* ``batch64``     : 64 blocks with extents drawn from {16,24,32,48}^3, h = 1/64,
                    origins uniform in [0,1)^3, 22 fields of 8 modes, k in [1,6]^3.
* ``periodic256`` : periodic 256^3, h = 2 pi/256, 8 fields of 32 modes, k in [1,120]^3.
* ``periodic_box``: small anisotropic periodic boxes (ragged line counts) for edge cases.
* ``lattice``     : a periodic box tiled by equal blocks with closures (ghosts sampled
                    from the same periodic field), for the hybrid closure iteration.
* ``wave192``     : periodic 192^3 plane wave k = (3,5,7) for the first-order wave
                    system (phi, Pi, psi_x, psi_y, psi_z), as one periodic block
                    or as a 4x4x4 lattice of 48^3 blocks.
* ``decomp_line`` : the paper's decomposition test functions g and h (Eqs.
                    test_grid_conv_g, test_grid_conv_h, with the parameters of the
                    decomposition study) on a periodic [0, 2 pi) line of N_M
                    cell-centred samples, split into blocks of N_B with ghosts.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

CLOSURE = 0
PERIODIC = 1


@dataclass
class Block:
    n: Tuple[int, int, int]            # interior extents (nx, ny, nz)
    ng: int                            # ghost layers per side
    h: Tuple[float, float, float]
    boundary: Tuple[int, int, int]     # CLOSURE / PERIODIC per direction
    origin: Tuple[float, float, float]  # coordinate of interior node 0 along each axis

    def padded(self) -> Tuple[int, int, int]:
        return tuple(n + 2 * self.ng for n in self.n)

    def coords(self, axis: int) -> np.ndarray:
        """Coordinates of nodes -ng .. n+ng-1 along ``axis``."""
        i = np.arange(-self.ng, self.n[axis] + self.ng, dtype=np.float64)
        return self.origin[axis] + i * self.h[axis]


@dataclass
class Modes:
    """f(x) = sum_j A_j sin(scale * k_j . x + phi_j)."""

    A: np.ndarray        # (J,)
    k: np.ndarray        # (J, 3) integers
    phi: np.ndarray      # (J,)
    scale: float = 1.0


@dataclass
class Workload:
    name: str
    blocks: List[Block]
    nfields: int
    data: np.ndarray                      # flat, [block][field][z][y][x] with ghosts
    in_offsets: List[int]
    modes: List[List[Modes]] = field(default_factory=list)   # per field, list of mode sets
    gauss: Optional[Tuple[Tuple[float, float, float], float]] = None   # (x0, sigma) for block128

    def field_view(self, b: int, f: int) -> np.ndarray:
        blk = self.blocks[b]
        PX, PY, PZ = blk.padded()
        n = PX * PY * PZ
        off = self.in_offsets[b] + f * n
        return self.data[off:off + n].reshape(PZ, PY, PX)

    @property
    def interior_points(self) -> int:
        return int(sum(np.prod(b.n) for b in self.blocks))


def packed_offsets(blocks: Sequence[Block], nfields: int) -> Tuple[List[int], int]:
    offs, cur = [], 0
    for b in blocks:
        offs.append(cur)
        cur += nfields * int(np.prod(b.padded()))
    return offs, cur


def eval_modes(m: Modes, x: np.ndarray, y: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Sum of plane waves on the tensor grid (z, y, x), via two real matmuls."""
    s = m.scale
    ax = s * m.k[:, 0:1] * x[None, :]            # (J, X)
    ay = s * m.k[:, 1:2] * y[None, :]            # (J, Y)
    az = s * m.k[:, 2:3] * z[None, :] + m.phi[:, None]   # (J, Z)
    axy = ay[:, :, None] + ax[:, None, :]        # (J, Y, X)
    J = m.A.size
    cxy = np.cos(axy).reshape(J, -1)
    sxy = np.sin(axy).reshape(J, -1)
    sz = (m.A[:, None] * np.sin(az)).T           # (Z, J)
    cz = (m.A[:, None] * np.cos(az)).T
    f = sz @ cxy + cz @ sxy                      # (Z, Y*X)
    return f.reshape(z.size, y.size, x.size)


def _fill(blocks, nfields, fill_fn):
    offs, total = packed_offsets(blocks, nfields)
    data = np.empty(total, dtype=np.float64)
    for b, blk in enumerate(blocks):
        x, y, z = blk.coords(0), blk.coords(1), blk.coords(2)
        PX, PY, PZ = blk.padded()
        n = PX * PY * PZ
        for f in range(nfields):
            data[offs[b] + f * n: offs[b] + (f + 1) * n] = fill_fn(b, f, x, y, z).ravel()
    return data, offs


def _random_modes(rng, J, kmin, kmax, scale, amp="uniform", exclude_zero=False) -> Modes:
    k = rng.integers(kmin, kmax + 1, size=(J, 3))
    if exclude_zero:
        while True:
            zero = np.all(k == 0, axis=1)
            if not zero.any():
                break
            k[zero] = rng.integers(kmin, kmax + 1, size=(int(zero.sum()), 3))
    if amp == "uniform":
        A = rng.uniform(-1.0, 1.0, size=J)
    else:
        A = rng.normal(0.0, amp, size=J)
    phi = rng.uniform(0.0, 2 * np.pi, size=J)
    return Modes(A=A, k=k, phi=phi, scale=scale)


# ---------------------------------------------------------------------------

def periodic32(seed: int = 1, n: int = 32) -> Workload:
    rng = np.random.default_rng(seed)
    h = 2 * np.pi / n
    blk = Block((n, n, n), 0, (h, h, h), (PERIODIC,) * 3, (0.0, 0.0, 0.0))
    m = _random_modes(rng, 8, 1, 12, 1.0)
    data, offs = _fill([blk], 1, lambda b, f, x, y, z: eval_modes(m, x, y, z))
    return Workload("periodic32", [blk], 1, data, offs, [[m]])


def block128(seed: int = 2, n: int = 128, ng: int = 4) -> Workload:
    rng = np.random.default_rng(seed)
    h = 2.0 / n
    origin = -1.0 + 0.5 * h                      # cell-centred on [-1, 1]
    blk = Block((n, n, n), ng, (h, h, h), (CLOSURE,) * 3, (origin,) * 3)
    x0 = (0.05, -0.03, 0.02)
    sigma = 0.2
    noise = _random_modes(rng, 64, 0, 40, np.pi, amp=1e-3, exclude_zero=True)

    def fill(b, f, x, y, z):
        gx = np.exp(-(x - x0[0]) ** 2 / (2 * sigma ** 2))
        gy = np.exp(-(y - x0[1]) ** 2 / (2 * sigma ** 2))
        gz = np.exp(-(z - x0[2]) ** 2 / (2 * sigma ** 2))
        return gz[:, None, None] * gy[None, :, None] * gx[None, None, :] + eval_modes(noise, x, y, z)

    data, offs = _fill([blk], 1, fill)
    return Workload("block128", [blk], 1, data, offs, [[noise]], gauss=(x0, sigma))


def batch64(seed: int = 3, nblocks: int = 64, nfields: int = 22, ng: int = 5,
            sizes=(16, 24, 32, 48), h: float = 1.0 / 64) -> Workload:
    rng = np.random.default_rng(seed)
    ext = rng.choice(np.array(sizes), size=(nblocks, 3))
    origins = rng.uniform(0.0, 1.0, size=(nblocks, 3))
    modes = [_random_modes(rng, 8, 1, 6, 2 * np.pi) for _ in range(nfields)]
    blocks = [Block(tuple(int(v) for v in ext[b]), ng, (h, h, h), (CLOSURE,) * 3,
                    tuple(float(origins[b, d] + 0.5 * h) for d in range(3))) for b in range(nblocks)]
    data, offs = _fill(blocks, nfields, lambda b, f, x, y, z: eval_modes(modes[f], x, y, z))
    return Workload("batch64", blocks, nfields, data, offs, [[m] for m in modes])


def periodic256(seed: int = 4, n: int = 256, nfields: int = 8, nmodes: int = 32, kmax: int = 120) -> Workload:
    rng = np.random.default_rng(seed)
    h = 2 * np.pi / n
    blk = Block((n, n, n), 0, (h, h, h), (PERIODIC,) * 3, (0.0, 0.0, 0.0))
    modes = [_random_modes(rng, nmodes, 1, kmax, 1.0) for _ in range(nfields)]
    data, offs = _fill([blk], nfields, lambda b, f, x, y, z: eval_modes(modes[f], x, y, z))
    return Workload("periodic256", [blk], nfields, data, offs, [[m] for m in modes])


def periodic_box(seed: int = 6, n=(64, 5, 7), nfields: int = 2, nmodes: int = 16, kmax: int = 20) -> Workload:
    """Anisotropic periodic box [0, 2 pi)^3 with n[d] nodes along axis d (no ghosts)."""
    rng = np.random.default_rng(seed)
    h = tuple(2 * np.pi / v for v in n)
    blk = Block(tuple(int(v) for v in n), 0, h, (PERIODIC,) * 3, (0.0, 0.0, 0.0))
    modes = [_random_modes(rng, nmodes, 0, kmax, 1.0, exclude_zero=True) for _ in range(nfields)]
    for m in modes:      # keep every mode resolved on the coarsest axis
        m.k = np.minimum(m.k, np.array([max(0, v // 2 - 1) for v in n]))
    data, offs = _fill([blk], nfields, lambda b, f, x, y, z: eval_modes(modes[f], x, y, z))
    return Workload("periodic_box", [blk], nfields, data, offs, [[m] for m in modes])


def lattice(n=(16, 16, 16), lat=(3, 2, 2), ng: int = 4, nfields: int = 2, nmodes: int = 12, kmax: int = 6,
            seed: int = 8) -> Workload:
    """A periodic box [0, 2 pi)^3 tiled by lat[0] x lat[1] x lat[2] equal blocks of n interior nodes
    (block index (kz*lat[1] + ky)*lat[0] + kx), cell-centred, with closures on every face; each field is
    one sum of plane waves sampled on every block including its ghosts, so the ghosts equal the
    neighbouring blocks' interior values."""
    rng = np.random.default_rng(seed)
    NG = [n[d] * lat[d] for d in range(3)]
    h = tuple(2 * np.pi / v for v in NG)
    modes = [_random_modes(rng, nmodes, 0, kmax, 1.0, exclude_zero=True) for _ in range(nfields)]
    blocks = []
    for kz in range(lat[2]):
        for ky in range(lat[1]):
            for kx in range(lat[0]):
                org = tuple((k * n[d] + 0.5) * h[d] for d, k in enumerate((kx, ky, kz)))
                blocks.append(Block(tuple(n), ng, h, (CLOSURE,) * 3, org))
    data, offs = _fill(blocks, nfields, lambda b, f, x, y, z: eval_modes(modes[f], x, y, z))
    return Workload("lattice", blocks, nfields, data, offs, [[m] for m in modes])


WAVE_K = (3, 5, 7)


def wave_state(x, y, z, t: float, k=WAVE_K) -> List[np.ndarray]:
    """Exact plane wave of the first-order wave system at time t:
    phi = sin(k.x - w t), Pi = -w cos(k.x - w t), psi_i = k_i cos(k.x - w t), w = |k|."""
    w = float(np.sqrt(sum(v * v for v in k)))
    ph = Modes(np.array([1.0]), np.array([k]), np.array([-w * t]))
    co = Modes(np.array([1.0]), np.array([k]), np.array([-w * t + np.pi / 2]))
    s = eval_modes(ph, x, y, z)
    c = eval_modes(co, x, y, z)
    return [s, -w * c, k[0] * c, k[1] * c, k[2] * c]


def wave192(n: int = 192, blocks_per_dim: int = 1, ng: int = 4) -> Workload:
    """Initial data of the wave test: 5 fields (phi, Pi, psi_x, psi_y, psi_z)."""
    h = 2 * np.pi / n
    if blocks_per_dim == 1:
        blocks = [Block((n, n, n), 0, (h, h, h), (PERIODIC,) * 3, (0.0, 0.0, 0.0))]
    else:
        nb = n // blocks_per_dim
        blocks = []
        for kz in range(blocks_per_dim):
            for ky in range(blocks_per_dim):
                for kx in range(blocks_per_dim):
                    blocks.append(Block((nb, nb, nb), ng, (h, h, h), (CLOSURE,) * 3,
                                        (kx * nb * h, ky * nb * h, kz * nb * h)))
    cache = {}

    def fill(b, f, x, y, z):
        if b not in cache:
            cache.clear()
            cache[b] = wave_state(x, y, z, 0.0)
        return cache[b][f]

    data, offs = _fill(blocks, 5, fill)
    return Workload(f"wave{n}", blocks, 5, data, offs)


def paper_g(x, A=0.05, S=1.0, N1=2, x0=0.2):
    """g of Eq. test_grid_conv_g, with the parameters of the first-degree decomposition study."""
    return A * np.exp(-S * np.sin(N1 * (np.asarray(x) - x0)))


def paper_h(x, S=3.0, x0=np.pi, N1=5, N2=11, phiS=3.0, c1=1.2, c2=-1.0):
    """h of Eq. test_grid_conv_h, with the parameters of the second-degree decomposition study (on
    [0, 2 pi) its Gaussian factor is below 2e-13 at the ends, so its samples are periodic to that)."""
    x = np.asarray(x)
    return np.exp(-S * (x - x0) ** 2) * (c1 * np.sin(N2 * x) + c2 * np.cos(N2 * x)) + np.sin(N1 * x - phiS)


def decomp_line(fn, NM: int = 128, NB: int = 16, ng: int = 4, ny: int = 1, nz: int = 1) -> Workload:
    """fn sampled cell-centred on a periodic [0, 2 pi) line of NM nodes (node j at (j + 1/2) 2 pi/NM, Eq.
    gridDisc), as NM/NB blocks of NB x ny x nz interior nodes along x (closures on every face, the value
    constant along y and z), ghosts sampled from the same periodic function (the exact exchange)."""
    NS = NM // NB
    h = 2 * np.pi / NM
    blocks = [Block((NB, ny, nz), ng, (h, h, h), (CLOSURE,) * 3, ((I * NB + 0.5) * h, 0.0, 0.0)) for I in range(NS)]

    def fill(b, f, x, y, z):
        row = fn(np.mod(x, 2 * np.pi))
        return np.broadcast_to(row[None, None, :], (z.size, y.size, x.size)).copy()

    data, offs = _fill(blocks, 1, fill)
    return Workload("decomp_line", blocks, 1, data, offs)
