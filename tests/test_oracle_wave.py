"""Pins of the oracle's wave-system RK4 and ghost fill.

The closed form (one Fourier mode, 5x5 amplitude matrix, RK4 stability
polynomial) and the stepped RK4 over line solves are two independent routes to
the same fully discrete result; the ghost fill is checked against sampling the
periodic analytic field."""
import numpy as np
import pytest

import synth
from oracle import schemes as S
from oracle import wave as W


def _state_from(wl):
    return [[wl.field_view(b, f).copy() for f in range(5)] for b in range(len(wl.blocks))]


@pytest.mark.parametrize("name", ["(1)Q1_3[1]", "(1)P1_2"])
def test_rk4_periodic_matches_closed_form(name):
    s = S.named(name)
    n = 16
    wl = synth.wave192(n=n)
    h = wl.blocks[0].h[0]
    dt = 0.25 * h
    st = _state_from(wl)
    W.rk4_blocks(s, st, n, 0, h, dt, 3, periodic=True)
    amp = W.mode_evolution(s, synth.WAVE_K, h, dt, 3)
    x = np.arange(n) * h
    for f in range(5):
        ref = W.mode_field(amp[f], synth.WAVE_K, x, x, x)
        assert np.max(np.abs(st[0][f] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), f


def test_mode_evolution_phase_tracks_exact_wave():
    """Small dt: the discrete mode's phase speed follows the modified wavenumber, close to |k|."""
    s = S.named("(1)Q1_3[1]")
    n = 64
    h = 2 * np.pi / n
    amp = W.mode_evolution(s, synth.WAVE_K, h, 0.05 * h, 200)
    t = 200 * 0.05 * h
    w = np.sqrt(83.0)
    exact = -1j * np.exp(-1j * w * t)
    # k = 7 at h = 2 pi/64: relative wavenumber error ~ 5e-5 eta^6 ~ 6e-6, times w t ~ 9
    assert abs(np.angle(amp[0] / exact)) < 2e-4


def test_ghost_fill_equals_periodic_sampling():
    wl = synth.wave192(n=24, blocks_per_dim=2, ng=4)
    st = _state_from(wl)
    for blk in st:
        for a in blk:
            a[:4] = 0; a[-4:] = 0; a[:, :4] = 0; a[:, -4:] = 0; a[:, :, :4] = 0; a[:, :, -4:] = 0
    W.fill_ghosts(st, 12, 4, (2, 2, 2))
    for b, blk in enumerate(wl.blocks):
        ref = wl.field_view(b, 0)
        sl = slice(4, 16)
        for face in ((slice(0, 4), sl, sl), (slice(16, 20), sl, sl), (sl, slice(0, 4), sl),
                     (sl, slice(16, 20), sl), (sl, sl, slice(0, 4)), (sl, sl, slice(16, 20))):
            assert np.allclose(st[b][0][face], ref[face], atol=1e-13)


def _lattice_table(bx, by, bz):
    """Neighbour table of a periodic bx*by*bz lattice (block (kz by + ky) bx + kx)."""
    t = []
    for b in range(bx * by * bz):
        kx, ky, kz = b % bx, (b // bx) % by, b // (bx * by)
        idx = lambda x, y, z: ((z % bz) * by + (y % by)) * bx + (x % bx)
        t.append([idx(kx - 1, ky, kz), idx(kx + 1, ky, kz), idx(kx, ky - 1, kz), idx(kx, ky + 1, kz),
                  idx(kx, ky, kz - 1), idx(kx, ky, kz + 1)])
    return t


def test_ghost_fill_table_equals_lattice_fill():
    """The table form with a lattice's table is the lattice form, exactly."""
    wl = synth.wave192(n=24, blocks_per_dim=2, ng=4)
    a, b = _state_from(wl), _state_from(wl)
    rng = np.random.default_rng(3)
    for blk in a:
        for x in blk:
            x[...] = rng.standard_normal(x.shape)
    b = [[x.copy() for x in blk] for blk in a]
    W.fill_ghosts(a, 12, 4, (2, 2, 2))
    W.fill_ghosts_table(b, 4, _lattice_table(2, 2, 2))
    for ba, bb in zip(a, b):
        for xa, xb in zip(ba, bb):
            assert np.array_equal(xa, xb)


def test_ghost_fill_table_samples_a_periodic_function_on_an_uneven_tiling():
    """Three blocks of 12, 20 and 8 nodes along x tile a periodic interval (y and z: each block its own
    neighbour, periodic); after the fill every face ghost holds the function at its position, and the
    faces marked -1 keep their old values."""
    ng, ny, nz, h = 4, 10, 6, 0.1
    nxs = [12, 20, 8]
    X = sum(nxs) * h
    x0 = np.cumsum([0] + nxs[:-1]) * h

    def f(x, y, z):
        return np.sin(2 * np.pi * x / X) + np.cos(2 * np.pi * y / (ny * h)) + np.sin(4 * np.pi * z / (nz * h))

    st, ref = [], []
    for b, nx in enumerate(nxs):
        xs = x0[b] + (np.arange(nx + 2 * ng) - ng) * h
        ys = (np.arange(ny + 2 * ng) - ng) * h
        zs = (np.arange(nz + 2 * ng) - ng) * h
        full = f(xs[None, None, :], ys[None, :, None], zs[:, None, None])
        ref.append(full)
        a = np.full_like(full, -7.0)
        a[ng:-ng, ng:-ng, ng:-ng] = full[ng:-ng, ng:-ng, ng:-ng]
        st.append([a])
    table = [[2, 1, 0, 0, 0, 0], [0, 2, 1, 1, -1, -1], [1, 0, 2, 2, 2, 2]]
    W.fill_ghosts_table(st, ng, table)
    sl = slice(ng, -ng)
    for b in range(3):
        a, r = st[b][0], ref[b]
        faces = [(sl, sl, slice(0, ng)), (sl, sl, slice(-ng, None)), (sl, slice(0, ng), sl),
                 (sl, slice(-ng, None), sl), (slice(0, ng), sl, sl), (slice(-ng, None), sl, sl)]
        for face, region in enumerate(faces):
            if table[b][face] < 0:
                assert np.all(a[region] == -7.0)
            else:
                assert np.allclose(a[region], r[region], atol=1e-12), (b, face)
        assert a[0, 0, 0] == -7.0            # corners untouched


def test_vertex_centred_ghost_fill_samples_the_function():
    """Vertex-centred blocks (N_B + 1 nodes, the extremal node shared with the neighbour, Eq. gridDisc):
    after the shared fill every face ghost holds the function at its position (the shared node is not
    repeated)."""
    ng, h = 3, 0.1
    nbs = [10, 6, 8]                    # cells per block along x: nodes = N_B + 1
    ny, nz = 7, 5                       # y, z: one VC block periodic onto itself (N_B = n - 1 cells)
    X = sum(nbs) * h
    x0 = np.cumsum([0] + nbs[:-1]) * h
    Y, Z = (ny - 1) * h, (nz - 1) * h

    def f(x, y, z):
        return np.sin(2 * np.pi * x / X) * np.cos(2 * np.pi * y / Y) + np.sin(2 * np.pi * z / Z)

    st, ref = [], []
    for b, nb in enumerate(nbs):
        xs = x0[b] + (np.arange(nb + 1 + 2 * ng) - ng) * h
        ys = (np.arange(ny + 2 * ng) - ng) * h
        zs = (np.arange(nz + 2 * ng) - ng) * h
        full = f(xs[None, None, :], ys[None, :, None], zs[:, None, None])
        ref.append(full)
        a = np.full_like(full, 5.0)
        a[ng:-ng, ng:-ng, ng:-ng] = full[ng:-ng, ng:-ng, ng:-ng]
        st.append([a])
    table = [[2, 1, 0, 0, 0, 0], [0, 2, 1, 1, 1, 1], [1, 0, 2, 2, 2, 2]]
    W.fill_ghosts_table(st, ng, table, shared=1)
    sl = slice(ng, -ng)
    for b in range(3):
        a, r = st[b][0], ref[b]
        for region in [(sl, sl, slice(0, ng)), (sl, sl, slice(-ng, None)), (sl, slice(0, ng), sl),
                       (sl, slice(-ng, None), sl), (slice(0, ng), sl, sl), (slice(-ng, None), sl, sl)]:
            assert np.allclose(a[region], r[region], atol=1e-12), b


def test_shared_node_average_means_every_copy():
    """A node shared by 2, 4 or 8 vertex-centred blocks ends with the mean of all its copies (the x, y,
    z sweeps compose to it), interior nodes are untouched, and a second pass changes nothing."""
    rng = np.random.default_rng(4)
    n = 5
    # 2 x 2 x 2 periodic lattice of VC blocks, interior-only arrays (ng = 0)
    blocks = [[rng.standard_normal((n, n, n))] for _ in range(8)]
    orig = [[a.copy() for a in blk] for blk in blocks]
    idx = lambda x, y, z: ((z % 2) * 2 + (y % 2)) * 2 + (x % 2)
    table = []
    for b in range(8):
        kx, ky, kz = b % 2, (b // 2) % 2, b // 4
        table.append([idx(kx - 1, ky, kz), idx(kx + 1, ky, kz), idx(kx, ky - 1, kz), idx(kx, ky + 1, kz),
                      idx(kx, ky, kz - 1), idx(kx, ky, kz + 1)])
    W.shared_node_average(blocks, 0, table)
    # global node coordinates: block (kx, ky, kz) node (i, j, k) sits at (kx (n-1) + i, ...) mod 2 (n-1)
    M = 2 * (n - 1)
    copies = {}
    for b in range(8):
        kx, ky, kz = b % 2, (b // 2) % 2, b // 4
        for k in range(n):
            for j in range(n):
                for i in range(n):
                    key = ((kx * (n - 1) + i) % M, (ky * (n - 1) + j) % M, (kz * (n - 1) + k) % M)
                    copies.setdefault(key, []).append((orig[b][0][k, j, i], blocks[b][0][k, j, i]))
    mult = set()
    for key, cs in copies.items():
        mean = np.mean([c[0] for c in cs])
        mult.add(len(cs))
        for _, new in cs:
            assert abs(new - mean) <= 1e-14 * max(1.0, abs(mean)), (key, len(cs))
    assert mult == {1, 2, 4, 8}
    again = [[a.copy() for a in blk] for blk in blocks]
    W.shared_node_average(again, 0, table)
    for x, y in zip(blocks, again):
        assert np.array_equal(x[0], y[0])
