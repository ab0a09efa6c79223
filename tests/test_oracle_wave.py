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
