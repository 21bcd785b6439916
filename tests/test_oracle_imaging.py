"""Pins for the imaging oracle (Sec. 8.1: gridding, inversion, Hogbom CLEAN)
from outside it: hand-worked gridding, the Hermitian symmetry the mirrors
fix, the inversion as a direct double sum, point sources that must land on
their pixels with unit peak, and CLEAN's closed forms (a lone source
through its own beam: geometric decay (1 - g)^k, total flux, one component
at gain 1)."""

import numpy as np
import pytest

from oracle import imaging

RNG = np.random.default_rng(2024)


def test_gridding_by_hand():
    """n = 8, cell such that du = 10 wavelengths: u = 23 -> floor(2.3 + .5)
    = 2 -> cell 6; v = -14.9 -> floor(-1.49 + .5) = -1 -> cell 3; mirror
    cells 8 - 6 = 2 and 8 - 3 = 5.  u = 45 -> cell 4 + 5 = 9 is outside."""
    n = 8
    cell = 1.0 / (n * 10.0)
    u = np.array([23.0, 45.0], np.float32)
    v = np.array([-14.9, 0.0], np.float32)
    vis = np.array([2 + 3j, 7.0])
    G, W = imaging.grid_nearest(u, v, vis, None, n, cell)
    assert W == 2.0
    assert G[6, 3] == 2 + 3j and G[2, 5] == 2 - 3j
    assert np.count_nonzero(G) == 2


def test_grid_is_hermitian_and_image_is_real():
    n = 32
    cell = 1e-3
    du = 1.0 / (n * cell)
    u = RNG.uniform(-14 * du, 14 * du, 500).astype(np.float32)
    v = RNG.uniform(-14 * du, 14 * du, 500).astype(np.float32)
    vis = RNG.normal(size=500) + 1j * RNG.normal(size=500)
    G, W = imaging.grid_nearest(u, v, vis, RNG.uniform(0.5, 2, 500), n, cell)
    a = np.arange(1, n)
    assert np.allclose(G[np.ix_(a, a)], np.conj(G[np.ix_(n - a, n - a)]), atol=1e-12)
    # the complex image's imaginary part vanishes: check through the direct sum
    c = np.arange(n) - n // 2
    E = np.exp(2j * np.pi * np.outer(c, c) / n)
    full = E.T @ G @ E
    assert np.max(np.abs(full.imag)) < 1e-9 * np.max(np.abs(full.real))


@pytest.mark.parametrize("n", [8, 16, 32])
def test_invert_equals_direct_double_sum(n):
    G = RNG.normal(size=(n, n)) + 1j * RNG.normal(size=(n, n))
    assert np.allclose(imaging.invert(G, 3.5), imaging.invert_direct(G, 3.5), rtol=0, atol=1e-10)


def _cell_centred_uv(n, cell, k):
    """k (u, v) samples exactly on cell centres (|index| < n/2 - 1)."""
    du = 1.0 / (n * cell)
    iu = RNG.integers(-(n // 2) + 2, n // 2 - 1, k)
    iv = RNG.integers(-(n // 2) + 2, n // 2 - 1, k)
    return (iu * du).astype(np.float32), (iv * du).astype(np.float32)


def test_point_source_at_centre_is_the_beam_with_unit_peak():
    n, cell = 64, 2e-3
    u, v = _cell_centred_uv(n, cell, 300)
    vis = imaging.point_source_vis(u, v, [(1.0, 0.0, 0.0)])
    D, P = imaging.dirty_and_psf(u, v, vis, None, n, cell)
    assert np.allclose(D, P, atol=1e-12)
    assert np.unravel_index(np.argmax(P), P.shape) == (n // 2, n // 2)
    assert P[n // 2, n // 2] == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("p,q", [(5, -3), (-7, 11), (0, 9)])
def test_point_source_on_a_pixel_lands_there(p, q):
    """With samples on cell centres, a source at pixel offset (p, q) gives
    the beam circularly shifted by (p, q), so its peak F sits on that pixel."""
    n, cell = 64, 2e-3
    u, v = _cell_centred_uv(n, cell, 400)
    F = 2.5
    vis = imaging.point_source_vis(u, v, [(F, p * cell, q * cell)])
    D, P = imaging.dirty_and_psf(u, v, vis, None, n, cell)
    assert np.allclose(D, F * np.roll(P, (p, q), axis=(0, 1)), atol=1e-9)
    assert np.unravel_index(np.argmax(D), D.shape) == (n // 2 + p, n // 2 + q)
    assert D[n // 2 + p, n // 2 + q] == pytest.approx(F, abs=1e-9)


@pytest.mark.parametrize("gain", [0.1, 0.3])
def test_clean_lone_source_decays_geometrically(gain):
    """A lone source at the centre through its own beam: every component
    sits on the centre with flux F g (1-g)^i, and the residual's central
    value after k components is F (1-g)^k (float32 arithmetic)."""
    n, cell = 32, 2e-3
    u, v = _cell_centred_uv(n, cell, 200)
    F = 3.0
    vis = imaging.point_source_vis(u, v, [(F, 0.0, 0.0)])
    D, P = imaging.dirty_and_psf(u, v, vis, None, n, cell)
    k = 12
    pix, flux, R = imaging.hogbom(D, P, gain, 0.0, k)
    assert len(pix) == k and np.all(pix == (n // 2) * n + n // 2)
    want = F * gain * (1 - gain) ** np.arange(k)
    assert np.allclose(flux, want, rtol=1e-5)
    assert flux.sum() == pytest.approx(F * (1 - (1 - gain) ** k), rel=1e-5)
    assert R[n // 2, n // 2] == pytest.approx(F * (1 - gain) ** k, rel=1e-4)
    # the residual is the beam scaled by what is left
    assert np.allclose(R, F * (1 - gain) ** k * P, atol=1e-5)


def test_clean_gain_one_takes_the_source_in_one_component_then_stops():
    n, cell = 32, 2e-3
    u, v = _cell_centred_uv(n, cell, 200)
    vis = imaging.point_source_vis(u, v, [(1.7, 0.0, 0.0)])
    D, P = imaging.dirty_and_psf(u, v, vis, None, n, cell)
    pix, flux, R = imaging.hogbom(D, P, 1.0, 1e-3, 50)
    assert len(pix) == 1 and flux[0] == pytest.approx(1.7, rel=1e-6)
    assert np.max(np.abs(R)) < 1e-5


def test_clean_ties_take_the_smallest_index_and_threshold_stops():
    n = 8
    P = np.zeros((n, n), np.float32)
    P[n // 2, n // 2] = 1.0            # a delta beam
    D = np.zeros((n, n), np.float32)
    D[5, 1] = -2.0
    D[2, 6] = 2.0                      # |same| peak, smaller flat index 2*8+6 = 22 < 41
    D[3, 3] = 0.5
    pix, flux, R = imaging.hogbom(D, P, 1.0, 0.6, 10)
    assert list(pix) == [22, 41] and list(flux) == [2.0, -2.0]
    assert R[3, 3] == np.float32(0.5)  # below the threshold: left alone


def test_clean_two_sources_recovered():
    n, cell = 64, 2e-3
    u, v = _cell_centred_uv(n, cell, 1500)
    src = [(1.0, 6 * cell, -4 * cell), (0.6, -9 * cell, 7 * cell)]
    vis = imaging.point_source_vis(u, v, src)
    D, P = imaging.dirty_and_psf(u, v, vis, None, n, cell)
    pix, flux, R = imaging.hogbom(D, P, 0.2, 1e-3, 400)
    model = np.zeros(n * n)
    np.add.at(model, pix, flux)
    model = model.reshape(n, n)
    assert model[n // 2 + 6, n // 2 - 4] == pytest.approx(1.0, abs=2e-3)
    assert model[n // 2 - 9, n // 2 + 7] == pytest.approx(0.6, abs=2e-3)
    assert np.abs(model).sum() == pytest.approx(1.6, abs=5e-3)   # nothing spurious
    assert np.max(np.abs(R)) < 1.1e-3


def test_clean_off_centre_source_decays_geometrically():
    """The circular shift: an off-centre lone source is removed exactly as
    a centred one (its dirty image is the beam rolled onto its pixel)."""
    n, cell = 32, 2e-3
    u, v = _cell_centred_uv(n, cell, 200)
    vis = imaging.point_source_vis(u, v, [(1.0, 11 * cell, -13 * cell)])
    D, P = imaging.dirty_and_psf(u, v, vis, None, n, cell)
    pix, flux, R = imaging.hogbom(D, P, 0.5, 0.0, 8)
    assert np.all(pix == (n // 2 + 11) * n + (n // 2 - 13))
    assert np.allclose(flux, 0.5 * 0.5 ** np.arange(8), rtol=1e-5)
    assert np.allclose(R, 0.5 ** 8 * np.roll(P, (11, -13), axis=(0, 1)), atol=1e-6)
