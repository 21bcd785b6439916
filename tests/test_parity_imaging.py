"""GPU parity: synthesis imaging (Sec. 8.1) against the FP64/float32 oracle.

* gridding: cells exact (same float64 decision), values within float32
  atomic-sum rounding (1e-5 of the largest cell), total weight exact;
* inversion: dirty image and beam within 1e-5 of the image peak, from the
  GPU grid and from the oracle grid;
* Hogbom CLEAN: on the same float32 dirty image and beam, components
  (pixel and flux) and the residual bit-identical to the oracle's (both
  round product and difference separately and break ties alike);
* end to end on a synthetic 4-antenna earth-rotation observation: the
  sources recovered within the gridding error.
"""

import numpy as np
import pytest

import synth
from oracle import imaging

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _random_uv(n, cell, k, seed, span=0.45):
    rng = np.random.default_rng(seed)
    du = 1.0 / (n * cell)
    u = rng.uniform(-span * n * du, span * n * du, k).astype(np.float32)
    v = rng.uniform(-span * n * du, span * n * du, k).astype(np.float32)
    vis = (rng.normal(size=k) + 1j * rng.normal(size=k)).astype(np.complex64)
    w = rng.uniform(0.2, 2.0, k).astype(np.float32)
    return u, v, vis, w


@pytest.mark.parametrize("n,k", [(64, 3000), (256, 50000), (1024, 200000)])
def test_grid_matches_oracle(qc, n, k):
    cell = 1e-3
    u, v, vis, w = _random_uv(n, cell, k, seed=n, span=0.55)   # some samples fall off the grid
    g, ws = qc.image_grid(_dev(u), _dev(v), _dev(vis), n, cell, weight=_dev(w))
    G_ref, W_ref = imaging.grid_nearest(u, v, vis, w, n, cell)
    G = g.cpu().numpy()
    assert np.array_equal(G != 0, G_ref != 0)
    assert np.max(np.abs(G - G_ref)) <= 1e-5 * np.max(np.abs(G_ref))
    assert ws.item() == pytest.approx(W_ref, rel=1e-12)


@pytest.mark.parametrize("n", [64, 256, 1024, 4096])
def test_invert_matches_oracle(qc, n):
    cell = 2e-3
    u, v, vis, w = _random_uv(n, cell, 20000, seed=7 + n)
    g, ws = qc.image_grid(_dev(u), _dev(v), _dev(vis), n, cell, weight=_dev(w))
    img = qc.image_invert(g, ws).cpu().numpy()
    ref = imaging.invert(g.cpu().numpy().astype(np.complex128), ws.item())
    assert np.max(np.abs(img - ref)) <= 1e-5 * np.max(np.abs(ref))
    G_ref, W_ref = imaging.grid_nearest(u, v, vis, w, n, cell)
    ref2 = imaging.invert(G_ref, W_ref)
    assert np.max(np.abs(img - ref2)) <= 1e-5 * np.max(np.abs(ref2))


def test_beam_peaks_at_one_on_the_centre(qc):
    o = synth.imaging_obs(n=256)
    _, psf = qc.image_dirty_and_psf(_dev(o.u), _dev(o.v), _dev(o.vis), o.n, o.cell_rad)
    P = psf.cpu().numpy()
    assert np.unravel_index(np.argmax(P), P.shape) == (128, 128)
    assert P[128, 128] == pytest.approx(1.0, abs=1e-6)


@pytest.mark.parametrize("n,gain,thr,iters", [(64, 0.1, 0.0, 300), (256, 0.2, 1e-3, 400), (256, 1.0, 0.05, 50),
                                              (128, 0.05, 0.0, 0)])
def test_clean_bit_identical_to_oracle(qc, n, gain, thr, iters):
    o = synth.imaging_obs(n=n, n_chan=64, n_time=32, noise=0.02, seed=5000 + n)
    D, P = imaging.dirty_and_psf(o.u, o.v, o.vis, None, n, o.cell_rad)
    D32, P32 = D.astype(np.float32), P.astype(np.float32)
    pix_r, flux_r, R_r = imaging.hogbom(D32, P32, gain, thr, iters)
    res = _dev(D32)
    pix, flux = qc.image_clean(res, _dev(P32), gain, thr, iters)
    assert np.array_equal(pix.cpu().numpy().astype(np.int64), pix_r)
    assert np.array_equal(flux.cpu().numpy(), flux_r)
    assert np.array_equal(res.cpu().numpy(), R_r)


def test_clean_ties_and_threshold(qc):
    n = 16
    P = np.zeros((n, n), np.float32)
    P[n // 2, n // 2] = 1.0
    D = np.zeros((n, n), np.float32)
    D[11, 3] = -2.0
    D[4, 13] = 2.0
    D[6, 6] = 0.5
    res = _dev(D)
    pix, flux = qc.image_clean(res, _dev(P), 1.0, 0.6, 10)
    assert pix.cpu().numpy().tolist() == [4 * n + 13, 11 * n + 3]
    assert flux.cpu().numpy().tolist() == [2.0, -2.0]
    assert res.cpu().numpy()[6, 6] == np.float32(0.5)


def test_end_to_end_synthetic_observation(qc):
    """4 antennas, 256 channels x 64 hour angles (98,304 visibilities), three
    point sources: dirty image, beam and CLEAN on the GPU; the components
    near each source add up to its flux within the nearest-cell gridding
    error, and CLEAN lowers the residual below 2 % of the dirty peak."""
    o = synth.imaging_obs(n=256)
    dirty, psf = qc.image_dirty_and_psf(_dev(o.u), _dev(o.v), _dev(o.vis), o.n, o.cell_rad)
    D0 = dirty.cpu().numpy().copy()
    pix, flux = qc.image_clean(dirty, psf, 0.1, 0.01, 1000)
    model = np.zeros(o.n * o.n)
    np.add.at(model, pix.cpu().numpy(), flux.cpu().numpy())
    model = model.reshape(o.n, o.n)
    for (F, l, m) in o.sources:
        il, im = int(round(l / o.cell_rad)) + o.n // 2, int(round(m / o.cell_rad)) + o.n // 2
        got = model[il - 1:il + 2, im - 1:im + 2].sum()
        assert got == pytest.approx(F, rel=0.08), (F, got)
    assert np.max(np.abs(dirty.cpu().numpy())) < 0.02 * np.max(D0)


def test_imaging_rejects_bad_arguments(qc):
    import torch
    g = torch.zeros((100, 100), dtype=torch.complex64, device="cuda")
    w = torch.zeros(1, dtype=torch.float64, device="cuda")
    x = torch.zeros(4, dtype=torch.float32, device="cuda")
    vis = torch.zeros(4, dtype=torch.complex64, device="cuda")
    with pytest.raises(qc.QCError):
        qc.image_grid(x, x, vis, 100, 1e-3, grid=g, wsum=w)      # n not a power of two
    with pytest.raises(qc.QCError):
        qc.image_grid(x, x, vis, 64, -1.0)                       # cell <= 0
    r = torch.zeros((64, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(qc.QCError):
        qc.image_clean(r, r, 1.5, 0.0, 5)                        # gain > 1
