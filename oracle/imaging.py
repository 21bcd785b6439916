"""Synthesis-imaging oracle: gridding, Fourier inversion, Hogbom CLEAN.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper's Sec. 8.1: calibrated visibilities are gridded,
transformed into a dirty image and a synthesized beam (PSF), and
deconvolved with standard CLEAN (Hogbom 1974), giving components and a
residual map.  The paper names the steps, not their formulas; the readings
taken here:

  * measurement equation: V(u, v) = sum_s F_s exp(-2 pi i (u l_s + v m_s)),
    u, v in wavelengths, l, m direction cosines (radians for small fields);
  * gridding: nearest cell.  An n x n grid of cell du = 1 / (n * cell)
    (cell = image pixel in radians) holds cell (iu, iv) at
    u = (iu - n/2) du, v = (iv - n/2) du.  A visibility goes to
    iu = floor(u/du + 1/2) + n/2 (same for v), its conjugate to the mirrored
    cell n - iu (same for v), each with its weight; samples whose cell or
    mirror falls outside [0, n) are dropped.  The cell decision is made in
    float64 from the float32 coordinates;
  * dirty image: I(il, im) = Re sum_{iu, iv} G[iu, iv]
    exp(+2 pi i ((iu - n/2)(il - n/2) + (iv - n/2)(im - n/2)) / n) / W with
    W the total gridded weight (both copies), so a unit point source at the
    phase centre peaks at exactly 1; pixel (il, im) is at
    l = (il - n/2) cell, m = (im - n/2) cell.  Evaluated with numpy's
    inverse FFT (a library step) around the centring shifts;
  * PSF (synthesized beam): the dirty image of unit visibilities gridded
    on the same n x n grid, so it is exactly the beam of that grid; its
    peak, 1, is at pixel (n/2, n/2);
  * Hogbom CLEAN, float32 throughout: the peak is the pixel of largest
    |residual| (ties to the smallest flat index il * n + im); stop when
    |peak| < threshold or after max_iter components; component flux
    g = gain * peak (rounded to float32); subtract
    g * psf[(p - peak + (n/2, n/2)) mod n] from every pixel p: the dirty
    image of gridded data is periodic over the field, so the beam of an
    off-centre source wraps around it, and the shift is taken circularly.
    The product and the difference are each rounded to float32 (no fused
    multiply-add).  Float decides the integer argmax, so both sides take it
    in the same precision.

Status: pinned (tests/test_oracle_imaging.py): gridding by brute force and
Hermitian symmetry; the dirty image by a direct sum on small grids and by
point sources landing on their pixels; CLEAN by closed forms (a lone
source through its own PSF, geometric decay with gain) and brute force.
"""

from __future__ import annotations

import numpy as np


def cell_index(coord, inv_du: float, n: int) -> np.ndarray:
    """Grid cell of each coordinate: floor(coord * inv_du + 1/2) + n/2 (int64),
    the product formed in float64 from the float32 coordinate."""
    x = np.asarray(coord, np.float32).astype(np.float64) * float(inv_du)
    return np.floor(x + 0.5).astype(np.int64) + n // 2


def grid_nearest(u, v, vis, weight, n: int, cell_rad: float):
    """Nearest-cell gridding with Hermitian mirrors.

    Returns (G, W): complex128 grid [n, n] (indexed [iu, iv]) and the total
    gridded weight W (both copies of every kept sample).
    """
    inv_du = n * cell_rad  # 1 / du
    iu = cell_index(u, inv_du, n)
    iv = cell_index(v, inv_du, n)
    ju, jv = n - iu, n - iv
    vis = np.asarray(vis, np.complex128)
    w = np.ones(vis.shape) if weight is None else np.asarray(weight, np.float64)
    G = np.zeros((n, n), np.complex128)
    W = 0.0
    for k in range(vis.size):
        a, b, c, d = iu[k], iv[k], ju[k], jv[k]
        if 0 <= a < n and 0 <= b < n and 0 <= c < n and 0 <= d < n:
            G[a, b] += w[k] * vis[k]
            G[c, d] += w[k] * np.conj(vis[k])
            W += 2.0 * w[k]
    return G, W


def invert(G, W: float) -> np.ndarray:
    """Dirty image [n, n] (float64) of a grid, as defined in the module."""
    G = np.asarray(G, np.complex128)
    n = G.shape[0]
    s = (-1.0) ** np.arange(n)
    # sum_iu G[iu] e^{2pi i (iu - n/2)(il - n/2)/n}
    #   = (-1)^{il} (-1)^{n/2} sum_iu ((-1)^{iu} G[iu]) e^{2pi i iu il / n}
    Gs = G * s[:, None] * s[None, :]
    img = np.fft.ifft2(Gs) * (n * n)
    sign = (-1.0) ** (n // 2)
    img = img * s[:, None] * s[None, :] * sign * sign
    return img.real / W


def invert_direct(G, W: float) -> np.ndarray:
    """The dirty image as the plain double sum (small grids only)."""
    G = np.asarray(G, np.complex128)
    n = G.shape[0]
    c = np.arange(n) - n // 2
    E = np.exp(2j * np.pi * np.outer(c, c) / n)  # E[iu, il]
    return (E.T @ G @ E).real / W


def dirty_and_psf(u, v, vis, weight, n: int, cell_rad: float):
    """(dirty image, PSF), both n x n and normalised."""
    G, W = grid_nearest(u, v, vis, weight, n, cell_rad)
    ones = np.ones(np.asarray(vis).shape, np.complex128)
    Gp, Wp = grid_nearest(u, v, ones, weight, n, cell_rad)
    return invert(G, W), invert(Gp, Wp)


def point_source_vis(u, v, sources):
    """V(u, v) = sum_s F_s exp(-2 pi i (u l_s + v m_s)) (complex128)."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    V = np.zeros(u.shape, np.complex128)
    for (F, l, m) in sources:
        V += F * np.exp(-2j * np.pi * (u * l + v * m))
    return V


def hogbom(dirty, psf, gain: float, threshold: float, max_iter: int):
    """Hogbom CLEAN in float32, as defined in the module.

    Returns (pix [k] int64 flat indices il * n + im, flux [k] float32,
    residual [n, n] float32).
    """
    r = np.array(dirty, np.float32, copy=True)
    P = np.asarray(psf, np.float32)
    n = r.shape[0]
    g32 = np.float32(gain)
    thr = np.float32(threshold)
    pix, flux = [], []
    for _ in range(max_iter):
        a = np.abs(r).ravel()
        k = int(np.argmax(a))            # ties: smallest flat index
        peak = r.ravel()[k]
        if np.abs(peak) < thr:
            break
        g = np.float32(g32 * peak)
        il, im = divmod(k, n)
        # beam value at pixel p: psf[(p - peak + (n/2, n/2)) mod n]
        shifted = np.roll(P, (il - n // 2, im - n // 2), axis=(0, 1))
        prod = (g * shifted).astype(np.float32)   # rounded product
        r = (r - prod).astype(np.float32)         # rounded difference
        pix.append(k)
        flux.append(g)
    return np.array(pix, np.int64), np.array(flux, np.float32), r
