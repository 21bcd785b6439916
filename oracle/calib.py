"""Delay/phase application and the three-step delay/phase solve.

Application follows the paper's Sec. 4.1 step 2 and eq. (1): a linear phase
rotation exp(+j 2 pi nu tau) compensates a delay.  Applied per baseline
b = (i, j) with per-antenna delays and phases:

    V'_b[k] = V_b[k] * exp(+i [2 pi f_k (tau_i - tau_j) + (phi_i - phi_j)]),
    f_k = f0 + k * df.

Sign reading: an antenna whose signal arrives d samples late has
X_a ~ exp(-2 pi i f_k d / fs), so V_ij ~ exp(-2 pi i f_k (d_i - d_j)/fs);
tau_a = d_a / fs then cancels it, matching eq. (1) with tau_g,ij = tau_i - tau_j.

The solve follows Sec. 7's three serial steps:
  1. coarse group delay from the peak of the delay spectrum (transform of the
     visibilities along frequency);
  2. fine delay from a weighted linear fit of unwrapped phase against
     frequency in a clean band, eq. (3): tau_res = (1/2pi) dphi/dnu (with
     the sign of the correction convention above: the fitted phase slope of
     the coarse-corrected visibility is -2 pi tau_res);
  3. residual phase from the mean complex vector in the clean band.
Per-antenna values come from a float64 least-squares fit over the cross
baselines with a reference antenna held at zero.

Readings (not fixed by the paper): visibilities are integrated over time
with flagged cells zeroed before the solve; the delay spectrum is a direct
transform on a grid of n_lag lags, n_lag the smallest power of two at least
lag_pad * n_chan, at most 8192 (and at least n_chan); fit weights are the
amplitudes of the time-integrated, flag-zeroed visibilities; the phase is
unwrapped as numpy.unwrap does (a step of magnitude above pi gets a 2 pi
correction of the opposite sign).
Status: pinned (tests/test_oracle.py): the delay spectrum by numpy's
inverse FFT of the zero-padded spectrum; the coarse delay by exact recovery
of on-grid delays of both signs and nearest-lag recovery off the grid; the
whole solve by noiseless recovery and by steep, noisy phases that only the
coarse step lets the fine fit unwrap.
"""

from __future__ import annotations

import numpy as np

from .xengine import baseline_pairs


def rotation_angles(n_ant, n_chan, f0, df, tau_s, phi_rad) -> np.ndarray:
    """theta[b, k] = 2 pi f_k (tau_i - tau_j) + (phi_i - phi_j), float64."""
    tau = np.asarray(tau_s, np.float64)
    phi = np.asarray(phi_rad, np.float64)
    f = f0 + np.arange(n_chan, dtype=np.float64) * df
    th = np.zeros((n_ant * (n_ant + 1) // 2, n_chan))
    for b, (i, j) in enumerate(baseline_pairs(n_ant)):
        th[b] = 2.0 * np.pi * f * (tau[i] - tau[j]) + (phi[i] - phi[j])
    return th


def apply_delay_phase(vis, n_ant, f0, df, tau_s, phi_rad) -> np.ndarray:
    """V' = V * exp(+i theta) for vis[n_time, n_base, n_chan] (complex128 out)."""
    V = np.asarray(vis, np.complex128)
    th = rotation_angles(n_ant, V.shape[2], f0, df, tau_s, phi_rad)
    return V * np.exp(1j * th)[None, :, :]


def delay_spectrum(Vb, n_lag: int) -> np.ndarray:
    """D[l] = sum_k Vb[k] exp(+2 pi i k l / n_lag), l = 0 .. n_lag-1."""
    Vb = np.asarray(Vb, np.complex128)
    k = np.arange(Vb.size, dtype=np.int64)[None, :]
    l = np.arange(n_lag, dtype=np.int64)[:, None]
    ph = ((k * l) % n_lag).astype(np.float64) / n_lag
    return np.exp(2j * np.pi * ph) @ Vb


def lag_grid(n_chan: int, lag_pad: int = 4) -> int:
    """Number of lags of the delay spectrum (see the module's readings)."""
    n = 1
    while n < lag_pad * n_chan:
        n *= 2
    n = min(n, 8192)
    while n < n_chan:
        n *= 2
    return n


def coarse_delay(Vb, df, n_lag: int) -> float:
    """Step 1 of Sec. 7: the delay at the peak of |delay spectrum|.

    Lag l of the n_lag-point grid is the delay l / (n_lag df) for
    l < n_lag/2 and (l - n_lag) / (n_lag df) above (the grid spans one
    period 1/df of the spectrum's delay response, centred on zero).  Ties go
    to the smallest l (numpy.argmax).
    """
    D = np.abs(delay_spectrum(Vb, n_lag))
    l = int(np.argmax(D))
    ls = l if l < n_lag // 2 else l - n_lag
    return ls / (n_lag * df)


def solve_baseline(Vb, f0, df, chan_lo, chan_hi, lag_pad: int = 4):
    """(tau, phi) for one baseline's time-integrated spectrum Vb[k].

    Model: Vb[k] ~ A exp(-i (2 pi f_k tau + phi)).
    """
    Vb = np.asarray(Vb, np.complex128)
    n_chan = Vb.size
    n_lag = lag_grid(n_chan, lag_pad)
    f = f0 + np.arange(n_chan, dtype=np.float64) * df
    # step 1: coarse delay from the delay-spectrum peak
    tau_c = coarse_delay(Vb, df, n_lag)
    # step 2: weighted LS of unwrapped phase vs frequency in the clean band
    W = Vb * np.exp(2j * np.pi * f * tau_c)
    band = slice(chan_lo, chan_hi)
    fb = f[band]
    psi = np.unwrap(np.angle(W[band]))
    w = np.abs(Vb[band])
    S0, S1, S2 = w.sum(), (w * fb).sum(), (w * fb * fb).sum()
    T0, T1 = (w * psi).sum(), (w * fb * psi).sum()
    det = S0 * S2 - S1 * S1
    slope = (S0 * T1 - S1 * T0) / det
    tau = tau_c - slope / (2.0 * np.pi)
    # step 3: residual phase from the mean complex vector in the band
    U = Vb[band] * np.exp(2j * np.pi * fb * tau)
    phi = -np.angle(U.sum())
    return tau, phi


def wrap(a):
    return (np.asarray(a) + np.pi) % (2.0 * np.pi) - np.pi


def antenna_solution(tau_b, phi_b, n_ant, ref_ant):
    """Per-antenna (tau, phi) from per-baseline values, ref antenna at zero.

    tau: float64 least squares of tau_i - tau_j = tau_b over cross baselines.
    phi: the reference-antenna baselines give a first solution; the wrapped
    residuals of every cross baseline then refine it by least squares.
    """
    pairs = [(i, j) for (i, j) in baseline_pairs(n_ant) if i != j]
    free = [a for a in range(n_ant) if a != ref_ant]
    col = {a: c for c, a in enumerate(free)}
    G = np.zeros((len(pairs), len(free)))
    for r, (i, j) in enumerate(pairs):
        if i in col:
            G[r, col[i]] += 1.0
        if j in col:
            G[r, col[j]] -= 1.0
    N = G.T @ G
    tau = np.zeros(n_ant)
    tau[free] = np.linalg.solve(N, G.T @ np.asarray(tau_b, np.float64))
    phi0 = np.zeros(n_ant)
    for r, (i, j) in enumerate(pairs):
        if j == ref_ant:
            phi0[i] = phi_b[r]
        elif i == ref_ant:
            phi0[j] = -phi_b[r]
    resid = np.array([wrap(phi_b[r] - (phi0[i] - phi0[j]))
                      for r, (i, j) in enumerate(pairs)])
    phi = phi0.copy()
    phi[free] += np.linalg.solve(N, G.T @ resid)
    return tau, wrap(phi)


def solve_delay_phase(vis, mask, n_ant, f0, df, ref_ant, chan_lo, chan_hi,
                      lag_pad: int = 4):
    """Per-antenna (tau_s, phi_rad) from flagged visibilities [n_time, n_base, n_chan]."""
    V = np.asarray(vis, np.complex128)
    keep = 1.0 - np.asarray(mask, np.float64) if mask is not None else 1.0
    Vi = (V * keep).sum(axis=0)
    taus, phis = [], []
    for b, (i, j) in enumerate(baseline_pairs(n_ant)):
        if i == j:
            continue
        t, p = solve_baseline(Vi[b], f0, df, chan_lo, chan_hi, lag_pad)
        taus.append(t)
        phis.append(p)
    return antenna_solution(np.array(taus), np.array(phis), n_ant, ref_ant)
