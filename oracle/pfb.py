"""F-engine oracle: polyphase FIR weighting followed by a direct DFT.

Follows the paper's Sec. 4.1 (step 1: the F-engine turns the voltage stream
into a spectrum), Sec. 4.2 ("F-engine (PFB and FFT)": a PFB stage precedes
the FFT) and Alg. 1 (F-Engine: apply PFB weighting, then FFT).  The paper
gives no filter formula for the hot path; the reading taken here is a
Hann-windowed sinc prototype of P*N taps, unnormalised.

Readings (the paper is silent on these):
  * start of stream: samples before x[0] are zero unless a history block is
    supplied, so a stream of S samples yields M = S // N spectra;
  * transform: forward kernel exp(-2*pi*i*k*n/N), no normalisation;
  * channels: a real N-point transform keeps k = 0 .. N/2-1 (Nyquist
    dropped) unless ``keep_nyquist``;
  * input words: real int8 (the 8-bit truncated mode of Sec. 3.3) or real
    int16 (the default 16-bit padded mode, the 14-bit ADC value taken as the
    integer it is) enter as exact float64; complex I/Q samples (the "complex
    voltage streams" of Sec. 4.2) take the same FIR on I and Q and an
    N-point complex DFT keeping all N channels k = 0 .. N-1 in natural
    order (k >= N/2 are the negative frequencies);
  * window variants (Fig. pfb_fft): a Kaiser window of shape beta in place
    of the Hann window, and the plain rectangular FFT (P = 1, all-ones
    taps) the figure compares against.

This is the plain definition evaluated directly (a twiddle matrix product),
not an FFT.  Status: pinned (see tests/test_oracle.py).
"""

from __future__ import annotations

import numpy as np


def hann_sinc_taps(n_fft: int, n_taps: int) -> np.ndarray:
    """Prototype filter h[q], q = 0 .. P*N-1 (float64).

    L = P*N, centre c = (L-1)/2, symmetric Hann w[q] = 0.5 - 0.5 cos(2 pi q/(L-1)),
    h[q] = w[q] * sinc((q - c)/N) with sinc(u) = sin(pi u)/(pi u), sinc(0) = 1.
    No normalisation.  The sinc's first zeros fall N samples from the centre,
    i.e. its passband is one channel wide.
    """
    L = n_fft * n_taps
    q = np.arange(L, dtype=np.float64)
    if L > 1:
        w = 0.5 - 0.5 * np.cos(2.0 * np.pi * q / (L - 1))
    else:
        w = np.ones(1)
    u = (q - (L - 1) / 2.0) / n_fft
    return w * np.sinc(u)


def kaiser_sinc_taps(n_fft: int, n_taps: int, beta: float) -> np.ndarray:
    """Kaiser-windowed sinc h[q], q = 0 .. P*N-1 (float64), unnormalised.

    w[q] = I0(beta sqrt(1 - (2q/(L-1) - 1)^2)) / I0(beta) (symmetric, L-1 in
    the denominator, as the Hann prototype), h[q] = w[q] sinc((q - c)/N),
    c = (L-1)/2.  The paper's figure uses P = 8 and beta = 8.
    """
    L = n_fft * n_taps
    q = np.arange(L, dtype=np.float64)
    if L > 1:
        r = 2.0 * q / (L - 1) - 1.0
        w = np.i0(beta * np.sqrt(np.maximum(0.0, 1.0 - r * r))) / np.i0(beta)
    else:
        w = np.ones(1)
    return w * np.sinc((q - (L - 1) / 2.0) / n_fft)


def rect_taps(n_fft: int) -> np.ndarray:
    """The plain FFT's all-ones window (P = 1): no filter at all."""
    return np.ones(int(n_fft))


def pfb_frames(x, n_fft: int, n_taps: int, taps=None, hist=None) -> np.ndarray:
    """Polyphase-FIR output y[a, m, n] (float64), n = 0 .. N-1.

    y[a, m, n] = sum_{p=0}^{P-1} h[p*N + n] * x_a[(m - P + 1 + p)*N + n]

    Spectrum m's newest block is block m of the stream.  ``x`` is int
    [n_ant, S] with S a multiple of N; ``hist`` (optional) is int
    [n_ant, (P-1)*N] holding the samples just before x[:, 0].
    """
    x = np.asarray(x)
    n_ant, S = x.shape
    N, P = int(n_fft), int(n_taps)
    if S % N:
        raise ValueError("stream length must be a multiple of N")
    h = hann_sinc_taps(N, P) if taps is None else np.asarray(taps, np.float64)
    if h.shape != (P * N,):
        raise ValueError("taps must have P*N entries")
    pad = np.zeros((n_ant, (P - 1) * N), np.float64)
    if hist is not None:
        pad[:] = np.asarray(hist, np.float64).reshape(n_ant, (P - 1) * N)
    xp = np.concatenate([pad, x.astype(np.float64)], axis=1)
    M = S // N
    blocks = xp.reshape(n_ant, M + P - 1, N)  # block j of xp is stream block j-(P-1)
    hp = h.reshape(P, N)
    y = np.zeros((n_ant, M, N), np.float64)
    for p in range(P):
        # stream block (m - P + 1 + p) is xp block (m + p)
        y += hp[p][None, None, :] * blocks[:, p:p + M, :]
    return y


def twiddle_matrix(n_fft: int, chans) -> np.ndarray:
    """T[k, n] = exp(-2 pi i ((k*n) mod N) / N) for the requested channels.

    The phase comes from the exact integer k*n mod N, so no large-argument
    error enters the twiddles.
    """
    N = int(n_fft)
    k = np.asarray(chans, dtype=np.int64)[:, None]
    n = np.arange(N, dtype=np.int64)[None, :]
    r = (k * n) % N
    return np.exp(-2j * np.pi * r.astype(np.float64) / N)


def default_chans(n_fft: int, keep_nyquist: bool = False) -> np.ndarray:
    return np.arange(n_fft // 2 + (1 if keep_nyquist else 0))


def dft(y, n_fft: int, chans=None, keep_nyquist: bool = False) -> np.ndarray:
    """X[..., k] = sum_n y[..., n] exp(-2 pi i k n / N) (direct, complex128)."""
    if chans is None:
        chans = default_chans(n_fft, keep_nyquist)
    T = twiddle_matrix(n_fft, chans)
    y = np.asarray(y, np.float64)
    return y @ T.T


def channelize(x, n_fft: int, n_taps: int, taps=None, hist=None, chans=None,
               keep_nyquist: bool = False) -> np.ndarray:
    """Channelised voltages X[a, m, k] (complex128): FIR weighting then DFT."""
    y = pfb_frames(x, n_fft, n_taps, taps=taps, hist=hist)
    return dft(y, n_fft, chans=chans, keep_nyquist=keep_nyquist)


def complex_frames(x, n_fft: int, n_taps: int, taps=None, hist=None) -> np.ndarray:
    """Polyphase-FIR output of complex streams (complex128), the same sum as
    pfb_frames with the real taps applied to I and Q alike."""
    x = np.asarray(x)
    n_ant, S = x.shape
    N, P = int(n_fft), int(n_taps)
    if S % N:
        raise ValueError("stream length must be a multiple of N")
    h = hann_sinc_taps(N, P) if taps is None else np.asarray(taps, np.float64)
    if h.shape != (P * N,):
        raise ValueError("taps must have P*N entries")
    pad = np.zeros((n_ant, (P - 1) * N), np.complex128)
    if hist is not None:
        pad[:] = np.asarray(hist, np.complex128).reshape(n_ant, (P - 1) * N)
    xp = np.concatenate([pad, x.astype(np.complex128)], axis=1)
    M = S // N
    blocks = xp.reshape(n_ant, M + P - 1, N)
    hp = h.reshape(P, N)
    y = np.zeros((n_ant, M, N), np.complex128)
    for p in range(P):
        y += hp[p][None, None, :] * blocks[:, p:p + M, :]
    return y


def channelize_complex(x, n_fft: int, n_taps: int, taps=None, hist=None, chans=None) -> np.ndarray:
    """Channelised voltages of complex I/Q streams: FIR, then the N-point
    complex DFT X[a, m, k] = sum_n y[a, m, n] exp(-2 pi i k n / N) on all
    N channels (or the requested ones)."""
    y = complex_frames(x, n_fft, n_taps, taps=taps, hist=hist)
    if chans is None:
        chans = np.arange(int(n_fft))
    return y @ twiddle_matrix(n_fft, chans).T


def stream_history(x, n_fft: int, n_taps: int, hist=None) -> np.ndarray:
    """The last (P-1)*N samples of (hist ++ x): the history the next chunk needs."""
    n_ant = x.shape[0]
    keep = (n_taps - 1) * n_fft
    pad = np.zeros((n_ant, keep), np.int64) if hist is None else np.asarray(hist, np.int64)
    full = np.concatenate([pad, np.asarray(x, np.int64)], axis=1)
    return full[:, full.shape[1] - keep:] if keep else full[:, :0]
