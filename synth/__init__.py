"""Seeded synthetic int8 voltage streams shaped like the paper's workloads.

Shared by the tests, the oracle's callers and the benchmark.  It holds no
part of the correlator's arithmetic (no taps, no transforms, no products):
only random draws, mixing and rounding to int8.

Stream model, per antenna a and sample n (all float32 until the final
round-half-even and clip to [-128, 127]):

    x_a[n] = sigma * g_a[n]                       independent noise
           + sqrt(corr) * sigma * c[n - d_a]       common sky component, lag d_a
           + tone[n] + lines[n] + bursts[n]        common to all antennas

Random numbers come from numpy's PCG64 seeded by SeedSequence((seed,
stream id, block index)), so any chunk can be regenerated on its own and
chunks are filled in parallel.  Tones and lines sit at frequencies k/period
and are evaluated over one period, then indexed.
"""

from __future__ import annotations

import concurrent.futures as cf
import math
import os
from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 22
C_BLOCK = 1 << 16      # granularity of the common (lagged) component


def _rng(seed: int, stream: int, chunk: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream, chunk])))


@dataclass
class StreamSpec:
    n_ant: int
    n_samp: int
    seed: int
    sigma: float = 16.0
    corr: float = 0.3
    lags: tuple = ()
    tone_amp: float = 0.0
    tone_cycles_per_sample: float = 0.0
    lines: list = field(default_factory=list)     # [(cycles_per_sample, amp, phase)]
    bursts: list = field(default_factory=list)    # [(start_sample, length, rms)]
    period: int = 0   # tone and line frequencies are multiples of 1/period
    # linear chirps [(start_sample, length, f0, f1, amp, phase)]: frequency
    # f0 -> f1 (cycles per sample) over the length, common to all antennas
    chirps: list = field(default_factory=list)
    # sample word: 8 -> int8 in [-128, 127]; 14 or 16 -> int16 clipped to
    # [-2^(bits-1), 2^(bits-1) - 1] (14 bits: the ADC range of the 16-bit
    # padded mode)
    bits: int = 8


def _common_component(spec: StreamSpec, lo: int, hi: int, max_lag: int) -> np.ndarray:
    """c[n] for n in [lo - max_lag, hi), assembled from seeded blocks."""
    out = np.empty(hi - lo + max_lag, np.float32)
    n = lo - max_lag
    pos = 0
    while n < hi:
        j = math.floor(n / C_BLOCK)
        c0 = j * C_BLOCK
        block = _rng(spec.seed, 1, j + 1_000_000).standard_normal(C_BLOCK, dtype=np.float32)
        a = n - c0
        b = min(C_BLOCK, hi - c0)
        out[pos:pos + b - a] = block[a:b]
        pos += b - a
        n = c0 + b
    return out


def _periodic_component(spec: StreamSpec) -> np.ndarray | None:
    """One period of the tone plus lines (float32), or None."""
    if not spec.tone_amp and not spec.lines:
        return None
    per = spec.period
    assert per > 0, "tones and lines need a period"
    n = np.arange(per, dtype=np.float64)
    acc = np.zeros(per, np.float64)
    if spec.tone_amp:
        acc += spec.tone_amp * np.cos(2.0 * np.pi * np.mod(n * spec.tone_cycles_per_sample, 1.0))
    for (f, amp, phase) in spec.lines:
        acc += amp * np.cos(2.0 * np.pi * np.mod(n * f, 1.0) + phase)
    return acc.astype(np.float32)


def _fill_chunk(spec: StreamSpec, x: np.ndarray, lo: int, lags, max_lag, periodic):
    n_ant, S = spec.n_ant, spec.n_samp
    hi = min(S, lo + CHUNK)
    j = lo // CHUNK
    L = hi - lo
    common = np.zeros(L, np.float32)
    if periodic is not None:
        per = periodic.size
        common += periodic[np.arange(lo, hi, dtype=np.int64) % per]
    for bi, (b0, blen, rms) in enumerate(spec.bursts):
        a, b = max(lo, b0), min(hi, b0 + blen)
        if a < b:
            r = _rng(spec.seed, 3, bi).standard_normal(blen, dtype=np.float32)
            common[a - lo:b - lo] += np.float32(rms) * r[a - b0:b - b0]
    for (c0, clen, f0, f1, amp, phase) in spec.chirps:
        a, b = max(lo, c0), min(hi, c0 + clen)
        if a < b:
            t = np.arange(a - c0, b - c0, dtype=np.float64)
            cyc = f0 * t + 0.5 * (f1 - f0) / clen * t * t
            common[a - lo:b - lo] += (amp * np.cos(2.0 * np.pi * np.mod(cyc, 1.0) + phase)).astype(np.float32)
    cpre = _common_component(spec, lo, hi, max_lag) if spec.corr else None
    k_corr = np.float32(math.sqrt(spec.corr) * spec.sigma)
    sig = np.float32(spec.sigma)
    for a_ in range(n_ant):
        v = _rng(spec.seed, 100 + a_, j).standard_normal(L, dtype=np.float32)
        v *= sig
        if cpre is not None:
            d = lags[a_]
            v += k_corr * cpre[max_lag - d:max_lag - d + L]
        v += common
        np.rint(v, out=v)
        top = float(2 ** (spec.bits - 1))
        np.clip(v, -top, top - 1, out=v)
        x[a_, lo:hi] = v.astype(x.dtype)


def generate(spec: StreamSpec, out: np.ndarray | None = None, threads: int | None = None) -> np.ndarray:
    """int8 (or int16 for bits > 8) [n_ant, n_samp] stream for ``spec``
    (deterministic in spec.seed)."""
    n_ant, S = spec.n_ant, spec.n_samp
    lags = tuple(spec.lags) if spec.lags else (0,) * n_ant
    assert len(lags) == n_ant
    max_lag = max(lags) if lags else 0
    x = np.empty((n_ant, S), np.int8 if spec.bits <= 8 else np.int16) if out is None else out
    periodic = _periodic_component(spec)
    starts = list(range(0, S, CHUNK))
    if threads is None:
        threads = min(16, len(os.sched_getaffinity(0)))
    if threads <= 1 or len(starts) == 1:
        for lo in starts:
            _fill_chunk(spec, x, lo, lags, max_lag, periodic)
    else:
        with cf.ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda lo: _fill_chunk(spec, x, lo, lags, max_lag, periodic), starts))
    return x


def generate_iq(spec: StreamSpec, threads: int | None = None) -> np.ndarray:
    """Complex I/Q stream [n_ant, n_samp, 2] (I, Q interleaved; int8 or int16).

    I is generate(spec); Q is an independent stream of the same shape with
    seed + 1 (its own noise and its own common component, so the common
    component is complex Gaussian with the same lags), and the tone and
    lines phase-shifted by -pi/2, so a tone becomes exp(+2 pi i f n).
    """
    import dataclasses
    q_lines = [(f, a, ph - math.pi / 2) for (f, a, ph) in spec.lines]
    if spec.tone_amp:
        q_lines.append((spec.tone_cycles_per_sample, spec.tone_amp, -math.pi / 2))
    qspec = dataclasses.replace(spec, seed=spec.seed + 1, tone_amp=0.0, lines=q_lines)
    xi = generate(spec, threads=threads)
    xq = generate(qspec, threads=threads)
    return np.stack([xi, xq], axis=-1)


# ---- the workloads (seed = 1000 * config number + realisation) -------------

@dataclass
class Workload:
    name: str
    x: np.ndarray
    n_fft: int
    n_taps: int
    spec_per_dump: int
    params: dict


def tone_stream(n_ant=4, n_samp=1 << 20, seed=1000, n_fft=1024, chan=137):
    """4 antennas, sigma 16 noise, 30% correlated power at lags {0,3,5,7},
    a tone of amplitude 16 centred on channel ``chan``, all seeded."""
    lags = (0, 3, 5, 7)[:n_ant] if n_ant <= 4 else tuple(range(n_ant))
    spec = StreamSpec(n_ant, n_samp, seed, corr=0.3, lags=lags,
                      tone_amp=16.0, tone_cycles_per_sample=chan / n_fft, period=n_fft)
    return spec


def plain_fx(n_samp=1 << 20, seed=1000) -> Workload:
    """Plain FX correlator: 4 ant, 2^20 samples, N=1024, P=4, one dump."""
    spec = tone_stream(4, n_samp, seed, 1024, 137)
    x = generate(spec)
    return Workload("plain_fx_4ant_n1024", x, 1024, 4, n_samp // 1024,
                    {"lags": spec.lags, "tone_chan": 137})


LINE_AMP = 1.4  # LSB: ~10x a channel's noise power at N=4096, sigma=16


def realtime_spec(n_samp=1 << 28, seed=2000, n_fft=4096, spec_per_dump=4096,
                  n_lines=20, burst_frac=0.05):
    """Real-time-shaped stream: lags U{0..40}, 20 lines, 5% bursts."""
    rng = _rng(seed, 7, 0)
    n_ant = 4
    lags = tuple(int(v) for v in rng.integers(0, 41, n_ant))
    n_chan = n_fft // 2
    chans = rng.choice(np.arange(8, n_chan - 8), n_lines, replace=False)
    lines = [(float(k) / n_fft, LINE_AMP, float(rng.uniform(-np.pi, np.pi))) for k in sorted(chans)]
    M = n_samp // n_fft
    bursts = []
    target = int(round(burst_frac * M))
    covered = 0
    while covered < target:
        blen = int(rng.integers(1, 65))
        start = int(rng.integers(0, max(1, M - blen)))
        bursts.append((start * n_fft, blen * n_fft, math.sqrt(10.0) * 16.0))
        covered += blen
    tau_s = np.array(lags, np.float64) * 1e-9      # 1 GS/s: one sample = 1 ns
    phi = rng.uniform(-np.pi, np.pi, n_ant)
    spec = StreamSpec(n_ant, n_samp, seed, corr=0.3, lags=lags, lines=lines, bursts=bursts,
                      period=n_fft)
    params = {"lags": lags, "line_chans": [int(k) for k in sorted(chans)],
              "tau_s": tau_s, "phi_rad": phi, "fs_hz": 1e9,
              "bursts": bursts}
    return spec, params


def realtime(n_samp=1 << 28, seed=2000) -> Workload:
    spec, params = realtime_spec(n_samp, seed)
    x = generate(spec)
    return Workload("realtime_4ant_n4096", x, 4096, 4, 4096, params)


def array_spec(n_ant=32, n_samp=1 << 24, seed=3000, corr=0.1, max_lag=40):
    rng = _rng(seed, 7, 0)
    lags = tuple(int(v) for v in rng.integers(0, max_lag + 1, n_ant))
    return StreamSpec(n_ant, n_samp, seed, corr=corr, lags=lags)


def precision(n_samp=1 << 24, seed=3000) -> Workload:
    """32 antennas, sigma 16, 10% correlated, lags U{0..40}, N=4096."""
    spec = array_spec(32, n_samp, seed)
    x = generate(spec)
    return Workload("precision_32ant_n4096", x, 4096, 4, n_samp // 4096, {"lags": spec.lags})


BATCH_ARRAYS = ((4, 512), (8, 1024), (16, 2048), (24, 2048), (32, 4096))


def batched(n_samp=1 << 22, seed=4000):
    """Five arrays (n_ant, n_chan); 30% correlated, lags U{0..7}; N = 2 n_chan."""
    out = []
    for idx, (na, nch) in enumerate(BATCH_ARRAYS):
        spec = array_spec(na, n_samp, seed + idx, corr=0.3, max_lag=7)
        out.append(Workload(f"batch_{na}ant_{nch}ch", generate(spec), 2 * nch, 4,
                            n_samp // (2 * nch), {"lags": spec.lags}))
    return out


# ---- streams with known injected RFI (training and judging the flagger) ------

# Nominal tap sums of the 4-tap Hann-sinc prototype, used only to set the
# injected amplitudes: sum h ~ N and sum h^2 ~ 0.8 N.
_SUM_H, _SUM_H2 = 1.0, 0.8


def _line_amp(snr, sigma, n_fft):
    """Amplitude of a bin-centred tone whose channel power is snr times the
    channel's noise power: A = 2 sigma sqrt(snr sum h^2) / sum h."""
    return 2.0 * sigma * math.sqrt(snr * _SUM_H2 * n_fft) / (_SUM_H * n_fft)


def rfi_realisation(seed, n_ant=32, n_samp=1 << 24, n_fft=4096, spec_per_dump=16, n_taps=4, corr=0.1,
                    n_lines=6, burst_frac=0.03, n_chirps=3, snr_range=(1.0, 50.0)):
    """Stream with injected RFI and its truth mask per (integration, channel).

    RFI is common to all antennas (one emitter), with log-uniform per-channel
    SNR (power in an affected channel over that channel's noise power, before
    integration):
      * persistent narrowband lines, bin-centred: truth = the line's channel
        in every integration;
      * broadband bursts of 1-64 spectra (white, rms sigma sqrt(snr)), about
        burst_frac of the spectra: truth = every channel of each integration
        holding a spectrum whose filter window overlaps the burst;
      * linear chirps over 256-2048 spectra (at most half the stream)
        sweeping 20-400 channels: truth =
        the channels swept while the window's central half (blocks m-2 and
        m-1 of spectrum m) passes, in that spectrum's integration.
    Returns (StreamSpec, truth uint8 [n_int, n_fft/2], params).
    """
    rng = _rng(seed, 11, 0)
    nch = n_fft // 2
    M = n_samp // n_fft
    n_int = M // spec_per_dump
    sigma = 16.0
    lo_s, hi_s = math.log(snr_range[0]), math.log(snr_range[1])

    def snr():
        return float(math.exp(rng.uniform(lo_s, hi_s)))

    lags = tuple(int(v) for v in rng.integers(0, 41, n_ant))
    truth = np.zeros((n_int, nch), np.uint8)
    chans = rng.choice(np.arange(8, nch - 8), n_lines, replace=False)
    lines, line_snr = [], []
    for k in sorted(int(c) for c in chans):
        sn = snr()
        lines.append((k / n_fft, _line_amp(sn, sigma, n_fft), float(rng.uniform(-np.pi, np.pi))))
        line_snr.append(sn)
        truth[:, k] = 1
    bursts, covered = [], 0
    target = int(round(burst_frac * M))
    while covered < target:
        blen = int(rng.integers(1, 65))
        m0 = int(rng.integers(0, M - blen))
        s0, s1 = m0 * n_fft, (m0 + blen) * n_fft
        bursts.append((s0, s1 - s0, sigma * math.sqrt(snr())))
        covered += blen
        m_first = s0 // n_fft
        m_last = min(M - 1, (s1 - 1) // n_fft + n_taps - 1)
        truth[m_first // spec_per_dump:m_last // spec_per_dump + 1, :] = 1
    chirps = []
    for _ in range(n_chirps):
        clen_spec = int(rng.integers(min(256, M // 4), min(2048, M // 2) + 1))
        m0 = int(rng.integers(0, M - clen_spec))
        k0 = float(rng.integers(8, nch - 8))
        span = float(rng.integers(20, 401)) * (1 if rng.random() < 0.5 else -1)
        k1 = min(max(k0 + span, 4.0), nch - 4.0)
        c0, clen = m0 * n_fft, clen_spec * n_fft
        chirps.append((c0, clen, k0 / n_fft, k1 / n_fft, _line_amp(snr(), sigma, n_fft),
                       float(rng.uniform(-np.pi, np.pi))))
        for m in range(m0, min(M, m0 + clen_spec + n_taps)):
            a = max(0, (m - 2) * n_fft - c0)
            b = min(clen, m * n_fft - c0)
            if a >= b:
                continue
            ka = k0 + (k1 - k0) * a / clen
            kb = k0 + (k1 - k0) * b / clen
            lo_k = int(math.floor(min(ka, kb) + 0.5))
            hi_k = int(math.floor(max(ka, kb) + 0.5))
            truth[m // spec_per_dump, max(0, lo_k):min(nch, hi_k + 1)] = 1
    spec = StreamSpec(n_ant, n_samp, seed, sigma=sigma, corr=corr, lags=lags, lines=lines, bursts=bursts,
                      period=n_fft, chirps=chirps)
    params = {"lags": lags, "line_snr": line_snr, "n_bursts": len(bursts), "chirps": chirps,
              "n_int": n_int, "n_chan": nch, "spec_per_dump": spec_per_dump, "n_fft": n_fft,
              "n_taps": n_taps}
    return spec, truth, params


# ---- synthetic interferometer observations for imaging --------------------

C_LIGHT = 299792458.0


@dataclass
class ImagingObs:
    u: np.ndarray        # float32 [n_vis], wavelengths
    v: np.ndarray        # float32 [n_vis]
    vis: np.ndarray      # complex64 [n_vis]
    sources: list        # [(flux, l, m)]
    n: int               # image size
    cell_rad: float      # image pixel


def imaging_obs(n_ant=4, n_chan=256, n_time=64, seed=5000, n=256, noise=0.0, sources=None,
                radius_m=60.0, f0_hz=1.30e9, bw_hz=1.0e8, lat_deg=36.7, dec_deg=58.8,
                ha_span_h=4.0):
    """Point sources observed by n_ant antennas at random positions within
    radius_m (east, north), over n_chan channels in [f0, f0 + bw) and n_time
    hour angles across ha_span_h hours (earth-rotation synthesis), at a
    source declination dec_deg from latitude lat_deg.  (u, v) per cross
    baseline i < j from the standard east-north to equatorial rotation.
    Visibilities V = sum_s F_s exp(-2 pi i (u l_s + v m_s)) plus complex
    Gaussian noise of rms `noise`.  The pixel size puts the longest
    projected baseline at n/4 cells (every cell and its mirror stay on the
    grid); the default sources sit on pixel centres."""
    rng = _rng(seed, 11, 0)
    rad = radius_m * np.sqrt(rng.uniform(0, 1, n_ant))
    ang = rng.uniform(0, 2 * np.pi, n_ant)
    east, north = rad * np.cos(ang), rad * np.sin(ang)
    lat, dec = np.radians(lat_deg), np.radians(dec_deg)
    ha = np.radians(15.0 * np.linspace(-ha_span_h / 2, ha_span_h / 2, n_time))
    freqs = f0_hz + (np.arange(n_chan) + 0.5) * (bw_hz / n_chan)
    us, vs = [], []
    for i in range(n_ant):
        for j in range(i + 1, n_ant):
            dE, dN = east[j] - east[i], north[j] - north[i]
            X, Y, Z = -np.sin(lat) * dN, dE, np.cos(lat) * dN
            u_m = np.sin(ha) * X + np.cos(ha) * Y
            v_m = -np.sin(dec) * np.cos(ha) * X + np.sin(dec) * np.sin(ha) * Y + np.cos(dec) * Z
            us.append(np.outer(u_m, freqs / C_LIGHT).ravel())
            vs.append(np.outer(v_m, freqs / C_LIGHT).ravel())
    u = np.concatenate(us).astype(np.float32)
    v = np.concatenate(vs).astype(np.float32)
    umax = float(max(np.abs(u).max(), np.abs(v).max()))
    cell = 1.0 / (4.0 * umax)          # |u| <= n/4 cells: every cell and mirror in range
    if sources is None:
        sources = [(1.0, 0.0, 0.0), (0.5, 12 * cell, -7 * cell), (0.3, -20 * cell, 15 * cell)]
    ud, vd = u.astype(np.float64), v.astype(np.float64)
    V = np.zeros(u.shape, np.complex128)
    for (F, l, m) in sources:
        V += F * np.exp(-2j * np.pi * np.mod(ud * l + vd * m, 1.0))
    if noise:
        V += noise * (rng.standard_normal(u.size) + 1j * rng.standard_normal(u.size)) / np.sqrt(2)
    return ImagingObs(u, v, V.astype(np.complex64), sources, n, cell)
