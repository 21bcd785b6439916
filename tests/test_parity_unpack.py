"""GPU parity: the F-engine and F+X over every input word (real int8 and
16-bit padded int16, complex int8 and int16 I/Q; Sec. 3.3 and Sec. 4.2),
and the prototype windows of Fig. pfb_fft (Kaiser-sinc, rectangular)
against the FP64 oracle.  Bars: channelised voltages 1e-5 of the channel
rms, visibilities 1e-5 of sqrt(V_ii V_jj) (float32 path), requantised paths
the significand bar of tests.util.quant_bar, scales and histories exact."""

import numpy as np
import pytest

import synth
from oracle import pfb, quant, xengine
from tests.util import quant_bar, vis_err

pytestmark = pytest.mark.gpu

TOL = 1e-5
WORDS = ["i8", "i16", "ci8", "ci16"]


def _stream(word, n_ant, n_samp, seed, **kw):
    bits = 14 if word.endswith("16") else 8
    sigma = 1200.0 if bits == 14 else 16.0
    spec = synth.StreamSpec(n_ant, n_samp, seed, sigma=sigma, corr=0.3,
                            lags=tuple(range(0, 3 * n_ant, 3))[:n_ant], bits=bits, **kw)
    return synth.generate_iq(spec) if word.startswith("c") else synth.generate(spec)


def _as_complex(x):
    return x[..., 0].astype(np.int64) + 1j * x[..., 1].astype(np.int64)


def _oracle_X(word, x, N, P, taps=None, hist=None, chans=None):
    if word.startswith("c"):
        h = None if hist is None else _as_complex(hist)
        return pfb.channelize_complex(_as_complex(x), N, P, taps=taps, hist=h, chans=chans)
    return pfb.channelize(x, N, P, taps=taps, hist=hist, chans=chans)


def _n_chan(word, N):
    return N if word.startswith("c") else N // 2


@pytest.mark.parametrize("word", WORDS)
@pytest.mark.parametrize("N,n_ant,P,n_spec", [(16, 3, 4, 37), (256, 4, 8, 21), (4096, 2, 4, 9),
                                              (1024, 1, 1, 12), (8192, 2, 2, 5)])
def test_channelize_any_word(qc, word, N, n_ant, P, n_spec):
    import torch
    x = _stream(word, n_ant, N * n_spec, seed=N + n_ant)
    rng = np.random.default_rng(N)
    keep = (P - 1) * N
    shape = (n_ant, keep, 2) if word.startswith("c") else (n_ant, keep)
    lim = 8000 if word.endswith("16") else 120
    hist = rng.integers(-lim, lim, shape).astype(x.dtype)
    xd = torch.from_numpy(x).cuda()
    hd = torch.from_numpy(hist).cuda() if keep else None
    hout = torch.empty_like(hd) if keep else None
    out, _ = qc.pfb_channelize_ex(xd, N, P, hist=hd, hist_out=hout)
    nch = _n_chan(word, N)
    assert tuple(out.shape) == (n_ant, n_spec, nch)
    X_ref = _oracle_X(word, x, N, P, hist=hist if keep else None)
    X = out.cpu().numpy()
    rms = np.sqrt(np.mean(np.abs(X_ref) ** 2))
    err = np.max(np.abs(X - X_ref)) / rms
    print(f"{word} N={N} P={P}: {err:.2e}")
    assert err <= TOL
    if keep:
        # the history for the next call: the last (P-1) N samples, exact
        full = np.concatenate([hist, x], axis=1)
        assert np.array_equal(hout.cpu().numpy(), full[:, full.shape[1] - keep:])


# The ring F-engine (P = 4, built-in taps, N = 1024..8192) for every word:
# several runs of spectra per antenna group (so runs start from in-stream
# history), partial last groups, a carried history, and the plain kernel's
# result beside it.  16-bit words at N = 8192 take the plain kernel.
@pytest.mark.parametrize("word", WORDS)
@pytest.mark.parametrize("N,n_ant,n_spec", [(4096, 5, 40), (2048, 3, 36), (1024, 7, 40), (8192, 3, 20)])
def test_channelize_ring_any_word(qc, word, N, n_ant, n_spec):
    import torch
    P = 4
    x = _stream(word, n_ant, N * n_spec, seed=5 * N + n_ant)
    rng = np.random.default_rng(N + 1)
    keep = (P - 1) * N
    shape = (n_ant, keep, 2) if word.startswith("c") else (n_ant, keep)
    lim = 8000 if word.endswith("16") else 120
    hist = rng.integers(-lim, lim, shape).astype(x.dtype)
    xd = torch.from_numpy(x).cuda()
    hd = torch.from_numpy(hist).cuda()
    assert qc.channelize_variant() == 0
    out, _ = qc.pfb_channelize_ex(xd, N, P, hist=hd)
    chans = np.unique(np.linspace(0, _n_chan(word, N) - 1, 40).astype(int))
    X_ref = _oracle_X(word, x, N, P, hist=hist, chans=chans)
    X = out.cpu().numpy()[:, :, chans]
    rms = np.sqrt(np.mean(np.abs(X_ref) ** 2))
    err = np.max(np.abs(X - X_ref)) / rms
    print(f"ring {word} N={N} ants={n_ant}: {err:.2e}")
    assert err <= TOL
    try:
        qc.channelize_variant(1)
        plain, _ = qc.pfb_channelize_ex(xd, N, P, hist=hd)
        torch.cuda.synchronize()
    finally:
        qc.channelize_variant(0)
    # two float32 paths (different FFT twiddle forms and rounding orders),
    # each about 1e-6 of the rms from the oracle
    assert np.max(np.abs(plain.cpu().numpy() - out.cpu().numpy())) / rms <= 5e-6


def test_i8_word_equals_plain_entry_point(qc):
    import torch
    x = _stream("i8", 4, 1024 * 20, seed=3)
    xd = torch.from_numpy(x).cuda()
    a, _ = qc.pfb_channelize_ex(xd, 1024, 4)
    b, _ = qc.pfb_channelize(xd, 1024, 4)
    X_ref = pfb.channelize(x, 1024, 4)
    rms = np.sqrt(np.mean(np.abs(X_ref) ** 2))
    assert np.max(np.abs(a.cpu().numpy() - X_ref)) / rms <= TOL
    assert np.max(np.abs(b.cpu().numpy() - X_ref)) / rms <= TOL
    V = qc.xcorrelate_ex(xd, 1024, 4, 10).cpu().numpy()
    W = qc.xcorrelate(xd, 1024, 4, 10).cpu().numpy()
    assert np.array_equal(V, W)


@pytest.mark.parametrize("word", ["i16", "ci8", "ci16"])
@pytest.mark.parametrize("N,n_ant,n_spec,spd", [(1024, 4, 40, 16), (64, 5, 33, 11), (256, 32, 12, 12)])
def test_xcorrelate_any_word(qc, word, N, n_ant, n_spec, spd):
    import torch
    x = _stream(word, n_ant, N * n_spec, seed=7 * N + n_ant)
    V = qc.xcorrelate_ex(torch.from_numpy(x).cuda(), N, 4, spd).cpu().numpy()
    assert V.shape == (n_spec // spd, n_ant * (n_ant + 1) // 2, _n_chan(word, N))
    V_ref = xengine.correlate_fast(_oracle_X(word, x, N, 4), spd)
    err = vis_err(V, V_ref, n_ant)
    print(f"{word} {n_ant} ant N={N}: {err:.2e}")
    assert err <= TOL
    for a in range(n_ant):
        b = a * n_ant - a * (a - 1) // 2
        assert np.all(V[:, b].imag == 0) and np.all(V[:, b].real >= 0)


# Real int16 words at a ring-tile shape take the fused F+X kernel (P = 4,
# built-in taps): several chunks per dump, a carried history, accumulation.
@pytest.mark.parametrize("N,n_ant,n_spec,spd", [(4096, 4, 24, 8), (4096, 2, 20, 10), (2048, 4, 30, 10),
                                                (1024, 4, 36, 12)])
def test_xcorrelate_i16_fused(qc, N, n_ant, n_spec, spd):
    import torch
    P = 4
    x = _stream("i16", n_ant, N * n_spec, seed=3 * N + n_ant)
    rng = np.random.default_rng(N + n_ant)
    hist = rng.integers(-8000, 8000, (n_ant, (P - 1) * N)).astype(np.int16)
    xd, hd = torch.from_numpy(x).cuda(), torch.from_numpy(hist).cuda()
    hout = torch.empty_like(hd)
    V = qc.xcorrelate_ex(xd, N, P, spd, hist=hd, hist_out=hout)
    V_ref = xengine.correlate_fast(pfb.channelize(x, N, P, hist=hist), spd)
    err = vis_err(V.cpu().numpy(), V_ref, n_ant)
    print(f"i16 fused {n_ant} ant N={N}: {err:.2e}")
    assert err <= TOL
    full = np.concatenate([hist, x], axis=1)
    assert np.array_equal(hout.cpu().numpy(), full[:, full.shape[1] - (P - 1) * N:])
    # accumulate adds onto what vis holds
    W = qc.xcorrelate_ex(xd, N, P, spd, hist=hd, vis=V.clone(), accumulate=True)
    torch.cuda.synchronize()
    assert np.max(np.abs(W.cpu().numpy() - 2 * V.cpu().numpy())) <= 1e-6 * np.abs(V_ref).max()


@pytest.mark.parametrize("word", ["i16", "ci8", "ci16"])
@pytest.mark.parametrize("prec", ["f16", "bf16", "fp8"])
def test_requantised_any_word(qc, word, prec):
    """Scales exactly the oracle's (|x|^2 power, power-of-two), and the
    requantised F+X on the matrix cores within the significand bar."""
    import torch
    n_ant, N, n_spec = 8, 256, 48
    x = _stream(word, n_ant, N * n_spec, seed=11)
    xd = torch.from_numpy(x).cuda()
    _, scale = qc.pfb_channelize_ex(xd, N, 4, out_prec=prec)
    qname = {"f16": "fp16", "bf16": "bf16", "fp8": "fp8"}[prec]
    xo = _as_complex(x) if word.startswith("c") else x
    s_ref = quant.pow2_scales(xo, pfb.hann_sinc_taps(N, 4), qname)
    assert np.array_equal(scale.cpu().numpy().astype(np.float64), s_ref)
    V = qc.xcorrelate_ex(xd, N, 4, n_spec, x_prec=prec).cpu().numpy()
    V_ref = xengine.correlate_fast(_oracle_X(word, x, N, 4), n_spec)
    err = vis_err(V, V_ref, n_ant)
    print(f"{word} {prec}: {err:.2e} (bar {quant_bar(prec, n_spec):.2e})")
    assert err <= quant_bar(prec, n_spec)


def test_complex_tone_signed_channels(qc):
    """I/Q tones at +37 and -37 channels (N = 256) land in channels 37 and
    219 on the GPU, as in the oracle, with >= 44 dB to the neighbours."""
    import torch
    N = 256
    for k0 in (37, -37):
        spec = synth.StreamSpec(1, N * 12, 9, sigma=0.0, corr=0.0, bits=14, tone_amp=6000.0,
                                tone_cycles_per_sample=(k0 % N) / N, period=N)
        x = synth.generate_iq(spec)
        X = qc.pfb_channelize_ex(torch.from_numpy(x).cuda(), N, 4)[0].cpu().numpy()[0, 3:]
        X_ref = _oracle_X("ci16", x, N, 4)[0, 3:]
        assert np.max(np.abs(X - X_ref)) <= 1e-6 * np.abs(X_ref).max()
        p = np.abs(X.astype(np.complex128)) ** 2
        k = k0 % N
        assert np.all(np.argmax(p, axis=1) == k)
        assert np.min(10 * np.log10(p[:, k] / np.maximum(p[:, (k + 1) % N], p[:, k - 1]))) >= 44.0


def test_any_word_rejects_bad_arguments(qc):
    import torch
    x = torch.zeros((2, 64, 2), dtype=torch.int16, device="cuda")
    lib = qc.lib()
    p = qc.PfbParams(16, 4, None, 0)
    import ctypes
    for sample, ld, n_samp in [(4, 64, 64), (3, 62, 64), (3, 64, 60), (-1, 64, 64)]:
        st = lib.qc_pfb_channelize_ex(ctypes.c_void_p(x.data_ptr()), sample, ld, 2, n_samp, ctypes.byref(p),
                                      None, None, 0, ctypes.c_void_p(x.data_ptr()), None, None)
        assert st == -1, (sample, ld, n_samp)
    # misaligned complex int16 rows (4 samples = 16 bytes)
    st = lib.qc_pfb_channelize_ex(ctypes.c_void_p(x.data_ptr() + 4), 3, 64, 2, 64, ctypes.byref(p), None, None,
                                  0, ctypes.c_void_p(x.data_ptr()), None, None)
    assert st == -1


# ---------------------------------------------------------------- windows ----

@pytest.mark.parametrize("window,N,P,beta", [("kaiser", 1024, 8, 8.0), ("kaiser", 64, 3, 5.0),
                                             ("hann", 256, 4, 0.0), ("rect", 128, 1, 0.0)])
def test_design_taps_match_oracle(qc, window, N, P, beta):
    taps = qc.design_taps(N, P, window, beta).cpu().numpy().astype(np.float64)
    ref = {"kaiser": lambda: pfb.kaiser_sinc_taps(N, P, beta), "hann": lambda: pfb.hann_sinc_taps(N, P),
           "rect": lambda: np.ones(N * P)}[window]()
    # designed in float64 and rounded once to float32
    assert np.max(np.abs(taps - ref)) <= 2.0 ** -24 * np.max(np.abs(ref))


@pytest.mark.parametrize("N,n_ant,n_spec,spd", [(1024, 4, 40, 20), (4096, 4, 24, 8), (512, 3, 30, 15)])
def test_kaiser_p8_fx_matches_oracle(qc, N, n_ant, n_spec, spd):
    """The 8-tap Kaiser (beta = 8) PFB of Fig. pfb_fft as user taps through
    the fused F+X (4 antennas) and the two-pass path (3 antennas)."""
    import torch
    x = _stream("i8", n_ant, N * n_spec, seed=N + 5)
    taps = qc.design_taps(N, 8, "kaiser", 8.0)
    h = taps.cpu().numpy().astype(np.float64)
    V = qc.xcorrelate(torch.from_numpy(x).cuda(), N, 8, spd, taps=taps).cpu().numpy()
    V_ref = xengine.correlate_fast(pfb.channelize(x, N, 8, taps=h), spd)
    assert vis_err(V, V_ref, n_ant) <= TOL


LEAK_OFFSETS = list(range(-10, 0)) + list(range(1, 11))


def leakage_db(X, k0):
    """Mean power at channels k0 + d (d = +-1..+-10) over that of the
    strongest channel, in dB (exact zeros, as a bin-centred tone gives
    through the plain FFT, read as -inf without a warning)."""
    p = np.mean(np.abs(np.asarray(X, np.complex128)) ** 2, axis=0)
    pk = p.max()
    with np.errstate(divide="ignore"):
        return np.array([10 * np.log10(p[(k0 + d) % p.size] / pk) for d in LEAK_OFFSETS])


@pytest.mark.parametrize("frac", [0.0, 0.25, 0.5])
def test_sidelobe_leakage_pfb_vs_fft(qc, frac):
    """Fig. pfb_fft as numbers: a complex 16-bit tone at channel 100 + frac
    (N = 1024) through the 8-tap Kaiser PFB and the plain FFT.  The GPU's
    leakage at +-1..+-10 channels equals the oracle's on the same samples
    (amplitude ratios within 2e-6 of the peak); the PFB leaks less than the
    FFT at every offset beyond the first for an off-bin tone."""
    import torch
    N, k0, M = 1024, 100, 24
    spec = synth.StreamSpec(1, N * M, 21, sigma=0.0, corr=0.0, bits=16, tone_amp=30000.0,
                            tone_cycles_per_sample=(k0 + frac) / N, period=4 * N)
    x = synth.generate_iq(spec)
    xd = torch.from_numpy(x).cuda()
    res = {}
    for name, P, taps in [("pfb", 8, qc.design_taps(N, 8, "kaiser", 8.0)), ("fft", 1, qc.design_taps(N, 1, "rect"))]:
        X = qc.pfb_channelize_ex(xd, N, P, taps=taps)[0].cpu().numpy()[0, P - 1:]
        X_ref = _oracle_X("ci16", x, N, P, taps=taps.cpu().numpy().astype(np.float64))[0, P - 1:]
        g, o = leakage_db(X, k0), leakage_db(X_ref, k0)
        # float32 spectra carry errors of ~1e-7 of the peak amplitude: the
        # leakage amplitudes (relative to the peak) agree within 2e-6
        assert np.all(np.abs(10 ** (g / 20) - 10 ** (o / 20)) <= 2e-6), (name, g, o)
        res[name] = o
    print(f"frac {frac}: pfb {np.round(res['pfb'], 1)}; fft {np.round(res['fft'], 1)}")
    if frac > 0:
        far = np.array([abs(d) >= 2 for d in LEAK_OFFSETS])
        assert np.all(res["pfb"][far] < res["fft"][far])
