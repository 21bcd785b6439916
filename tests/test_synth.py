"""The seeded stream generator: deterministic, chunk- and thread-invariant,
and with the statistics its recipe states."""

import numpy as np

import synth


def test_deterministic_and_thread_invariant():
    spec, _ = synth.realtime_spec(1 << 23, 2000)
    a = synth.generate(spec, threads=1)
    b = synth.generate(spec, threads=4)
    assert np.array_equal(a, b)
    spec2, _ = synth.realtime_spec(1 << 23, 2001)
    assert not np.array_equal(a, synth.generate(spec2, threads=2))


def test_prefix_is_a_prefix():
    """A shorter stream of the same recipe equals the longer one's prefix
    (chunks are seeded by index, not by length)."""
    s1 = synth.array_spec(3, 1 << 23, 7, corr=0.3, max_lag=9)
    s2 = synth.array_spec(3, 1 << 22, 7, corr=0.3, max_lag=9)
    assert np.array_equal(synth.generate(s1)[:, :1 << 22], synth.generate(s2))


def test_noise_and_correlation_statistics():
    spec = synth.StreamSpec(2, 1 << 22, 11, sigma=16.0, corr=0.3, lags=(0, 5))
    x = synth.generate(spec).astype(np.float64)
    var = x.var(axis=1)
    # sigma^2 (1 + corr) plus the rounding variance 1/12
    assert np.allclose(var, 256 * 1.3 + 1 / 12, rtol=0.01)
    # the common component appears at the injected relative lag
    r5 = np.mean(x[0, :-5] * x[1, 5:]) / np.sqrt(var[0] * var[1])
    r0 = np.mean(x[0] * x[1]) / np.sqrt(var[0] * var[1])
    assert abs(r5 - 0.3 / 1.3) < 0.01 and abs(r0) < 0.01


def test_tone_is_bin_centred():
    spec = synth.tone_stream(4, 1 << 16, 1000, 1024, 137)
    x = synth.generate(spec).astype(np.float64)
    p = np.abs(np.fft.rfft(x[0, :1024 * 32])) ** 2
    assert np.argmax(p[1:]) + 1 == 137 * 32


def test_realtime_recipe():
    spec, params = synth.realtime_spec(1 << 24, 2000)
    assert len(params["line_chans"]) == 20 and len(set(params["line_chans"])) == 20
    M = (1 << 24) // 4096
    covered = sum(b[1] // 4096 for b in params["bursts"])
    assert covered >= 0.05 * M
    assert all(0 <= l <= 40 for l in params["lags"])
    assert np.allclose(params["tau_s"], np.array(params["lags"]) * 1e-9)


def test_rfi_realisation_truth_and_determinism():
    spec, truth, params = synth.rfi_realisation(3, n_ant=2, n_samp=1 << 20, n_lines=3, n_chirps=1,
                                                burst_frac=0.02)
    n_int = (1 << 20) // 4096 // 16
    assert truth.shape == (n_int, 2048) and truth.dtype == np.uint8
    # every line channel is flagged in every integration
    for (f, amp, ph) in spec.lines:
        assert truth[:, int(round(f * 4096))].all()
    # bursts flag whole integrations
    full = truth.all(axis=1)
    assert full.any() and params["n_bursts"] >= 1
    a = synth.generate(spec)
    b = synth.generate(spec)
    assert np.array_equal(a, b)
    spec2, truth2, _ = synth.rfi_realisation(3, n_ant=2, n_samp=1 << 20, n_lines=3, n_chirps=1,
                                             burst_frac=0.02)
    assert np.array_equal(truth, truth2)


def test_chirp_instantaneous_frequency():
    """A lone chirp: phase increments sweep linearly from f0 to f1."""
    L = 1 << 16
    spec = synth.StreamSpec(1, L, 1, sigma=0.0, corr=0.0, chirps=[(0, L, 0.01, 0.05, 100.0, 0.3)])
    x = synth.generate(spec, threads=1).astype(np.float64)[0]
    # zero crossings per unit time ~ 2 f: count them in a window at the start and end
    def freq(seg):
        return np.count_nonzero(np.diff(np.signbit(seg))) / (2.0 * seg.size)
    assert abs(freq(x[:4096]) - (0.01 + 0.04 * 2048 / L)) < 2e-3
    assert abs(freq(x[-4096:]) - (0.05 - 0.04 * 2048 / L)) < 2e-3
