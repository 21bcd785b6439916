"""Pins for the FP64 oracle: each check comes from outside the oracle.

Sources of truth used here: numpy/scipy library transforms reached by a
different route, closed forms, exact integer arithmetic, identities the
definitions imply (Parseval, Hermitian symmetry, Cauchy-Schwarz, PSD) and
statistics with derived error bars.  Runs on the CPU only.
"""

import math
import statistics

import numpy as np
import pytest
import scipy.signal

from oracle import calib, mad, pfb, quant, xengine

RNG = np.random.default_rng(12345)


# ---------------------------------------------------------------- taps ----

def test_taps_match_scipy_hann_times_sinc():
    for N, P in [(16, 4), (64, 3), (1024, 4)]:
        L = N * P
        h = pfb.hann_sinc_taps(N, P)
        w = scipy.signal.windows.hann(L, sym=True)
        q = np.arange(L)
        ref = w * np.sinc((q - (L - 1) / 2) / N)
        assert np.allclose(h, ref, rtol=0, atol=1e-15)
        assert np.allclose(h, h[::-1], atol=1e-15)          # symmetric
        assert h[0] == 0.0 and abs(h[-1]) < 1e-15            # Hann end zeros


# ----------------------------------------------------------- F-engine ----

@pytest.mark.parametrize("N,P,n_ant,M", [(16, 4, 2, 9), (32, 3, 3, 6), (8, 1, 1, 5)])
def test_pfb_equals_decimated_long_fft(N, P, n_ant, M):
    """X_m[k] = FFT_{PN}(h * segment)[P k]: the PFB is a long windowed DFT
    sampled every P bins (exp(-2pi i kq/N) = exp(-2pi i (Pk) q/(PN)))."""
    x = RNG.integers(-128, 128, (n_ant, M * N))
    h = pfb.hann_sinc_taps(N, P)
    X = pfb.channelize(x, N, P)
    xp = np.concatenate([np.zeros((n_ant, (P - 1) * N)), x], axis=1)
    for m in range(M):
        seg = xp[:, m * N:m * N + P * N]          # stream samples (m-P+1)N .. (m+1)N-1
        F = np.fft.fft(seg * h[None, :], axis=1)
        ref = F[:, ::P][:, :N // 2]
        assert np.allclose(X[:, m], ref, rtol=1e-12, atol=1e-9)


def test_p1_rectangular_is_rfft():
    N = 64
    x = RNG.integers(-128, 128, (2, 10 * N))
    X = pfb.channelize(x, N, 1, taps=np.ones(N), keep_nyquist=True)
    ref = np.fft.rfft(x.reshape(2, 10, N).astype(np.float64), axis=2)
    assert np.allclose(X, ref, rtol=1e-12, atol=1e-9)


def test_parseval_per_frame():
    N, P = 128, 4
    x = RNG.integers(-128, 128, (2, 12 * N))
    y = pfb.pfb_frames(x, N, P)
    X = pfb.dft(y, N, keep_nyquist=True)
    lhs = np.sum(y * y, axis=2)
    p = np.abs(X) ** 2
    rhs = (p[..., 0] + p[..., N // 2] + 2 * p[..., 1:N // 2].sum(axis=2)) / N
    assert np.allclose(lhs, rhs, rtol=1e-11)


def test_exact_integer_n4_ones_taps_by_hand():
    """N=4, P=2, all-ones taps: y = x[block m-1] + x[block m]; twiddles +-1, +-i."""
    x = np.array([[3, -1, 4, 1, -5, 9, 2, -6, 5, 3, -5, 8]])
    X = pfb.channelize(x, 4, 2, taps=np.ones(8), keep_nyquist=True)
    blocks = [[0, 0, 0, 0], [3, -1, 4, 1], [-5, 9, 2, -6], [5, 3, -5, 8]]
    for m in range(3):
        y = [blocks[m][n] + blocks[m + 1][n] for n in range(4)]
        want = [y[0] + y[1] + y[2] + y[3],
                complex(y[0] - y[2], -(y[1] - y[3])),
                y[0] - y[1] + y[2] - y[3]]
        assert np.allclose(X[0, m], want, atol=1e-12)


def test_tone_closed_form_and_isolation():
    """x = A cos(2 pi f0 n): for full windows,
    X_m[k] = (A/2)[e^{2pi i f0 s} H(k/N - f0) + e^{-2pi i f0 s} H(k/N + f0)],
    H(nu) = sum_q h[q] e^{-2pi i nu q}, s = (m-P+1)N (window start)."""
    N, P, A, kc, M = 256, 4, 16.0, 37, 8
    f0 = kc / N
    n = np.arange(M * N)
    x = A * np.cos(2 * np.pi * f0 * n)
    h = pfb.hann_sinc_taps(N, P)
    X = pfb.channelize(x[None, :], N, P)[0]
    q = np.arange(P * N)

    def H(nu):
        return np.sum(h * np.exp(-2j * np.pi * nu * q))

    for m in range(P - 1, M):
        s = (m - P + 1) * N
        for k in [kc - 2, kc - 1, kc, kc + 1, 100]:
            want = A / 2 * (np.exp(2j * np.pi * f0 * s) * H(k / N - f0)
                            + np.exp(-2j * np.pi * f0 * s) * H(k / N + f0))
            assert abs(X[m, k] - want) < 1e-8 * abs(X[m, kc])
    # the bin-centred tone sits in its channel with >40 dB to its neighbours
    p = np.abs(X[P - 1:]) ** 2
    assert np.all(10 * np.log10(p[:, kc] / p[:, kc + 1]) > 40)
    assert np.all(10 * np.log10(p[:, kc] / p[:, kc - 1]) > 40)


def test_int8_tone_rounding_bound():
    """Rounding a tone to int8 moves each channel by at most 0.5 * sum|h|."""
    N, P, A, kc = 1024, 4, 16.0, 137
    n = np.arange(8 * N)
    xf = A * np.cos(2 * np.pi * kc / N * n)
    xi = np.rint(xf)
    h = pfb.hann_sinc_taps(N, P)
    d = pfb.channelize(xi[None], N, P)[0] - pfb.channelize(xf[None], N, P)[0]
    assert np.max(np.abs(d)) <= 0.5 * np.sum(np.abs(h)) + 1e-9


def test_kaiser_taps_match_scipy_kaiser_times_sinc():
    for N, P, beta in [(16, 8, 8.0), (1024, 8, 8.0), (64, 3, 5.0)]:
        L = N * P
        h = pfb.kaiser_sinc_taps(N, P, beta)
        w = scipy.signal.windows.kaiser(L, beta, sym=True)
        ref = w * np.sinc((np.arange(L) - (L - 1) / 2) / N)
        assert np.allclose(h, ref, rtol=0, atol=1e-14)
        assert np.allclose(h, h[::-1], atol=1e-15)


def test_complex_p1_rectangular_is_numpy_fft():
    N = 64
    x = RNG.integers(-128, 128, (2, 10 * N)) + 1j * RNG.integers(-128, 128, (2, 10 * N))
    X = pfb.channelize_complex(x, N, 1, taps=np.ones(N))
    ref = np.fft.fft(x.reshape(2, 10, N), axis=2)
    assert np.allclose(X, ref, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("N,P", [(16, 4), (32, 8)])
def test_complex_pfb_equals_decimated_long_fft(N, P):
    M = 7
    x = RNG.integers(-9000, 9000, (2, M * N)) + 1j * RNG.integers(-9000, 9000, (2, M * N))
    h = pfb.kaiser_sinc_taps(N, P, 8.0)
    X = pfb.channelize_complex(x, N, P, taps=h)
    xp = np.concatenate([np.zeros((2, (P - 1) * N)), x], axis=1)
    for m in range(M):
        F = np.fft.fft(xp[:, m * N:m * N + P * N] * h[None, :], axis=1)
        assert np.allclose(X[:, m], F[:, ::P], rtol=1e-12, atol=1e-6)


def test_complex_is_linear_in_i_and_q_and_real_input_is_hermitian():
    N, P = 32, 4
    xi = RNG.integers(-128, 128, (3, 6 * N))
    xq = RNG.integers(-128, 128, (3, 6 * N))
    allk = np.arange(N)
    Xc = pfb.channelize_complex(xi + 1j * xq, N, P)
    Xi = pfb.channelize(xi, N, P, chans=allk)
    Xq = pfb.channelize(xq, N, P, chans=allk)
    assert np.allclose(Xc, Xi + 1j * Xq, rtol=1e-12, atol=1e-8)
    # real input: X[N-k] = conj X[k]; the first N/2 channels are the real path's
    Xr = pfb.channelize_complex(xi + 0j, N, P)
    assert np.allclose(Xr[..., 1:][..., ::-1], np.conj(Xr[..., 1:]), atol=1e-8)
    assert np.allclose(Xr[..., :N // 2], pfb.channelize(xi, N, P), atol=1e-8)


@pytest.mark.parametrize("k0", [37, -37])
def test_complex_tone_lands_in_its_signed_channel(k0):
    """exp(2 pi i k0 n / N) lands in channel k0 mod N: negative frequencies
    occupy k >= N/2, with >= 44 dB to the neighbours (Hann-sinc, P = 4)."""
    N, P = 256, 4
    n = np.arange(8 * N)
    x = np.rint(8000 * np.exp(2j * np.pi * k0 * n / N).real) + 1j * np.rint(8000 * np.exp(2j * np.pi * k0 * n / N).imag)
    X = pfb.channelize_complex(x[None], N, P)[0, P - 1:]
    k = k0 % N
    p = np.abs(X) ** 2
    assert np.all(np.argmax(p, axis=1) == k)
    assert np.all(10 * np.log10(p[:, k] / p[:, (k + 1) % N]) > 44)
    assert np.all(10 * np.log10(p[:, k] / p[:, (k - 1) % N]) > 44)


def test_int16_exact_integer_n4_by_hand():
    """16-bit padded samples enter as the integers they are."""
    x = np.array([[8191, -8192, 4000, 1, -7000, 9, 2, -6]], np.int16)
    X = pfb.channelize(x, 4, 2, taps=np.ones(8), keep_nyquist=True)
    b = [[0, 0, 0, 0], [8191, -8192, 4000, 1], [-7000, 9, 2, -6]]
    for m in range(2):
        y = [b[m][n] + b[m + 1][n] for n in range(4)]
        want = [sum(y), complex(y[0] - y[2], -(y[1] - y[3])), y[0] - y[1] + y[2] - y[3]]
        assert np.allclose(X[0, m], want, atol=1e-9)


def test_rectangular_half_bin_leakage_is_the_dirichlet_kernel():
    """A complex tone half a bin above channel k0 through the plain FFT: the
    power at channel k0 + d relative to channel k0 is
    |D(d - 1/2)|^2 / |D(-1/2)|^2 with D(v) = sin(pi v) / sin(pi v / N)."""
    N, k0 = 128, 40
    n = np.arange(4 * N)
    x = np.exp(2j * np.pi * (k0 + 0.5) * n / N)
    X = pfb.channelize_complex(x[None], N, 1, taps=pfb.rect_taps(N))[0]
    p = np.mean(np.abs(X) ** 2, axis=0)

    def D(v):
        return np.sin(np.pi * v) / np.sin(np.pi * v / N)

    for d in list(range(-10, 0)) + list(range(1, 11)):
        want = (D(d - 0.5) / D(-0.5)) ** 2
        assert p[k0 + d] / p[k0] == pytest.approx(want, rel=1e-9)


def test_pow2_scale_complex_reduces_to_real():
    x = RNG.integers(-300, 300, (2, 1 << 12))
    h = pfb.hann_sinc_taps(64, 4)
    assert np.array_equal(quant.pow2_scales(x + 0j, h, "fp16"), quant.pow2_scales(x, h, "fp16"))
    # doubling |x| halves the scale
    assert np.array_equal(quant.pow2_scales(2 * x + 2j * x, h, "fp8"),
                          quant.pow2_scales(x + 1j * x, h, "fp8") / 2)


def test_history_carry_equals_one_shot():
    N, P = 32, 4
    x = RNG.integers(-128, 128, (3, 20 * N))
    full = pfb.channelize(x, N, P)
    cut = 7 * N
    hist = pfb.stream_history(x[:, :cut], N, P)
    second = pfb.channelize(x[:, cut:], N, P, hist=hist)
    assert np.array_equal(full[:, 7:], second)


def test_channel_subset_matches_full():
    N, P = 64, 4
    x = RNG.integers(-128, 128, (2, 6 * N))
    full = pfb.channelize(x, N, P)
    sub = pfb.channelize(x, N, P, chans=[0, 5, 31])
    assert np.allclose(full[:, :, [0, 5, 31]], sub, rtol=0, atol=1e-9)


# ----------------------------------------------------------- X-engine ----

def _random_X(n_ant, M, C):
    return RNG.normal(size=(n_ant, M, C)) + 1j * RNG.normal(size=(n_ant, M, C))


def test_xengine_matches_gram_matrix_route():
    X = _random_X(5, 12, 7)
    V = xengine.correlate(X, 4)
    pairs = xengine.baseline_pairs(5)
    for d in range(3):
        seg = X[:, 4 * d:4 * d + 4, :]
        for k in range(7):
            G = seg[:, :, k] @ seg[:, :, k].conj().T          # G_ij = sum_m X_i X_j*
            for b, (i, j) in enumerate(pairs):
                assert abs(V[d, b, k] - G[i, j]) < 1e-10


@pytest.mark.parametrize("n_ant,M,C,D", [(1, 7, 5, 3), (4, 11, 9, 4), (32, 5, 3, 2), (3, 9, 4, 9),
                                         (2, 4, 6, 5)])
def test_correlate_fast_equals_explicit_mac(n_ant, M, C, D):
    """The vectorised sum over a dump is the explicit per-spectrum MAC of
    correlate(): same pairs, same conjugated operand, same dropped tail
    (ragged M), autos exactly real.  correlate() is pinned by the Gram,
    Hermitian and PSD tests, so correlate_fast inherits those pins."""
    X = _random_X(n_ant, M, C) * 37.0
    Vf = xengine.correlate_fast(X, D)
    V = xengine.correlate(X, D)
    assert Vf.shape == V.shape == (M // D, n_ant * (n_ant + 1) // 2, C)
    assert np.allclose(Vf, V, rtol=0, atol=1e-12 * np.abs(V).max() if V.size else 0)
    for a in range(n_ant):
        assert np.all(Vf[:, xengine.baseline_index(a, a, n_ant)].imag == 0)
    # the conjugate falls on the second antenna: V_01 = sum X_0 conj(X_1)
    if n_ant >= 2 and M >= D:
        ref = np.sum(X[0, :D] * np.conj(X[1, :D]), axis=0)
        assert np.allclose(Vf[0, 1], ref, rtol=0, atol=1e-9)
        assert not np.allclose(Vf[0, 1], np.conj(ref), rtol=0, atol=1e-9)


def test_xengine_hermitian_autos_cauchy_schwarz_psd():
    n_ant = 6
    X = _random_X(n_ant, 20, 9)
    V = xengine.correlate(X, 20)[0]
    Vr = xengine.correlate(X[::-1], 20)[0]
    pairs = xengine.baseline_pairs(n_ant)
    bidx = {p: b for b, p in enumerate(pairs)}
    for b, (i, j) in enumerate(pairs):
        # reversed order maps (i, j) to (n-1-j, n-1-i) with conjugation
        rb = bidx[(n_ant - 1 - j, n_ant - 1 - i)]
        assert np.allclose(Vr[rb], np.conj(V[b]), atol=1e-10)
        if i == j:
            assert np.all(V[b].imag == 0) and np.all(V[b].real >= 0)
    for k in range(9):
        G = np.zeros((n_ant, n_ant), complex)
        for b, (i, j) in enumerate(pairs):
            G[i, j] = V[b, k]
            G[j, i] = np.conj(V[b, k])
        assert np.min(np.linalg.eigvalsh(G)) > -1e-9
        for i in range(n_ant):
            for j in range(n_ant):
                assert abs(G[i, j]) ** 2 <= G[i, i].real * G[j, j].real * (1 + 1e-12)


def test_baseline_index_formula():
    for n in [1, 2, 4, 7, 32]:
        for b, (i, j) in enumerate(xengine.baseline_pairs(n)):
            assert xengine.baseline_index(i, j, n) == b
        assert len(xengine.baseline_pairs(n)) == n * (n + 1) // 2


def test_partial_dump_is_dropped():
    X = _random_X(2, 10, 3)
    V = xengine.correlate(X, 4)
    assert V.shape == (2, 3, 3)


def test_noise_auto_expectation():
    """E[V_ii[k]] = M sigma^2 sum h^2 for white input (no rounding)."""
    N, P, M = 64, 4, 400
    sig = 3.0
    x = sig * RNG.normal(size=(1, (M + P) * N))
    X = pfb.channelize(x, N, P)[:, P:]
    V = xengine.correlate(X, M - P)[0, 0].real
    h = pfb.hann_sinc_taps(N, P)
    expect = (M - P) * sig ** 2 * np.sum(h ** 2)
    # each channel is a chi-square with 2(M-P) dof; mean over 31 channels
    est = V[1:].mean()
    assert abs(est / expect - 1) < 4 / math.sqrt((M - P) * 31)


def test_delay_phase_slope():
    """A common component lagged by d_i, d_j gives E[V_ij[k]] ~ R e^{-2pi i k (d_i-d_j)/N}."""
    N, P, M = 128, 4, 300
    c = RNG.normal(size=M * N + 64)
    d = (0, 5)
    x = np.stack([c[64 - d[0]:64 - d[0] + M * N], c[64 - d[1]:64 - d[1] + M * N]])
    X = pfb.channelize(x, N, P)[:, P:]
    V = xengine.correlate(X, M - P)[0]
    k = np.arange(4, 60)
    ph = np.angle(V[1, k] * np.exp(2j * np.pi * k * (d[0] - d[1]) / N))
    # after removing the predicted slope the phase is flat at ~0
    assert np.max(np.abs(ph)) < 0.2
    assert abs(np.mean(ph)) < 0.03


# ---------------------------------------------------------------- MAD ----

def test_median_sorted_matches_statistics_median():
    for n in [1, 2, 3, 10, 11, 1000]:
        v = RNG.normal(size=n)
        assert mad.median_sorted(v) == statistics.median(v.tolist())


@pytest.mark.parametrize("n", [1, 2, 7, 8, 101, 1000])
def test_mad_closed_form_one_to_n(n):
    """A = 1..n: med = (n+1)/2; deviations |i - med|, their median closed form."""
    A = np.arange(1, n + 1, dtype=np.float64)
    med, m, T = mad.mad_threshold(A, 5.0)
    assert med == (n + 1) / 2
    # deviations: for odd n: 0,1,1,2,2,...; for even n: .5,.5,1.5,1.5,...
    if n % 2:
        devs = sorted([0] + [v for v in range(1, (n - 1) // 2 + 1) for _ in (0, 1)])
    else:
        devs = sorted([v + 0.5 for v in range(n // 2) for _ in (0, 1)])
    assert m == statistics.median(devs)
    assert T == med + (5.0 * 1.4826) * m


def test_mad_flags_outliers_and_affine_invariance():
    A = np.abs(RNG.normal(size=(1, 1, 4000))).astype(np.float32)
    A[0, 0, [10, 500, 3000]] = 50.0
    vis = A.astype(np.complex64)
    m1, T1 = mad.mad_flag(vis, 5.0, 0)
    assert set(np.flatnonzero(m1)) >= {10, 500, 3000}
    # exact affine map: alpha a power of two, beta chosen so sums stay exact
    m2, _ = mad.mad_flag((A * 4 + 0).astype(np.complex64), 5.0, 0)
    assert np.array_equal(m1, m2)
    # strict '>' : a value exactly at T is not flagged
    med, madv, T = mad.mad_threshold(np.array([1.0, 2.0, 3.0, 4.0, 5.0]), 0.0)
    assert T == 3.0
    mk, _ = mad.mad_flag(np.array([1, 2, 3, 4, 5], np.complex64).reshape(1, 1, 5), 0.0, 0)
    assert mk.ravel().tolist() == [0, 0, 0, 1, 1]


def test_mad_populations_shapes():
    vis = (RNG.normal(size=(5, 3, 4)) + 1j * RNG.normal(size=(5, 3, 4))).astype(np.complex64)
    for pop, tshape in [(0, (3,)), (1, (3, 4)), (2, (5, 3))]:
        mk, T = mad.mad_flag(vis, 3.0, pop)
        assert mk.shape == vis.shape and T.shape == tshape


def test_amplitude_is_correctly_rounded():
    v = np.array([3 + 4j, 1e-3 + 2e-3j, -7.5 + 0j], np.complex64)
    a = mad.amplitude_f32(v)
    assert a[0] == np.float32(5.0) and a[2] == np.float32(7.5)
    assert a[1] == np.float32(math.hypot(float(np.float32(1e-3)), float(np.float32(2e-3))))


# --------------------------------------------------------- delay/phase ----

def test_apply_identity_inverse_autos():
    n_ant, C = 4, 16
    V = (RNG.normal(size=(2, 10, C)) + 1j * RNG.normal(size=(2, 10, C)))
    z = calib.apply_delay_phase(V, n_ant, 0.0, 1e6, np.zeros(n_ant), np.zeros(n_ant))
    assert np.array_equal(z, V)
    tau = RNG.uniform(0, 40e-9, n_ant)
    phi = RNG.uniform(-np.pi, np.pi, n_ant)
    W = calib.apply_delay_phase(V, n_ant, 1.3e9, 0.25e6, tau, phi)
    back = calib.apply_delay_phase(W, n_ant, 1.3e9, 0.25e6, -tau, -phi)
    assert np.allclose(back, V, atol=1e-9)
    for b, (i, j) in enumerate(xengine.baseline_pairs(n_ant)):
        if i == j:
            assert np.allclose(W[:, b], V[:, b], atol=0)


def test_apply_before_x_equals_after_x():
    """Rotating each antenna's voltages by e^{i(2pi f tau_a + phi_a)} before
    correlating equals rotating the visibilities afterwards."""
    n_ant, C, M = 4, 24, 6
    f0, df = 1.3e9, 2.5e6
    X = _random_X(n_ant, M, C)
    tau = RNG.uniform(0, 40e-9, n_ant)
    phi = RNG.uniform(-np.pi, np.pi, n_ant)
    f = f0 + df * np.arange(C)
    rot = np.exp(1j * (2 * np.pi * f[None, :] * tau[:, None] + phi[:, None]))
    before = xengine.correlate(X * rot[:, None, :], M)
    after = calib.apply_delay_phase(xengine.correlate(X, M), n_ant, f0, df, tau, phi)
    assert np.allclose(before, after, atol=1e-9)


def test_lag_is_cancelled_by_tau_equal_lag_over_fs():
    """An injected integer lag d_a (samples) is removed by tau_a = d_a/fs."""
    N, P, M = 128, 4, 200
    fs = 1e9
    c = RNG.normal(size=M * N + 64)
    d = (0, 9)
    x = np.stack([c[64 - v:64 - v + M * N] for v in d])
    V = xengine.correlate(pfb.channelize(x, N, P)[:, P:], M - P)
    W = calib.apply_delay_phase(V, 2, 0.0, fs / N, np.array(d) / fs, np.zeros(2))
    ph = np.angle(W[0, 1, 5:58])
    assert np.max(np.abs(ph)) < 0.2


def test_solve_recovers_noiseless_delay_and_phase():
    n_ant, C = 5, 512
    f0, df = 1.3e9, 1e9 / 4096
    tau = np.array([0.0, 13.3e-9, -7.1e-9, 25.0e-9, 38.9e-9])
    phi = np.array([0.0, 0.4, -2.0, 2.9, -0.7])
    f = f0 + df * np.arange(C)
    pairs = xengine.baseline_pairs(n_ant)
    V = np.zeros((3, len(pairs), C), complex)
    for b, (i, j) in enumerate(pairs):
        V[:, b] = np.exp(-1j * (2 * np.pi * f * (tau[i] - tau[j]) + (phi[i] - phi[j])))
    t, p = calib.solve_delay_phase(V, None, n_ant, f0, df, 0, 40, 480)
    assert np.allclose(t, tau, atol=1e-15)
    assert np.allclose(calib.wrap(p - phi), 0, atol=1e-9)
    # and applying the solution flattens every cross baseline
    W = calib.apply_delay_phase(V, n_ant, f0, df, t, p)
    assert np.allclose(np.angle(W), 0, atol=1e-7)


def test_delay_spectrum_is_scaled_inverse_fft_of_padded_spectrum():
    """D[l] = sum_k V[k] e^{+2 pi i k l / L} is L * ifft of V zero-padded to L
    (numpy's inverse FFT carries the + sign and a 1/L factor)."""
    for C, L in [(7, 16), (64, 256), (100, 128)]:
        Vb = RNG.normal(size=C) + 1j * RNG.normal(size=C)
        ref = L * np.fft.ifft(np.concatenate([Vb, np.zeros(L - C)]))
        assert np.allclose(calib.delay_spectrum(Vb, L), ref, rtol=0, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("lag", [0, 1, 5, -3, -500, 511, -512, 300])
def test_coarse_delay_recovers_on_grid_delays_both_signs(lag):
    """A noiseless V[k] = exp(-2 pi i f_k tau) with tau = lag / (L df) on the
    delay grid peaks exactly at that lag (|D| = C there, < C elsewhere);
    the grid covers lags -L/2 .. L/2 - 1."""
    C = 256
    L = calib.lag_grid(C)
    f0, df = 1.3e9, 1e9 / 4096
    tau = lag / (L * df)
    Vb = np.exp(-2j * np.pi * (f0 + df * np.arange(C)) * tau + 0.7j)
    assert calib.coarse_delay(Vb, df, L) == pytest.approx(tau, abs=1e-6 / (L * df))


def test_coarse_delay_off_grid_is_nearest_lag():
    C, f0, df = 512, 0.2e9, 1e9 / 1024
    L = calib.lag_grid(C)
    for frac in [-0.49, -0.3, -0.01, 0.2, 0.37, 0.48]:
        tau = frac / df
        Vb = np.exp(-2j * np.pi * (f0 + df * np.arange(C)) * tau)
        tc = calib.coarse_delay(Vb, df, L)
        assert abs(tc - tau) <= 0.5 / (L * df) + 1e-18


def _steep_noisy(n_ant, C, f0, df, tau, phi, seed, amp=0.35 * np.pi):
    """Cross phases with a slope of up to 0.94 pi per channel plus bounded
    phase noise: unwrapping without the coarse step mistracks."""
    rng = np.random.default_rng(seed)
    pairs = xengine.baseline_pairs(n_ant)
    f = f0 + df * np.arange(C)
    V = np.zeros((2, len(pairs), C), complex)
    for b, (i, j) in enumerate(pairs):
        eps = rng.uniform(-amp, amp, C) if i != j else 0.0
        V[:, b] = np.exp(-1j * (2 * np.pi * f * (tau[i] - tau[j]) + (phi[i] - phi[j])) + 1j * eps)
    return V


def test_solve_needs_the_coarse_step_on_steep_noisy_phases():
    """Sec. 7 step 1 matters once the per-channel phase step plus noise
    passes pi: baseline (1, 2) steps 0.92 pi per channel (every baseline
    stays inside the delay grid, |dtau df| < 1/2) and the noise moves each
    step by up to 0.7 pi.  The coarse step removes the slope to within one
    lag cell first, so the fine fit unwraps correctly; without it (or with
    its transform's sign flipped) the unwrap mistracks and tau is off by
    microseconds."""
    n_ant, C = 4, 512
    f0, df = 1.3e9, 1e9 / 4096
    tau = np.array([0.0, 0.22, -0.24, 0.1]) / df
    phi = np.array([0.0, 1.1, -2.5, 0.3])
    V = _steep_noisy(n_ant, C, f0, df, tau, phi, seed=7)
    # the raw phase steps of baseline (1, 2) do pass pi
    b12 = xengine.baseline_index(1, 2, n_ant)
    assert np.any(np.abs(np.diff(np.angle(V[0, b12, 40:480]))) > np.pi)
    t, p = calib.solve_delay_phase(V, None, n_ant, f0, df, 0, 40, 480)
    assert np.max(np.abs(t - tau)) < 0.5e-9
    # each baseline's own (tau, phi) flattens its band (the per-antenna fit
    # spreads the baselines' tau scatter, which 2 pi f0 turns into phase)
    f = f0 + df * np.arange(C)
    for b, (i, j) in enumerate(xengine.baseline_pairs(n_ant)):
        if i != j:
            tb, pb = calib.solve_baseline(V.sum(axis=0)[b], f0, df, 40, 480)
            assert abs(tb - (tau[i] - tau[j])) < 0.5e-9
            W = V[0, b, 40:480] * np.exp(1j * (2 * np.pi * f[40:480] * tb + pb))
            assert abs(np.angle(W.sum())) < 0.05


# -------------------------------------------------------------- quant ----

def test_fp16_matches_numpy_half():
    v = RNG.normal(scale=300, size=20000)
    assert np.array_equal(quant.to_fp16(v), v.astype(np.float16).astype(np.float64))
    assert quant.to_fp16(np.array([1e6]))[0] == 65504.0


def test_bf16_and_e4m3_match_torch_casts():
    torch = pytest.importorskip("torch")
    v = RNG.normal(scale=50, size=20000).astype(np.float32)
    t = torch.from_numpy(v)
    assert np.array_equal(quant.to_bf16(v), t.to(torch.bfloat16).to(torch.float64).numpy())
    vin = v[np.abs(v) < 440]
    e = torch.from_numpy(vin).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(quant.to_e4m3(vin), e)
    assert quant.to_e4m3(np.array([1000.0, -449.0]))[0] == 448.0
    assert quant.to_e4m3(np.array([-449.0]))[0] == -448.0


def test_e4m3_grid_and_ties():
    # representable values near 1: step 1/8; tie 1 + 1/16 rounds to even (1.0)
    assert quant.to_e4m3(np.array([1.0625]))[0] == 1.0
    assert quant.to_e4m3(np.array([1.1875]))[0] == 1.25
    # subnormal step 2^-9
    assert quant.to_e4m3(np.array([2.0 ** -9 * 1.4]))[0] == 2.0 ** -9


def test_pow2_scale():
    x = RNG.integers(-40, 40, (3, 1 << 12))
    h = pfb.hann_sinc_taps(64, 4)
    s = quant.pow2_scales(x, h, "fp8")
    rms = np.sqrt(np.mean(x.astype(float) ** 2, axis=1) * np.sum(h ** 2))
    for a in range(3):
        e = np.log2(s[a])
        assert e == int(e) and abs(np.log2(32 / rms[a]) - e) <= 0.5
