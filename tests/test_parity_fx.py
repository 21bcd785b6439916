"""GPU parity: F-engine, fused F+X and the two-pass F -> X path against the
FP64 oracle.  Bar for the FP32 path: max |V - V_ref| / sqrt(V_ii V_jj) <= 1e-5."""

import numpy as np
import pytest

import synth
from oracle import pfb, xengine
from tests.util import vis_err

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _stream(n_ant, n_samp, seed, corr=0.3):
    spec = synth.array_spec(n_ant, n_samp, seed, corr=corr, max_lag=9)
    return synth.generate(spec)


def _chans(N, n=48, seed=0):
    nch = N // 2
    if nch <= 96:
        return np.arange(nch)
    rng = np.random.default_rng(seed)
    pick = set(rng.choice(nch, n, replace=False).tolist()) | {0, 1, nch // 2, nch - 2, nch - 1}
    return np.array(sorted(pick))


def _oracle_vis(x, N, P, spd, hist=None, chans=None):
    X = pfb.channelize(x, N, P, hist=hist, chans=chans)
    return xengine.correlate_fast(X, spd)


def _gpu_vis(qc, x, N, P, spd, **kw):
    import torch
    xd = torch.from_numpy(x).cuda()
    V = qc.xcorrelate(xd, N, P, spd, **kw)
    torch.cuda.synchronize()
    return V.cpu().numpy()


# (n_fft, n_ant, n_spec, spec_per_dump): fused shapes (4 and 8 antennas, pairs),
# and two-pass shapes (odd antenna counts, small and large N); ragged dumps
# (trailing spectra not a multiple of spec_per_dump) included.
CASES = [
    (1024, 4, 37, 12),
    (1024, 4, 1024, 1024),     # plain-FX shape, full length
    (4096, 4, 41, 16),
    (4096, 4, 70, 35),
    (2048, 4, 30, 10),
    (512, 4, 66, 33),
    (1024, 8, 20, 10),
    (2048, 8, 21, 7),
    (1024, 2, 23, 23),
    (4096, 2, 17, 8),
    (16, 3, 50, 7),
    (4, 5, 40, 9),
    (64, 1, 33, 11),
    (256, 6, 24, 24),
    (8192, 4, 10, 5),
    (128, 32, 20, 10),
]


@pytest.mark.parametrize("N,n_ant,n_spec,spd", CASES)
def test_xcorrelate_matches_oracle(qc, N, n_ant, n_spec, spd):
    P = 4
    x = _stream(n_ant, N * n_spec, seed=11 + N + n_ant)
    chans = _chans(N)
    V_ref = _oracle_vis(x, N, P, spd, chans=chans)
    V = _gpu_vis(qc, x, N, P, spd)
    assert V.shape == (n_spec // spd, n_ant * (n_ant + 1) // 2, N // 2)
    V = V[:, :, chans]
    err = vis_err(V, V_ref, n_ant)
    assert err <= TOL, err
    # autos: exactly real, non-negative
    for a in range(n_ant):
        b = a * n_ant - a * (a - 1) // 2
        assert np.all(V[:, b].imag == 0) and np.all(V[:, b].real >= 0)


@pytest.mark.parametrize("N,n_ant,P", [(1024, 4, 4), (64, 3, 2), (4096, 2, 8), (16, 4, 1)])
def test_channelize_f32_matches_oracle(qc, N, n_ant, P):
    import torch
    n_spec = 19
    x = _stream(n_ant, N * n_spec, seed=5 + N)
    chans = _chans(N)
    X_ref = pfb.channelize(x, N, P, chans=chans)
    out, _ = qc.pfb_channelize(torch.from_numpy(x).cuda(), N, P)
    X = out.cpu().numpy()[:, :, chans]
    rms = np.sqrt(np.mean(np.abs(X_ref) ** 2))
    assert np.max(np.abs(X - X_ref)) / rms <= TOL


def test_user_taps(qc):
    import torch
    N, P, n_ant = 256, 3, 4
    x = _stream(n_ant, N * 20, seed=3)
    taps = np.random.default_rng(1).normal(size=N * P).astype(np.float32)
    V_ref = xengine.correlate_fast(pfb.channelize(x, N, P, taps=taps.astype(np.float64)), 20)
    V = _gpu_vis(qc, x, N, P, 20, taps=torch.from_numpy(taps).cuda())
    assert vis_err(V, V_ref, n_ant) <= TOL


@pytest.mark.parametrize("N,n_ant", [(1024, 4), (4096, 4), (64, 3)])
def test_history_carry_equals_one_shot(qc, N, n_ant):
    import torch
    P, spd = 4, 8
    x = _stream(n_ant, N * 48, seed=21)
    cut = N * 24
    xd = torch.from_numpy(x).cuda()
    hist = torch.zeros((n_ant, (P - 1) * N), dtype=torch.int8, device="cuda")
    v1 = qc.xcorrelate(xd[:, :cut].contiguous(), N, P, spd, hist_out=hist)
    v2 = qc.xcorrelate(xd[:, cut:].contiguous(), N, P, spd, hist=hist)
    one = qc.xcorrelate(xd, N, P, spd)
    both = torch.cat([v1, v2]).cpu().numpy()
    # identical arithmetic: same spectra, same partial grouping per dump
    assert vis_err(both, one.cpu().numpy(), n_ant) <= 1e-6
    V_ref = _oracle_vis(x, N, P, spd, chans=_chans(N))
    assert vis_err(both[:, :, _chans(N)], V_ref, n_ant) <= TOL
    # the history output is exactly the last (P-1)N input samples
    assert np.array_equal(hist.cpu().numpy(), x[:, cut - (P - 1) * N:cut])


def test_accumulate_and_determinism(qc):
    import torch
    N, n_ant = 1024, 4
    x = torch.from_numpy(_stream(n_ant, N * 64, seed=7)).cuda()
    a = qc.xcorrelate(x, N, 4, 32)
    b = qc.xcorrelate(x, N, 4, 32)
    assert torch.equal(a, b)                           # bitwise deterministic
    c = qc.xcorrelate(x, N, 4, 32, vis=b.clone(), accumulate=True)
    assert torch.allclose(c, 2 * a, rtol=1e-6, atol=0)


def test_zero_input_gives_zero(qc):
    import torch
    x = torch.zeros((4, 4096 * 8), dtype=torch.int8, device="cuda")
    V = qc.xcorrelate(x, 4096, 4, 8)
    assert torch.count_nonzero(V) == 0


def test_extreme_values(qc):
    """Full-scale +-128/127 input: no overflow, still within tolerance."""
    N, n_ant = 1024, 4
    rng = np.random.default_rng(9)
    x = rng.choice(np.array([-128, 127], np.int8), size=(n_ant, N * 16))
    V_ref = _oracle_vis(x, N, 4, 16)
    V = _gpu_vis(qc, x, N, 4, 16)
    assert vis_err(V, V_ref, n_ant) <= TOL


FUSED_PAIRS = [(4096, 4), (1024, 4), (2048, 4), (512, 4), (1024, 8), (2048, 8), (1024, 2), (4096, 2)]


@pytest.mark.parametrize("N,n_ant", FUSED_PAIRS)
def test_every_fused_tile_matches_oracle(qc, N, n_ant):
    """Every tile shape of the fused kernel computes the same sums."""
    import torch
    P, spd, n_spec = 4, 9, 21
    x = _stream(n_ant, N * n_spec, seed=40 + N + n_ant)
    chans = _chans(N, n=24)
    V_ref = _oracle_vis(x, N, P, spd, chans=chans)
    xd = torch.from_numpy(x).cuda()
    n = qc.fx_tile_count(N, n_ant)
    assert n >= 1
    try:
        for t in range(n):
            qc.fx_set_tile(N, n_ant, t)
            V = qc.xcorrelate(xd, N, P, spd).cpu().numpy()[:, :, chans]
            assert vis_err(V, V_ref, n_ant) <= TOL, (t, vis_err(V, V_ref, n_ant))
            # with a run-time tap count (tile 0), and with asymmetric user taps
            # (every tile: those that take any prototype run them themselves)
            if t == 0:
                V3 = qc.xcorrelate(xd, N, 3, spd).cpu().numpy()[:, :, chans]
                R3 = _oracle_vis(x, N, 3, spd, chans=chans)
                assert vis_err(V3, R3, n_ant) <= TOL
            h = np.random.default_rng(N).normal(size=4 * N).astype(np.float32)
            Vu = qc.xcorrelate(xd, N, 4, spd, taps=torch.from_numpy(h).cuda()).cpu().numpy()
            Ru = xengine.correlate_fast(pfb.channelize(x, N, 4, taps=h.astype(np.float64),
                                                       chans=chans), spd)
            assert vis_err(Vu[:, :, chans], Ru, n_ant) <= TOL, (t, "user taps")
    finally:
        qc.fx_set_tile(N, n_ant, 0)


def test_autotune_picks_a_tile(qc):
    import torch
    x = torch.from_numpy(_stream(4, 1024 * 64, seed=3)).cuda()
    best, ms = qc.fx_autotune(x, 1024, 4, 32, reps=2)
    assert 0 <= best < qc.fx_tile_count(1024, 4) and len(ms) == qc.fx_tile_count(1024, 4)
    assert qc.fx_get_tile(1024, 4) == best and min(ms) == ms[best] and all(m > 0 for m in ms)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    assert qc.fx_get_width(1024, 4) in (0, n_cu, 4 * n_cu)
    qc.fx_set_tile(1024, 4, 0)
    qc.fx_set_width(1024, 4, 0)
    with pytest.raises(qc.QCError):
        qc.fx_set_tile(1024, 4, 99)


@pytest.mark.parametrize("N,n_ant", [(4096, 4), (1024, 8)])
def test_fused_launch_widths_match_oracle(qc, N, n_ant):
    """Any launch width (chunks per dump from 1 to the cap of 8 spectra per
    chunk) gives the oracle's sums, for the default tile and the last one."""
    import torch
    P, spd, n_spec = 4, 80, 170
    x = _stream(n_ant, N * n_spec, seed=7 + N + n_ant)
    chans = _chans(N, n=24)
    V_ref = _oracle_vis(x, N, P, spd, chans=chans)
    xd = torch.from_numpy(x).cuda()
    last = qc.fx_tile_count(N, n_ant) - 1
    try:
        for t in sorted({0, last}):
            qc.fx_set_tile(N, n_ant, t)
            for w in (1, 7, 256, 1024, 0):
                qc.fx_set_width(N, n_ant, w)
                assert qc.fx_get_width(N, n_ant) == w
                V = qc.xcorrelate(xd, N, P, spd).cpu().numpy()[:, :, chans]
                assert vis_err(V, V_ref, n_ant) <= TOL, (t, w, vis_err(V, V_ref, n_ant))
    finally:
        qc.fx_set_tile(N, n_ant, 0)
        qc.fx_set_width(N, n_ant, 0)


# N = 8192 runs two antennas (one packed transform) per workgroup; odd
# counts leave the second half of the last transform empty.
RING_CHAN = [(4096, 5, 20), (2048, 9, 18), (1024, 4, 33), (4096, 32, 6), (1024, 1, 17),
             (8192, 3, 9), (8192, 2, 12), (8192, 1, 5)]


@pytest.mark.parametrize("N,n_ant,n_spec", RING_CHAN)
def test_channelize_ring_matches_oracle(qc, N, n_ant, n_spec):
    """The register-ring F-engine (P = 4, built-in taps), including odd
    antenna groups and a carried history."""
    import torch
    P = 4
    x = _stream(n_ant, N * n_spec, seed=70 + N + n_ant)
    chans = _chans(N, n=24)
    assert qc.channelize_variant() == 0
    xd = torch.from_numpy(x).cuda()
    out, _ = qc.pfb_channelize(xd, N, P)
    X_ref = pfb.channelize(x, N, P, chans=chans)
    rms = np.sqrt(np.mean(np.abs(X_ref) ** 2))
    assert np.max(np.abs(out.cpu().numpy()[:, :, chans] - X_ref)) / rms <= TOL
    # second half with the first half's history
    cut = N * (n_spec // 2)
    hist = torch.zeros((n_ant, (P - 1) * N), dtype=torch.int8, device="cuda")
    qc.pfb_channelize(xd[:, :cut].contiguous(), N, P, hist_out=hist)
    o2, _ = qc.pfb_channelize(xd[:, cut:].contiguous(), N, P, hist=hist)
    torch.cuda.synchronize()
    assert np.max(np.abs(o2.cpu().numpy() - out.cpu().numpy()[:, n_spec // 2:])) / rms <= 1e-6


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16", "fp8"])
@pytest.mark.parametrize("N,n_ant,n_spec", [(4096, 6, 12), (8192, 5, 10)])
def test_channelize_variants_agree(qc, prec, N, n_ant, n_spec):
    import torch
    P = 4
    xd = torch.from_numpy(_stream(n_ant, N * n_spec, seed=99)).cuda()
    try:
        qc.channelize_variant(1)
        a, sa = qc.pfb_channelize(xd, N, P, out_prec=prec)
        qc.channelize_variant(0)
        b, sb = qc.pfb_channelize(xd, N, P, out_prec=prec)
        torch.cuda.synchronize()
    finally:
        qc.channelize_variant(0)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    if prec == "f32":
        rms = np.sqrt(np.mean(np.abs(a) ** 2))
        assert np.max(np.abs(a - b)) / rms <= 1e-6
    else:
        assert np.array_equal(sa.cpu().numpy(), sb.cpu().numpy())
        # identical up to rare rounding-boundary flips of the requantiser
        assert np.mean(a != b) <= 1e-3


# Float32 X-engine on both kernels over the same complex64 spectra: the
# vector-ALU kernel (variant 1) and the matrix-core kernel (variant 2; it
# serves n_ant <= 32 with n_chan % 16 == 0 on 32 x 32 tiles, or 16 x 16
# tiles up to 16 antennas; other shapes fall back to the vector ALU).  Ragged stages (spec_per_dump not a multiple of the 16
# spectra one stage holds), trailing spectra past the last dump, antenna
# counts from 1 to 32 and several dumps.  With the inputs exact, the only
# error is the float32 summation: bar 2e-6 of sqrt(V_ii V_jj).
XENG_F32 = [
    (32, 128, 20, 10),
    (17, 256, 35, 33),
    (24, 512, 64, 64),
    (5, 64, 50, 16),
    (32, 2048, 40, 40),
    (1, 32, 33, 11),
    (31, 64, 48, 17),
    (16, 256, 70, 35),    # up to 16 antennas the matrix cores use 16 x 16 tiles
    (12, 128, 64, 64),
    (9, 512, 40, 33),
    (3, 16, 50, 7),       # 8 channels: vector ALU under either variant
]


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("n_ant,N,n_spec,spd", XENG_F32)
def test_xengine_f32_kernels_match_oracle(qc, variant, n_ant, N, n_spec, spd):
    import torch
    x = _stream(n_ant, N * n_spec, seed=500 + n_ant + N)
    X = pfb.channelize(x, N, 4).astype(np.complex64)
    v = torch.from_numpy(X).cuda()
    old = qc.xengine_variant()
    try:
        qc.xengine_variant(variant)
        V = qc.xcorrelate_chan(v, "f32", None, n_ant, n_spec, N // 2, spd)
        torch.cuda.synchronize()
    finally:
        qc.xengine_variant(old)
    V_ref = xengine.correlate_fast(X, spd)
    assert V.shape == V_ref.shape
    err = vis_err(V.cpu().numpy(), V_ref, n_ant)
    assert err <= 2e-6, err


def test_xengine_f32_default_variant(qc):
    """Default: matrix cores from 5 antennas, vector ALU below; both paths
    of the default agree with the explicit variants bit for bit."""
    import torch
    assert qc.xengine_variant() == 0
    for n_ant, expect in ((4, 1), (5, 2), (16, 2), (17, 2), (32, 2)):
        N, n_spec, spd = 256, 32, 32
        X = pfb.channelize(_stream(n_ant, N * n_spec, seed=n_ant), N, 4).astype(np.complex64)
        v = torch.from_numpy(X).cuda()
        a = qc.xcorrelate_chan(v, "f32", None, n_ant, n_spec, N // 2, spd).cpu().numpy()
        try:
            qc.xengine_variant(expect)
            b = qc.xcorrelate_chan(v, "f32", None, n_ant, n_spec, N // 2, spd).cpu().numpy()
        finally:
            qc.xengine_variant(0)
        assert np.array_equal(a, b), n_ant
