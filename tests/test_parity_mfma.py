"""GPU parity: requantising F-engine and the matrix-core X-engine.

* requantiser: per-antenna power-of-two scales equal the oracle's exactly;
  codes equal the oracle's quantisation of its FP64 spectra except for rare
  rounding-boundary flips (the GPU's FP32 spectra differ from FP64 by
  ~1e-7 relative), each between the two grid neighbours of the exact value;
* matrix-core X-engine, exact: fed the oracle's own quantised codes, it
  matches the oracle's float64 multiply-accumulate of those codes to float32
  accumulation error (products of the formats are exact in FP32);
* end to end (F-engine -> requantise -> matrix cores) against the plain FP64
  oracle: every format within the bar its significand width sets for the
  dump length (tests.util.quant_bar: z * 2^(1-p) / sqrt(3 M), z = 5).
"""

import numpy as np
import pytest

import synth
from oracle import pfb, quant, xengine
from tests.util import per_baseline_errors, quant_bar, vis_err

pytestmark = pytest.mark.gpu

PRECS = ["f16", "bf16", "fp8"]
QNAME = {"f16": "fp16", "bf16": "bf16", "fp8": "fp8"}


def _torch_dtype(prec):
    import torch
    return {"f16": torch.float16, "bf16": torch.bfloat16, "fp8": torch.float8_e4m3fn}[prec]


def _decode(raw, prec):
    import torch
    f = torch.from_numpy(raw).view(_torch_dtype(prec)).float().numpy().astype(np.float64)
    return f[..., 0::2] + 1j * f[..., 1::2]


def _encode(Q, prec):
    """Exactly representable complex values -> interleaved (re, im) bytes."""
    import torch
    inter = np.stack([Q.real, Q.imag], axis=-1).reshape(*Q.shape[:-1], 2 * Q.shape[-1])
    t = torch.from_numpy(np.ascontiguousarray(inter)).to(_torch_dtype(prec))
    assert np.array_equal(t.double().numpy(), inter)          # the cast was exact
    return t.view(torch.uint8)


def _setup(n_ant, N, n_spec, seed):
    spec = synth.array_spec(n_ant, N * n_spec, seed, corr=0.1, max_lag=40)
    return synth.generate(spec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n_ant,N,n_spec", [(32, 1024, 96), (5, 128, 40)])
def test_requantiser(qc, prec, n_ant, N, n_spec):
    import torch
    P = 4
    x = _setup(n_ant, N, n_spec, seed=100 + n_ant)
    out, scale = qc.pfb_channelize(torch.from_numpy(x).cuda(), N, P, out_prec=prec)
    s_ref = quant.pow2_scales(x, pfb.hann_sinc_taps(N, P), QNAME[prec])
    assert np.array_equal(scale.cpu().numpy().astype(np.float64), s_ref)
    Xs = pfb.channelize(x, N, P) * s_ref[:, None, None]
    Q_ref = quant.quantise_complex(Xs, QNAME[prec])
    Q = _decode(out.cpu().numpy(), prec)
    f = quant.QUANTISERS[QNAME[prec]]
    # the GPU's float32 spectra carry an error ~1e-7 of the channel rms
    tol = 1e-5 * np.sqrt(np.mean(np.abs(Xs) ** 2, axis=(1, 2)))[:, None, None] * np.ones(Xs.shape)
    for part in (np.real, np.imag):
        q, r, v = part(Q), part(Q_ref), part(Xs)
        diff = q != r
        assert diff.mean() < 1e-2, diff.mean()
        if diff.any():
            # a flip happens only next to a rounding boundary: the two codes
            # are the grid neighbours of the exact value
            lo = np.minimum(q[diff], r[diff])
            hi = np.maximum(q[diff], r[diff])
            vv, tt = v[diff], tol[diff]
            assert np.all((lo <= vv + tt) & (vv <= hi + tt))
            # where the code spacing exceeds the spectra's error, the two
            # codes are neighbours (no code strictly between them)
            big = (hi - lo) > 2 * tt
            mid = f((lo[big] + hi[big]) / 2)
            assert np.all((mid == lo[big]) | (mid == hi[big]))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n_ant,N,n_spec,spd", [(32, 1024, 96, 48), (24, 512, 64, 64),
                                                (5, 128, 40, 20), (17, 256, 35, 33)])
def test_mfma_xengine_exact(qc, prec, n_ant, N, n_spec, spd):
    import torch
    P = 4
    x = _setup(n_ant, N, n_spec, seed=200 + n_ant)
    s_ref = quant.pow2_scales(x, pfb.hann_sinc_taps(N, P), QNAME[prec])
    Q_ref = quant.quantise_complex(pfb.channelize(x, N, P) * s_ref[:, None, None], QNAME[prec])
    v = _encode(Q_ref, prec).cuda()
    scale = torch.from_numpy(s_ref.astype(np.float32)).cuda()
    V = qc.xcorrelate_chan(v, prec, scale, n_ant, n_spec, N // 2, spd).cpu().numpy()
    V_q = xengine.correlate_fast(Q_ref / s_ref[:, None, None], spd)
    err = vis_err(V, V_q, n_ant)
    print(f"{prec} n_ant={n_ant}: exact-input err {err:.2e}")
    # FP16/BF16 products are exact in FP32 and the sums round like an FP32
    # accumulator.  The E4M3 matrix-core dot products were measured to carry
    # an error of ~5e-5 of the auto scale (they are not FP32-exact sums), so
    # that format gets its own bar.
    assert err <= (2e-4 if prec == "fp8" else 1e-6), err


@pytest.mark.parametrize("prec", PRECS)
def test_mfma_end_to_end_accuracy(qc, prec):
    import torch
    n_ant, N, n_spec, spd = 32, 1024, 96, 96
    x = _setup(n_ant, N, n_spec, seed=300)
    out, scale = qc.pfb_channelize(torch.from_numpy(x).cuda(), N, 4, out_prec=prec)
    V = qc.xcorrelate_chan(out, prec, scale, n_ant, n_spec, N // 2, spd).cpu().numpy()
    V_ref = xengine.correlate_fast(pfb.channelize(x, N, 4), spd)
    err = vis_err(V, V_ref, n_ant)
    amp, ph, nerr = per_baseline_errors(V, V_ref, n_ant)
    print(f"{prec}: err vs fp64 {err:.2e}; median per-baseline err {np.median(nerr):.2e}; "
          f"bar {quant_bar(prec, spd):.2e}")
    assert err <= quant_bar(prec, spd), err


def test_mfma_hermitian_structure(qc):
    """Autos real and non-negative; crosses obey Cauchy-Schwarz."""
    import torch
    n_ant, N, n_spec = 32, 256, 64
    x = torch.from_numpy(_setup(n_ant, N, n_spec, seed=5)).cuda()
    out, scale = qc.pfb_channelize(x, N, 4, out_prec="f16")
    V = qc.xcorrelate_chan(out, "f16", scale, n_ant, n_spec, N // 2, n_spec).cpu().numpy()[0]
    pairs = [(i, j) for i in range(n_ant) for j in range(i, n_ant)]
    idx = {p: b for b, p in enumerate(pairs)}
    for a in range(n_ant):
        assert np.all(V[idx[(a, a)]].imag == 0) and np.all(V[idx[(a, a)]].real >= 0)
    for (i, j), b in idx.items():
        lhs = np.abs(V[b]) ** 2
        rhs = V[idx[(i, i)]].real * V[idx[(j, j)]].real
        assert np.all(lhs <= rhs * (1 + 1e-5))


@pytest.mark.parametrize("prec", PRECS)
def test_xcorrelate_reduced_precision_two_pass(qc, prec):
    """qc_xcorrelate with a reduced x_prec = channelise + matrix-core X."""
    import torch
    n_ant, N, n_spec = 16, 512, 32
    x = _setup(n_ant, N, n_spec, seed=77)
    V = qc.xcorrelate(torch.from_numpy(x).cuda(), N, 4, 16, x_prec=prec).cpu().numpy()
    V_ref = xengine.correlate_fast(pfb.channelize(x, N, 4), 16)
    err = vis_err(V, V_ref, n_ant)
    print(f"two-pass {prec}: err vs fp64 {err:.2e}; bar {quant_bar(prec, 16):.2e}")
    assert err <= quant_bar(prec, 16), err


def test_mfma_rejects_unsupported(qc):
    import torch
    v = torch.zeros((40, 8, 64 * 4), dtype=torch.uint8, device="cuda")
    scale = torch.ones(40, device="cuda")
    with pytest.raises(qc.QCError):
        qc.xcorrelate_chan(v, "f16", scale, 40, 8, 64, 8)     # 40 antennas > 32


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N,n_samp", [(16, 16 * 81), (64, (1 << 20) + 64 * 65)])
def test_scales_strided_and_past_prefix(qc, prec, N, n_samp):
    """Scales over a strided view (row stride a multiple of 4 but not of
    16), with a loud stretch at the end of the stream: it counts when the
    stream is shorter than the 2^20-sample prefix the scales are taken
    from, and is ignored when it lies past that prefix."""
    import torch
    n_ant, P = 3, 4
    W = n_samp + 12
    rng = np.random.default_rng(n_samp)
    full = rng.integers(-40, 41, (n_ant, W)).astype(np.int8)
    full[1] //= 3                                  # different powers per antenna
    full[2, n_samp - 64:n_samp] = 127
    x = full[:, :n_samp]
    xd = torch.from_numpy(full).cuda()[:, :n_samp]
    assert xd.stride(0) == W
    _, scale = qc.pfb_channelize(xd, N, P, out_prec=prec)
    s_ref = quant.pow2_scales(x, pfb.hann_sinc_taps(N, P), QNAME[prec])
    assert np.array_equal(scale.cpu().numpy().astype(np.float64), s_ref)
