"""Reduced-precision quantisers for the MFMA X-engine reference.

The paper runs its X-engine in one precision and does not discuss reduced
precision.  The MFMA X-engine requantises channelised voltages to FP16,
BF16 or FP8 (E4M3) after a per-antenna power-of-two scale and accumulates
in FP32.  This module gives the plain definitions of those number formats
so that a quantisation-aware reference (quantise X, then an exact
multiply-accumulate) can be formed; errors against the unquantised FP64
reference are reported separately.

Formats (round to nearest, ties to even; values beyond the largest finite
magnitude saturate to it):
  * FP16: IEEE binary16, 11 significant bits, max 65504, min normal 2^-14;
  * BF16: 8 significant bits, float32 exponent range;
  * E4M3 (OCP FP8, "fn" variant): 4 significant bits, max 448, min normal
    2^-6, subnormal step 2^-9, no infinities.

Per-antenna scale (reading): s_a = 2^round(log2(target / rms_a)), where
rms_a is the expected channel rms from the input power,
rms_a = sqrt(mean(|x_a|^2) * sum_q h[q]^2), the mean taken over the first
min(S, 2^20) samples of antenna a (|x|^2 = I^2 + Q^2 for complex samples).  Targets: E4M3 32, FP16 256, BF16 1.
round() here is round-half-to-even on the float64 log2.
Status: pinned (tests/test_oracle.py: grids, ties, saturation).
"""

from __future__ import annotations

import numpy as np

PREC_TARGET = {"fp16": 256.0, "bf16": 1.0, "fp8": 32.0}
SCALE_PREFIX = 1 << 20


def _round_to_grid(v, exp_min: int, mant_bits: int, max_val: float) -> np.ndarray:
    """RNE of float64 v onto a binary grid with mant_bits significant bits."""
    v = np.asarray(v, np.float64)
    a = np.abs(v)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    # exact exponent: correct log2 rounding at powers of two
    e = np.where(np.ldexp(1.0, e.astype(np.int64)) > a, e - 1, e)
    e = np.where(np.ldexp(1.0, (e + 1).astype(np.int64)) <= a, e + 1, e)
    e = np.maximum(e, exp_min)
    q = np.ldexp(1.0, (e - (mant_bits - 1)).astype(np.int64))
    r = np.round(a / q) * q  # numpy rounds half to even
    r = np.minimum(r, max_val)
    return np.where(a > 0, np.sign(v) * r, 0.0 * v)


def to_fp16(v):
    return _round_to_grid(v, -14, 11, 65504.0)


def to_bf16(v):
    return _round_to_grid(v, -126, 8, float(np.float32(3.3895313892515355e38)))


def to_e4m3(v):
    return _round_to_grid(v, -6, 4, 448.0)


QUANTISERS = {"fp16": to_fp16, "bf16": to_bf16, "fp8": to_e4m3}


def quantise_complex(X, prec: str):
    f = QUANTISERS[prec]
    X = np.asarray(X)
    return f(X.real) + 1j * f(X.imag)


def pow2_scales(x, taps, prec: str) -> np.ndarray:
    """Per-antenna power-of-two scale s_a (float64) from the input power."""
    x = np.asarray(x)
    n = min(x.shape[1], SCALE_PREFIX)
    if np.iscomplexobj(x):
        # complex I/Q samples: the power is |x|^2 = I^2 + Q^2
        re = x[:, :n].real.astype(np.int64)
        im = x[:, :n].imag.astype(np.int64)
        p = (re * re + im * im).sum(axis=1).astype(np.float64) / n
    else:
        p = (x[:, :n].astype(np.int64) ** 2).sum(axis=1).astype(np.float64) / n
    h2 = float(np.sum(np.asarray(taps, np.float64) ** 2))
    rms = np.sqrt(p * h2)
    e = np.zeros(x.shape[0])
    ok = rms > 0
    e[ok] = np.round(np.log2(PREC_TARGET[prec] / rms[ok]))
    return np.ldexp(1.0, e.astype(np.int64))
