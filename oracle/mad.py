"""MAD RFI-flagging oracle.

Follows the paper's Sec. 7, eq. (2): threshold T = median(A) + sigma *
MAD(A) * 1.4826 on visibility amplitude A, with sigma = 5 in the paper's
results and a mask that marks outliers.

Readings (the paper is silent on these):
  * population: per baseline over its whole (time x channel) plane by
    default; population 1 = per (baseline, channel) over time,
    population 2 = per (baseline, time) over channel;
  * median of an even count = mean of the two middle values;
  * MAD(A) = median(|A - median(A)|);
  * one-sided, strict: flag iff A > T.  MAD = 0 gives T = median;
  * arithmetic: amplitudes are |V| formed in float64 from the float32
    visibilities and rounded once to float32 (the kernel's precision takes
    this decision); the medians, deviations, threshold and the comparison
    are float64, with T = med + (sigma * 1.4826) * MAD in that order.

The median is written as "sort, then take the middle element(s)".
Status: pinned (see tests/test_oracle.py).
"""

from __future__ import annotations

import numpy as np

MAD_TO_SIGMA = 1.4826


def amplitude_f32(vis) -> np.ndarray:
    """|V| for complex64 input: float64 sqrt(re^2 + im^2), rounded to float32."""
    v = np.asarray(vis)
    re = v.real.astype(np.float64)
    im = v.imag.astype(np.float64)
    return np.sqrt(re * re + im * im).astype(np.float32)


def median_sorted(values) -> float:
    """Median by sorting: middle element, or the mean of the two middles."""
    s = np.sort(np.asarray(values, np.float64).ravel())
    n = s.size
    if n == 0:
        raise ValueError("median of an empty population")
    if n % 2:
        return float(s[n // 2])
    return float((s[n // 2 - 1] + s[n // 2]) / 2.0)


def mad_threshold(A, sigma: float):
    """(median, MAD, T) of one population, all float64."""
    A = np.asarray(A, np.float64).ravel()
    med = median_sorted(A)
    mad = median_sorted(np.abs(A - med))
    T = med + (np.float64(np.float32(sigma)) * MAD_TO_SIGMA) * mad
    return med, mad, T


def mad_flag(vis, sigma: float = 5.0, population: int = 0):
    """Mask (uint8, same shape as vis[n_time, n_base, n_chan]) and thresholds.

    Returns (mask, T) where T has shape [n_base] (population 0),
    [n_base, n_chan] (population 1) or [n_time, n_base] (population 2).
    """
    A = amplitude_f32(vis).astype(np.float64)
    n_time, n_base, n_chan = A.shape
    mask = np.zeros(A.shape, np.uint8)
    if population == 0:
        T = np.zeros(n_base)
        for b in range(n_base):
            _, _, t = mad_threshold(A[:, b, :], sigma)
            T[b] = t
            mask[:, b, :] = A[:, b, :] > t
    elif population == 1:
        T = np.zeros((n_base, n_chan))
        for b in range(n_base):
            for k in range(n_chan):
                _, _, t = mad_threshold(A[:, b, k], sigma)
                T[b, k] = t
                mask[:, b, k] = A[:, b, k] > t
    elif population == 2:
        T = np.zeros((n_time, n_base))
        for d in range(n_time):
            for b in range(n_base):
                _, _, t = mad_threshold(A[d, b, :], sigma)
                T[d, b] = t
                mask[d, b, :] = A[d, b, :] > t
    else:
        raise ValueError("population must be 0, 1 or 2")
    return mask, T
