"""X-engine oracle: per-channel cross-multiply and integration.

Follows the paper's Sec. 4.1 eq. (1) (cross-power V_i V_j^*, time-integrated)
and Sec. 4.2 / Alg. 1 ("X-Engine: compute V_i V_j^* for all baselines",
"Integration: accumulate results in GPU global memory").

Readings:
  * baselines are all pairs i <= j (autos included), upper triangle in
    row-major order: b(i, j) = i*Na - i*(i-1)/2 + (j - i);
  * integration is a plain sum over spec_per_dump consecutive spectra
    (the paper says "accumulated"), full dumps only;
  * autos carry an imaginary part of exactly zero.

The multiply-accumulate is written out per baseline.  Status: pinned.
correlate() by the Gram-matrix route, Hermitian/PSD/Cauchy-Schwarz
identities and noise and delay statistics; correlate_fast() by exact
agreement with correlate() on ragged dumps from 1 to 32 antennas, with a
check of which operand carries the conjugate (tests/test_oracle.py).
"""

from __future__ import annotations

import numpy as np


def baseline_pairs(n_ant: int):
    """[(i, j)] for 0 <= i <= j < n_ant in row-major upper-triangle order."""
    return [(i, j) for i in range(n_ant) for j in range(i, n_ant)]


def baseline_index(i: int, j: int, n_ant: int) -> int:
    return i * n_ant - i * (i - 1) // 2 + (j - i)


def correlate(X, spec_per_dump: int) -> np.ndarray:
    """V[d, b, k] = sum_{m in dump d} X[i, m, k] * conj(X[j, m, k]).

    ``X`` is complex [n_ant, M, n_chan]; returns complex128
    [M // spec_per_dump, n_base, n_chan].  Spectra past the last full dump
    are not integrated.
    """
    X = np.asarray(X, np.complex128)
    n_ant, M, n_chan = X.shape
    D = int(spec_per_dump)
    n_dump = M // D
    pairs = baseline_pairs(n_ant)
    V = np.zeros((n_dump, len(pairs), n_chan), np.complex128)
    for d in range(n_dump):
        seg = X[:, d * D:(d + 1) * D, :]
        for b, (i, j) in enumerate(pairs):
            acc = np.zeros(n_chan, np.complex128)
            for m in range(D):
                acc += seg[i, m] * np.conj(seg[j, m])
            if i == j:
                acc = acc.real.astype(np.complex128)
            V[d, b] = acc
    return V


def correlate_fast(X, spec_per_dump: int) -> np.ndarray:
    """Same sums as :func:`correlate`, with the m-loop done by numpy.

    Used at sizes where the per-spectrum Python loop is too slow; the
    arithmetic (sum of X_i conj(X_j) over the dump) is identical.
    """
    X = np.asarray(X, np.complex128)
    n_ant, M, n_chan = X.shape
    D = int(spec_per_dump)
    n_dump = M // D
    pairs = baseline_pairs(n_ant)
    V = np.zeros((n_dump, len(pairs), n_chan), np.complex128)
    for d in range(n_dump):
        seg = X[:, d * D:(d + 1) * D, :]
        for b, (i, j) in enumerate(pairs):
            acc = np.sum(seg[i] * np.conj(seg[j]), axis=0)
            if i == j:
                acc = acc.real.astype(np.complex128)
            V[d, b] = acc
    return V
