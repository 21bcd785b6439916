"""Shared test helpers (no correlator arithmetic here)."""

import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qc.h")


def header_functions():
    """Names of every function declared in include/qc.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(qc_[a-z0-9_]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def auto_scale(V_ref, n_ant):
    """sqrt(V_ii V_jj) per (dump, baseline, channel) from reference autos."""
    pairs = [(i, j) for i in range(n_ant) for j in range(i, n_ant)]
    idx = {p: b for b, p in enumerate(pairs)}
    autos = np.stack([V_ref[:, idx[(a, a)], :].real for a in range(n_ant)], axis=1)
    sc = np.empty(V_ref.shape, np.float64)
    for b, (i, j) in enumerate(pairs):
        sc[:, b, :] = np.sqrt(np.maximum(autos[:, i, :] * autos[:, j, :], 0.0))
    return sc


def vis_err(V_gpu, V_ref, n_ant):
    """max |V_gpu - V_ref| / sqrt(V_ii V_jj) (autos from the reference)."""
    sc = auto_scale(V_ref, n_ant)
    d = np.abs(np.asarray(V_gpu, np.complex128) - np.asarray(V_ref, np.complex128))
    return float(np.max(d / np.maximum(sc, 1e-300)))


def per_baseline_errors(V, V_ref, n_ant):
    """Per-baseline amplitude error, phase error (deg) and auto-normalised error."""
    sc = auto_scale(V_ref, n_ant)
    V = np.asarray(V, np.complex128)
    amp = np.abs(np.abs(V) - np.abs(V_ref)) / np.maximum(np.abs(V_ref), 1e-300)
    ph = np.degrees(np.abs(np.angle(V * np.conj(V_ref))))
    nerr = np.abs(V - V_ref) / np.maximum(sc, 1e-300)
    return amp.max(axis=(0, 2)), ph.max(axis=(0, 2)), nerr.max(axis=(0, 2))


SIG_BITS = {"f16": 11, "fp16": 11, "bf16": 8, "fp8": 4, "e4m3": 4}


def quant_bar(prec, M, z=5.0):
    """Bar on the auto-normalised visibility error of a requantised X-engine.

    Rounding each component of X to a p-bit significand (round to nearest)
    leaves an error e with E|e|^2 <= delta^2 |X|^2, delta = 2^(1-p)/sqrt(12)
    (uniform error over one unit in the last place, whose size relative to
    the value is at most 2^(1-p)).  To first order a dump of M spectra then
    carries sum_m (X_i e_j* + e_i X_j*), whose rms over sqrt(V_ii V_jj) is
    sqrt(2/M) delta for a cross baseline and sqrt(4/M) delta for an auto.
    The bar is z times the larger, z * 2^(1-p) / sqrt(3 M); z = 5 covers the
    maximum over ~10^6 visibilities.  FP32 accumulation (~1e-7) is below
    it for every format here.
    """
    p = SIG_BITS[prec]
    return z * 2.0 ** (1 - p) / np.sqrt(3.0 * M)
