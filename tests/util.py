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
