"""Hand-worked fixtures of the paper's formulas (tests/golden/), checked
against the oracle (CPU) and the HIP path (GPU)."""

import os

import numpy as np
import pytest

from oracle import calib, mad

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append([f.strip() for f in line.split("|")])
    return out


def _mad_cases():
    for label_vals, med, madv, thr, flags in _rows("mad_eq2_worked.txt"):
        vals = [float(v) for v in label_vals.split()[1].split(",")]
        yield vals, float(med), float(madv), float(thr), [int(f) for f in flags.split(",")]


def _apply_cases():
    return [(b, int(k), float(re), float(im)) for b, k, re, im in _rows("apply_eq1_worked.txt")]


def test_oracle_mad_matches_worked_example():
    for vals, med, madv, thr, flags in _mad_cases():
        m, d, t = mad.mad_threshold(np.array(vals), 5.0)
        assert (m, d) == (med, madv)
        assert t == pytest.approx(thr, abs=1e-12)
        vis = np.array(vals, np.complex64).reshape(1, 1, -1)
        mk, _ = mad.mad_flag(vis, 5.0, 0)
        assert mk.ravel().tolist() == flags


def test_oracle_apply_matches_worked_example():
    vis = np.ones((1, 3, 4), np.complex64)
    out = calib.apply_delay_phase(vis, 2, 0.0, 1e6, [2.5e-7, 0.0], [0.25 * np.pi, 0.0])
    bidx = {"00": 0, "01": 1, "11": 2}
    for b, k, re, im in _apply_cases():
        assert out[0, bidx[b], k] == pytest.approx(complex(re, im), abs=1e-12)


@pytest.mark.gpu
def test_gpu_mad_matches_worked_example(qc):
    import torch
    for vals, med, madv, thr, flags in _mad_cases():
        vis = torch.tensor(np.array(vals, np.complex64).reshape(1, 1, -1)).cuda()
        mk, t = qc.mad_flag(vis, 5.0, 0)
        assert mk.cpu().numpy().ravel().tolist() == flags
        assert float(t.cpu()[0]) == pytest.approx(thr, abs=1e-12)


@pytest.mark.gpu
def test_gpu_apply_matches_worked_example(qc):
    import torch
    vis = torch.ones((1, 3, 4), dtype=torch.complex64, device="cuda")
    qc.apply_delay_phase(vis, 2, 0.0, 1e6, [2.5e-7, 0.0], [0.25 * np.pi, 0.0])
    out = vis.cpu().numpy()
    bidx = {"00": 0, "01": 1, "11": 2}
    for b, k, re, im in _apply_cases():
        assert out[0, bidx[b], k] == pytest.approx(complex(re, im), abs=1e-6)
