"""The measurement helpers that give the bench its achievable rates: each
kind runs and reports a rate between a loose floor and the published peak
(no kernel can beat the hardware; a rate far below it means the helper
measures something else)."""

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,lo,hi", [
    ("hbm_read", 1000.0, 8000.0),      # GB/s; published HBM3E 8 TB/s
    ("hbm_copy", 1000.0, 8000.0),
    ("valu_f32", 20.0, 157.3),         # TFLOP/s; scalar FP32 FMA, published 157.3 with packed FP32
    ("mfma_f32", 40.0, 157.3),
    ("mfma_f16", 300.0, 2500.0),
])
def test_measure_peak_in_range(qc, kind, lo, hi):
    import torch
    buf = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    rate = qc.measure_peak(kind, buf, reps=2)
    assert lo <= rate <= hi * 1.02, (kind, rate)
