"""Kernel timing modes of the measurement interface: argument checks on the
host, and on the GPU that both modes record every timed call and leave the
results unchanged, and that chained figures tile the stream's time."""

import numpy as np
import pytest

import paper_2604_20640_amd as qc_mod

QC_EINVAL = -1


def test_timing_modes_host():
    L = qc_mod.lib()
    for bad in (-1, 3):
        assert L.qc_timing_enable(bad) == QC_EINVAL
    for mode in (2, 1, 0):
        assert L.qc_timing_enable(mode) == 0
    # nothing recorded: zero launches, no device work
    assert qc_mod.timing_read("fx_fused") == (0.0, 0)


@pytest.mark.gpu
def test_timing_modes_count_tile_and_leave_results_unchanged(qc):
    import torch
    from synth import array_spec, generate

    N, P, spd, reps = 1024, 4, 64, 6
    x = torch.from_numpy(generate(array_spec(4, 8 * spd * N, 41))).cuda()
    ref = qc.xcorrelate(x, N, P, spd)
    m_ref, _ = qc.mad_flag(ref, 5.0, 0)
    names = ("fx_fused", "reduce", "mad")

    def run(mode):
        vis = torch.empty_like(ref)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        qc.timing_enable(mode)
        e0.record()
        for _ in range(reps):
            qc.xcorrelate(x, N, P, spd, vis=vis)
            m, _ = qc.mad_flag(vis, 5.0, 0)
        e1.record()
        torch.cuda.synchronize()
        got = {k: qc.timing_read(k) for k in names}
        qc.timing_enable(False)
        assert torch.equal(vis, ref) and torch.equal(m, m_ref)
        return got, e0.elapsed_time(e1)

    (pairs, _), (chained, elapsed) = run(True), run("chained")
    for k in names:
        assert pairs[k][1] == chained[k][1] == reps, (k, pairs[k], chained[k])
        assert pairs[k][0] > 0 and chained[k][0] > 0
    # chained figures tile the stream: they sum to the region's elapsed time
    # less what lies outside the first call's start and the last call's end
    # (the host's time to reach the first launch, well under 0.3 ms)
    total = sum(chained[k][0] for k in names)
    assert elapsed - 0.3 <= total <= elapsed + 1e-3, (total, elapsed)


@pytest.mark.gpu
def test_chained_timing_leaves_graph_capture_alone(qc):
    """With chained timing on, a plan captured into a graph carries no timing
    events: the capture succeeds and each replay equals the eager result."""
    import torch
    from synth import array_spec, generate

    arrays = [dict(n_ant=4, n_samp=1024 * 64, n_fft=1024, spec_per_dump=32)]
    xs = [torch.from_numpy(generate(array_spec(4, 1024 * 64, 43))).cuda()]
    plan = qc.Plan(arrays)
    eager = plan.empty_vis()
    plan.execute(xs, eager)
    torch.cuda.synchronize()
    vis = plan.empty_vis()
    s = torch.cuda.Stream()
    qc.timing_enable("chained")
    try:
        with torch.cuda.stream(s):
            plan.capture_graph(xs, vis)
        torch.cuda.synchronize()
        for r in range(3):
            for v in vis:
                v.zero_()
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                plan.replay()
            s.synchronize()
            for a, b in zip(vis, eager):
                assert torch.equal(a, b), r
    finally:
        qc.timing_enable(False)
