"""Batched plans: uneven arrays correlated together, hipGraph replay,
autotuner, and (persistent mode) the bounded-wait error path.

Parity bar: the graph mode runs qc_xcorrelate's own kernels, so against it
max |V - V_ref| / sqrt(V_ii V_jj) <= 1e-6 (only the grouping of partial
sums may differ).  The persistent mode runs other float32 kernels (the
plain F-engine, the non-ring fused body and the vector-ALU X-engine, where
qc_xcorrelate may take the ring F-engine, the ring fused tile and the
matrix-core X-engine), so the two round differently; each is held to the
FP32 bar of 1e-5 against the FP64 oracle, and between them the bar is the
sum of the two, 2e-5.  A lost or doubled work item would show as an error
of order 1 / spec_per_dump, far above either bar.

The persistent mode (one launch, work-item queue, waits between dependent
items) runs every case the graph mode runs.  Its kernel's loop once
compiled into a lane-divergent nest in which the lanes other than lane 0
re-ran their first item for ever; tests/test_isa_loops.py checks the built
code objects for barriers inside lane-divergent loops."""

import ctypes

import numpy as np
import pytest

import synth
from oracle import pfb, xengine
from tests.util import vis_err

TOL = 1e-5


def _cross_bar(mode):
    """Bar between a plan's result and qc_xcorrelate's (see the module)."""
    return 1e-6 if mode == "graph" else 2 * TOL

MODES = ["graph", "persistent"]

# (n_ant, n_fft, n_spec, spec_per_dump): fused (4 ant N=1024/4096, 8 ant
# N=2048) and two-pass (odd and larger antenna counts) arrays, ragged dumps.
SMALL = [(4, 1024, 40, 12), (8, 2048, 21, 7), (16, 4096, 10, 5), (24, 4096, 9, 3),
         (32, 8192, 6, 6), (3, 64, 70, 9), (4, 4096, 17, 8), (1, 256, 30, 10)]


def _desc(n_ant, N, n_spec, spd, P=4):
    return {"n_ant": n_ant, "n_samp": N * n_spec, "n_fft": N, "n_taps": P, "spec_per_dump": spd}


def _x(n_ant, n_samp, seed):
    return synth.generate(synth.array_spec(n_ant, n_samp, seed, corr=0.3, max_lag=7))


def _chans(N, seed):
    nch = N // 2
    if nch <= 64:
        return np.arange(nch)
    rng = np.random.default_rng(seed)
    return np.array(sorted(set(rng.choice(nch, 20, replace=False).tolist()) | {0, nch - 1}))


def _inputs(arrays, seed=100):
    import torch
    hx = [_x(a["n_ant"], a["n_samp"], seed + i) for i, a in enumerate(arrays)]
    return hx, [torch.from_numpy(h).cuda() for h in hx]


# ---------------------------------------------------------------- CPU checks

@pytest.mark.parametrize("bad", [
    [],                                           # no arrays
    [_desc(4, 1024, 8, 8)] * 9,                   # too many arrays
    [_desc(0, 1024, 8, 8)],                       # no antennas
    [_desc(65, 1024, 8, 8)],                      # too many antennas
    [dict(_desc(4, 1024, 8, 8), n_fft=1000)],     # not a power of two
    [dict(_desc(4, 1024, 8, 8), n_fft=8)],        # below 16
    [dict(_desc(4, 1024, 8, 8), n_samp=1024 * 8 + 1)],   # not a multiple of n_fft
    [_desc(4, 1024, 8, 9)],                       # no full dump
    [dict(_desc(4, 1024, 8, 8), n_taps=0)],
    [_desc(4, 1024, 8, 8), _desc(4, 16, 1 << 27, 8)],    # n_samp = 2^31
])
def test_plan_create_rejects(bad):
    import paper_2604_20640_amd as qc
    try:
        L = qc.lib()
    except OSError:
        pytest.skip("library not built")
    n = len(bad)
    arr = (qc.ArrayDesc * max(n, 1))(*[qc.ArrayDesc(a["n_ant"], a["n_samp"], a["n_fft"], a["n_taps"],
                                                     a["spec_per_dump"]) for a in bad])
    h = ctypes.c_void_p()
    assert L.qc_plan_create(arr, n, ctypes.byref(h)) == -1     # QC_EINVAL, before any device call
    assert not h.value


def test_plan_null_handles():
    import paper_2604_20640_amd as qc
    try:
        L = qc.lib()
    except OSError:
        pytest.skip("library not built")
    assert L.qc_plan_create(None, 1, None) == -1
    assert L.qc_plan_set_mode(None, 0) == -1
    assert L.qc_plan_set_wait_timeout(None, 5) == -1
    assert L.qc_plan_set_wait_bias(None, 0) == -1
    assert L.qc_plan_info(None, None, None, None, None) == -1
    L.qc_plan_destroy(None)


# ---------------------------------------------------------------- GPU parity

@pytest.mark.gpu
@pytest.mark.parametrize("mode", MODES)
def test_plan_matches_xcorrelate_and_oracle(qc, mode):
    import torch
    arrays = [_desc(*s) for s in SMALL]
    hx, xs = _inputs(arrays)
    plan = qc.Plan(arrays, mode)
    n_launch, conc, tiles, splits = plan.info()
    if mode == "graph":
        assert n_launch >= 2 * len(arrays) and conc in (0, 1) and min(splits) >= 1
    else:
        assert n_launch == 2                      # counter reset + the persistent kernel
    assert [t >= 0 for t in tiles] == [qc.fx_tile_count(a["n_fft"], a["n_ant"]) > 0 for a in arrays]
    vis = plan.empty_vis()
    plan.execute(xs, vis)
    plan.check()
    for i, (a, h, x, v) in enumerate(zip(arrays, hx, xs, vis)):
        na, N, spd = a["n_ant"], a["n_fft"], a["spec_per_dump"]
        ref = qc.xcorrelate(x, N, a["n_taps"], spd)
        torch.cuda.synchronize()
        got = v.cpu().numpy()
        assert got.shape == ref.shape
        assert vis_err(got, ref.cpu().numpy(), na) <= _cross_bar(mode), i
        ch = _chans(N, i)
        V_ref = xengine.correlate_fast(pfb.channelize(h, N, a["n_taps"], chans=ch), spd)
        assert vis_err(got[:, :, ch], V_ref, na) <= TOL, i


@pytest.mark.gpu
@pytest.mark.parametrize("mode", MODES)
def test_plan_batch_workload_shapes(qc, mode):
    """The five uneven arrays of the batched workload, at a short length."""
    import torch
    arrays, hx = [], []
    for i, (na, nch) in enumerate(synth.BATCH_ARRAYS):
        N = 2 * nch
        n_spec = max(8, (1 << 17) // N)
        arrays.append(_desc(na, N, n_spec, n_spec // 2))
        hx.append(_x(na, N * n_spec, 500 + i))
    xs = [torch.from_numpy(h).cuda() for h in hx]
    plan = qc.Plan(arrays, mode)
    vis = plan.empty_vis()
    plan.execute(xs, vis)
    plan.check()
    sep = plan.empty_vis()
    plan.execute_separate(xs, sep)
    torch.cuda.synchronize()
    for i, a in enumerate(arrays):
        assert vis_err(vis[i].cpu().numpy(), sep[i].cpu().numpy(), a["n_ant"]) <= _cross_bar(mode), i
    # oracle on one sampled channel set of the largest array
    a, h = arrays[-1], hx[-1]
    ch = _chans(a["n_fft"], 9)
    V_ref = xengine.correlate_fast(pfb.channelize(h, a["n_fft"], 4, chans=ch), a["spec_per_dump"])
    assert vis_err(vis[-1].cpu().numpy()[:, :, ch], V_ref, a["n_ant"]) <= TOL


@pytest.mark.gpu
@pytest.mark.parametrize("mode", MODES)
def test_plan_is_deterministic_and_overwrites(qc, mode):
    import torch
    arrays = [_desc(*s) for s in SMALL[:4]]
    _, xs = _inputs(arrays, seed=7)
    plan = qc.Plan(arrays, mode)
    v1, v2 = plan.empty_vis(), plan.empty_vis()
    for v in v2:
        v.fill_(123.0)
    plan.execute(xs, v1)
    plan.execute(xs, v2)
    plan.check()
    for a, b in zip(v1, v2):
        assert torch.equal(a, b)


@pytest.mark.gpu
def test_plan_persistent_new_inputs_each_execution(qc):
    """Executions on alternating inputs: each result equals the graph mode's
    for the same input.  The persistent kernel hands spectra and partials
    between workgroups through buffers that every execution reuses, so data
    left over from the previous execution (or not yet visible from this
    one) would show here, where a repeated input could not reveal it."""
    arrays = [_desc(*s) for s in SMALL[:5]]
    _, xa = _inputs(arrays, seed=21)
    _, xb = _inputs(arrays, seed=57)
    g = qc.Plan(arrays, "graph")
    ref = {}
    for name, xs in (("a", xa), ("b", xb)):
        ref[name] = g.empty_vis()
        g.execute(xs, ref[name])
    g.check()
    p = qc.Plan(arrays, "persistent")
    for name, xs in (("a", xa), ("b", xb), ("a", xa), ("b", xb)):
        vis = p.empty_vis()
        p.execute(xs, vis)
        p.check()
        for i, a in enumerate(arrays):
            err = vis_err(vis[i].cpu().numpy(), ref[name][i].cpu().numpy(), a["n_ant"])
            assert err <= _cross_bar("persistent"), (name, i, err)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", MODES)
def test_plan_graph_replays(qc, mode):
    """Replays of the captured graph, with eager work on the same device
    between them, each equal to the eager execution."""
    import torch
    arrays = [_desc(*s) for s in SMALL[:5]]
    _, xs = _inputs(arrays, seed=11)
    plan = qc.Plan(arrays, mode)
    eager = plan.empty_vis()
    plan.execute(xs, eager)
    plan.check()
    vis = plan.empty_vis()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture_graph(xs, vis)
    torch.cuda.synchronize()
    other = torch.from_numpy(_x(4, 1024 * 16, 3)).cuda()
    for r in range(4):
        for v in vis:
            v.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            plan.replay()
        s.synchronize()
        plan.check()
        for a, b in zip(vis, eager):
            assert torch.equal(a, b), r
        qc.xcorrelate(other, 1024, 4, 8)        # eager work between replays
        plan.execute(xs, plan.empty_vis())
        torch.cuda.synchronize()


@pytest.mark.gpu
def test_plan_capture_needs_side_stream(qc):
    import torch
    arrays = [_desc(*SMALL[0])]
    _, xs = _inputs(arrays)
    plan = qc.Plan(arrays)
    with pytest.raises(qc.QCError):
        plan.capture_graph(xs, plan.empty_vis())   # the legacy default stream cannot capture
    with pytest.raises(qc.QCError):
        plan.replay()                              # nothing captured
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture_graph(xs, plan.empty_vis())
    with pytest.raises(qc.QCError):
        plan.replay()                              # replays need a created stream too
    with torch.cuda.stream(s):
        plan.replay()
    s.synchronize()


@pytest.mark.gpu
def test_plan_wait_timeout_reports_error(qc):
    """Dependencies made unsatisfiable from the host: every bounded wait
    expires, the kernel still drains, check() reports it, and the next
    normal execution is correct again."""
    import torch
    arrays = [_desc(16, 1024, 12, 6), _desc(5, 256, 20, 10)]      # two-pass arrays: waits
    _, xs = _inputs(arrays, seed=13)
    plan = qc.Plan(arrays, "persistent")
    good = plan.empty_vis()
    plan.execute(xs, good)
    plan.check()
    plan.set_wait_timeout(2000)          # 2 ms
    plan.set_wait_bias(1)
    bad = plan.empty_vis()
    plan.execute(xs, bad)
    with pytest.raises(qc.QCError) as ei:
        plan.check()
    assert ei.value.status == -5
    plan.set_wait_bias(0)
    plan.set_wait_timeout(2000000)
    again = plan.empty_vis()
    plan.execute(xs, again)
    plan.check()
    for a, b in zip(again, good):
        assert torch.equal(a, b)


@pytest.mark.gpu
def test_plan_autotune_and_cache(qc, tmp_path):
    import torch
    arrays = [_desc(*s) for s in SMALL[:5]]
    _, xs = _inputs(arrays, seed=17)
    cache = str(tmp_path / "plan_tune.txt")
    plan = qc.Plan(arrays)
    ref = plan.empty_vis()
    plan.execute(xs, ref)
    plan.check()
    vis = plan.empty_vis()
    assert plan.autotune(xs, vis, reps=1, cache=cache) is False
    knobs = plan.info()
    plan.execute(xs, vis)
    plan.check()
    for a, b, d in zip(vis, ref, arrays):
        assert vis_err(a.cpu().numpy(), b.cpu().numpy(), d["n_ant"]) <= 1e-6
    plan2 = qc.Plan(arrays)
    assert plan2.autotune(xs, plan2.empty_vis(), reps=1, cache=cache) is True
    assert plan2.info() == knobs
    torch.cuda.synchronize()


@pytest.mark.gpu
def test_plan_serial_equals_concurrent(qc):
    """Arrays forked to streams of their own or run in order on the caller's
    stream: identical sums (same kernels, same splits)."""
    import os
    import tempfile

    import torch
    arrays = [_desc(*s) for s in SMALL]
    _, xs = _inputs(arrays, seed=23)
    plan = qc.Plan(arrays)
    a = plan.empty_vis()
    plan.execute(xs, a)
    plan.check()
    n, conc, tiles, splits = plan.info()
    assert conc == 1
    # switch concurrency off through a cache entry (the tuner's own format)
    sig = ",".join(f"{d['n_ant']}x{d['n_samp']}x{d['n_fft']}x{d['n_taps']}x{d['spec_per_dump']}"
                   for d in arrays)
    knobs = " ".join(f"{t} {s}" for t, s in zip(tiles, splits))
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "c.txt")
        with open(path, "w") as f:
            f.write(f"{sig} 0 {knobs}\n")
        assert plan.autotune(xs, plan.empty_vis(), reps=1, cache=path) is True
    assert plan.info()[1] == 0
    b = plan.empty_vis()
    plan.execute(xs, b)
    plan.check()
    for u, v in zip(a, b):
        assert torch.equal(u, v)


@pytest.mark.gpu
def test_plan_mode_switch(qc):
    """graph -> persistent -> graph -> persistent on one plan: each mode
    repeats itself bit for bit, and the two agree to the cross bar."""
    arrays = [_desc(*s) for s in SMALL[:6]]
    _, xs = _inputs(arrays, seed=17)
    plan = qc.Plan(arrays)
    runs = []
    for mode in ("graph", "persistent", "graph", "persistent"):
        plan.set_mode(mode)
        if mode == "persistent":
            assert plan.info()[0] == 2
        v = plan.empty_vis()
        plan.execute(xs, v)
        plan.check()
        runs.append([t.cpu().numpy() for t in v])
    for i, a in enumerate(arrays):
        assert np.array_equal(runs[0][i], runs[2][i]) and np.array_equal(runs[1][i], runs[3][i])
        assert vis_err(runs[1][i], runs[0][i], a["n_ant"]) <= _cross_bar("persistent"), i
