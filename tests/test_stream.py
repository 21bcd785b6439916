"""Streaming ingest (Alg. 1): pinned host chunks -> device ring -> fused F+X
with the filter history carried between chunks."""

import ctypes
import os

import numpy as np
import pytest

import synth
from oracle import pfb, xengine
from tests.util import vis_err

import paper_2604_20640_amd as qc_mod


@pytest.mark.skipif(not os.path.exists(qc_mod.LIB_PATH), reason="libqc.so not built")
def test_stream_create_rejects_bad_arguments():
    L = qc_mod.lib()
    h = ctypes.c_void_p()
    ok = qc_mod.PfbParams(1024, 4, None, 0)
    assert L.qc_stream_create(4, 1024 * 10, ctypes.byref(ok), 4, 2, ctypes.byref(h)) == -1  # 10 % 4
    assert L.qc_stream_create(4, 1000, ctypes.byref(ok), 1, 2, ctypes.byref(h)) == -1       # not k*N
    assert L.qc_stream_create(0, 4096, ctypes.byref(ok), 1, 2, ctypes.byref(h)) == -1
    assert L.qc_stream_create(4, 4096, ctypes.byref(ok), 1, 0, ctypes.byref(h)) == -1
    bad = qc_mod.PfbParams(1000, 4, None, 0)
    assert L.qc_stream_create(4, 4000, ctypes.byref(bad), 1, 2, ctypes.byref(h)) == -1
    assert h.value is None


def _pinned(x):
    import torch
    t = torch.empty(x.shape, dtype=torch.int8, pin_memory=True)
    t.copy_(torch.from_numpy(x))
    return t


@pytest.mark.gpu
@pytest.mark.parametrize("N,n_ant,spd,chunk_dumps,n_chunks,depth", [
    (4096, 4, 16, 2, 5, 3), (1024, 4, 32, 1, 6, 2), (256, 6, 8, 3, 4, 4), (64, 3, 5, 2, 7, 1)])
def test_stream_equals_one_shot(qc, N, n_ant, spd, chunk_dumps, n_chunks, depth):
    import torch
    P = 4
    chunk = N * spd * chunk_dumps
    x = synth.generate(synth.array_spec(n_ant, chunk * n_chunks, 31, corr=0.3, max_lag=9))
    one = qc.xcorrelate(torch.from_numpy(x).cuda(), N, P, spd).cpu().numpy()
    st = qc.Stream(n_ant, chunk, N, P, spd, depth=depth)
    hosts = [_pinned(x[:, i * chunk:(i + 1) * chunk]) for i in range(n_chunks)]
    outs = [torch.empty((chunk_dumps, n_ant * (n_ant + 1) // 2, N // 2), dtype=torch.complex64,
                        device="cuda") for _ in range(n_chunks)]
    for i in range(n_chunks):
        assert st.push(hosts[i], i, outs[i]) == chunk_dumps
    st.sync()
    got = torch.cat(outs).cpu().numpy()
    st.close()
    assert vis_err(got, one, n_ant) <= 1e-6
    chans = np.arange(0, N // 2, max(1, N // 64))
    V_ref = xengine.correlate_fast(pfb.channelize(x, N, P, chans=chans), spd)
    assert vis_err(got[:, :, chans], V_ref, n_ant) <= 1e-5


@pytest.mark.gpu
def test_stream_gap_restarts_history(qc):
    import torch
    N, n_ant, spd, P = 1024, 4, 8, 4
    chunk = N * spd
    x = synth.generate(synth.array_spec(n_ant, chunk * 4, 5, corr=0.3, max_lag=9))
    st = qc.Stream(n_ant, chunk, N, P, spd, depth=2)
    outs = [torch.empty((1, 10, N // 2), dtype=torch.complex64, device="cuda") for _ in range(3)]
    st.push(_pinned(x[:, :chunk]), 0, outs[0])
    st.push(_pinned(x[:, chunk:2 * chunk]), 1, outs[1])
    st.push(_pinned(x[:, 3 * chunk:]), 3, outs[2])              # chunk 2 dropped
    st.sync()
    alone = qc.xcorrelate(torch.from_numpy(np.ascontiguousarray(x[:, 3 * chunk:])).cuda(), N, P, spd)
    assert vis_err(outs[2].cpu().numpy(), alone.cpu().numpy(), n_ant) <= 1e-6
    with pytest.raises(qc.QCError):
        st.push(_pinned(x[:, :chunk]), 3, outs[0])               # sequence must increase
    st.close()


@pytest.mark.gpu
@pytest.mark.parametrize("spd,chunk_dumps", [(8, 2), (2, 3)])
def test_stream_dropped_chunk_zero_fill_and_weights(qc, spd, chunk_dumps):
    """A dropped chunk (pushed as None) counts as zeros: its dumps are zero
    visibilities with no valid spectrum, and the next chunk equals that
    chunk correlated alone from a zero history.  Valid spectra per dump:
    spec_per_dump, less the first P-1 spectra after a zero-filled history
    (stream start, a dropped chunk, a gap); with spec_per_dump < P-1 the
    deficit runs on into the following dumps."""
    import torch
    N, n_ant, P = 256, 3, 4
    chunk = N * spd * chunk_dumps
    x = synth.generate(synth.array_spec(n_ant, chunk * 6, 9, corr=0.3, max_lag=5))
    st = qc.Stream(n_ant, chunk, N, P, spd, depth=2)
    nb = n_ant * (n_ant + 1) // 2
    out = {k: torch.full((chunk_dumps, nb, N // 2), 7.0 + 0j, dtype=torch.complex64, device="cuda")
           for k in range(6)}
    hosts = {k: _pinned(x[:, k * chunk:(k + 1) * chunk]) for k in range(6)}

    def fresh():
        w, bad = [], P - 1
        for _ in range(chunk_dumps):
            k = min(bad, spd)
            w.append(spd - k)
            bad -= k
        return w

    full = [spd] * chunk_dumps
    weights = {}
    for k in (0, 1):
        assert st.push(hosts[k], k, out[k]) == chunk_dumps
        weights[k] = st.valid_spectra()
    assert st.push(None, 2, out[2]) == chunk_dumps           # dropped: zero-filled
    weights[2] = st.valid_spectra()
    st.push(hosts[3], 3, out[3])
    weights[3] = st.valid_spectra()
    st.push(hosts[5], 5, out[5])                             # chunk 4 missing: a gap
    weights[5] = st.valid_spectra()
    st.sync()
    assert weights == {0: fresh(), 1: full, 2: [0] * chunk_dumps, 3: fresh(), 5: fresh()}
    assert torch.count_nonzero(out[2]).item() == 0
    one = qc.xcorrelate(torch.from_numpy(np.ascontiguousarray(x[:, :2 * chunk])).cuda(), N, P, spd)
    got = torch.cat([out[0], out[1]]).cpu().numpy()
    assert vis_err(got, one.cpu().numpy(), n_ant) <= 1e-6
    for k in (3, 5):
        alone = qc.xcorrelate(hosts[k].cuda(), N, P, spd)
        assert vis_err(out[k].cpu().numpy(), alone.cpu().numpy(), n_ant) <= 1e-6
    st.close()


@pytest.mark.skipif(not os.path.exists(qc_mod.LIB_PATH), reason="libqc.so not built")
def test_stream_valid_spectra_rejects_bad_arguments():
    L = qc_mod.lib()
    n = (ctypes.c_int64 * 4)()
    assert L.qc_stream_valid_spectra(None, n, 4) == -1
