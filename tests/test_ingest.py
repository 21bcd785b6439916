"""File ingest (Alg. 1 reader threads, pinned buffers, bounded queue; the
batch-packets / queue-max knobs of Sec. 6).

CPU: argument checks that happen before any device call.  GPU: visibilities
from files equal the resident stream's (same kernels, history carried
across batches) for batches smaller than, equal to and larger than a dump,
one or several reader threads, queue depths 1..16 and 16-bit words, and
the oracle's on a small case."""

import os

import numpy as np
import pytest

import synth
from oracle import pfb, xengine
from tests.util import vis_err


def _write(tmp_path, x, name="ant"):
    paths = []
    for a in range(x.shape[0]):
        p = os.path.join(str(tmp_path), f"{name}{a}.raw")
        np.ascontiguousarray(x[a]).tofile(p)
        paths.append(p)
    return paths


def _lib():
    import paper_2604_20640_amd as qc
    try:
        return qc, qc.lib()
    except ImportError:
        pytest.skip("libqc.so not built")


def _cfg(qc, n_ant, packet, batch, qmax, N=256, P=4, spd=16, sample=0, readers=1, depth=2):
    return qc.IngestConfig(n_ant, sample, packet, batch, qmax, readers, depth, qc.PfbParams(N, P, None, 0), spd)


def test_ingest_rejects_bad_configs(tmp_path):
    import ctypes
    qc, L = _lib()
    x = np.zeros((2, 4096), np.int8)
    paths = _write(tmp_path, x)
    arr = (ctypes.c_char_p * 2)(*[os.fsencode(p) for p in paths])
    st = qc.IngestStats()
    bad = [
        _cfg(qc, 2, 100, 1, 2),            # batch not a whole number of spectra
        _cfg(qc, 2, 256, 3, 2, spd=2),     # 3 spectra per batch vs 2 per dump
        _cfg(qc, 2, 256, 1, 0),            # queue_max 0
        _cfg(qc, 2, 256, 1, 2, N=100),     # n_fft not a power of two
        _cfg(qc, 2, 256, 1, 2, sample=7),  # bad word
        _cfg(qc, 2, 256, 1, 2, depth=0),
    ]
    for c in bad:
        assert L.qc_ingest_run(arr, ctypes.byref(c), None, -1, ctypes.byref(st)) == -1
    missing = (ctypes.c_char_p * 2)(os.fsencode(paths[0]), b"/nonexistent/antenna1.raw")
    c = _cfg(qc, 2, 256, 1, 2)
    assert L.qc_ingest_run(missing, ctypes.byref(c), None, -1, ctypes.byref(st)) == -1
    assert b"cannot open" in L.qc_last_error()


@pytest.mark.gpu
@pytest.mark.parametrize("packet,batch,qmax,readers,spd", [
    (1024, 4, 2, 1, 16),      # 4 spectra per batch, 4 batches per dump
    (4096, 4, 4, 4, 16),      # one dump per batch
    (4096, 8, 1, 2, 16),      # two dumps per batch, queue of one
    (1024, 1, 16, 3, 64),     # one spectrum per batch, deep queue
])
def test_ingest_equals_resident_stream(qc, tmp_path, packet, batch, qmax, readers, spd):
    import torch
    n_ant, N, P = 4, 1024, 4
    S = N * spd * 6 + 3000          # six dumps and a ragged tail
    x = synth.generate(synth.array_spec(n_ant, S, 61, corr=0.3, max_lag=9))
    paths = _write(tmp_path, x)
    V, stats = qc.ingest_run(paths, N, P, spd, packet, batch, qmax, n_readers=readers)
    n_full = (S // (packet * batch)) * (packet * batch)
    ref = qc.xcorrelate(torch.from_numpy(np.ascontiguousarray(x[:, :n_full])).cuda(), N, P, spd)
    assert V.shape[0] == stats["dumps"] == ref.shape[0]
    R = ref.cpu().numpy()[:V.shape[0]]
    assert vis_err(V.cpu().numpy(), R, n_ant) <= 1e-6
    assert stats["bytes"] == stats["batches"] * n_ant * packet * batch
    assert stats["wall_s"] > 0 and stats["h2d_s"] > 0 and stats["compute_s"] > 0


@pytest.mark.gpu
def test_ingest_matches_oracle_int16(qc, tmp_path):
    n_ant, N, P, spd = 3, 256, 4, 8
    spec = synth.StreamSpec(n_ant, N * spd * 5, 62, sigma=1500.0, corr=0.3, lags=(0, 2, 5), bits=14)
    x = synth.generate(spec)
    paths = _write(tmp_path, x)
    V, stats = qc.ingest_run(paths, N, P, spd, N, 4, 3, sample="i16")   # 4 spectra per batch
    V_ref = xengine.correlate_fast(pfb.channelize(x, N, P), spd)
    assert V.shape == V_ref.shape == (5, 6, N // 2)
    assert vis_err(V.cpu().numpy(), V_ref, n_ant) <= 1e-5


@pytest.mark.gpu
def test_ingest_max_dumps(qc, tmp_path):
    n_ant, N, P, spd = 2, 256, 4, 4
    x = synth.generate(synth.array_spec(n_ant, N * spd * 10, 63, corr=0.3, max_lag=3))
    paths = _write(tmp_path, x)
    # three dumps per batch: a limit of 7 dumps takes two batches (6 dumps)
    V, stats = qc.ingest_run(paths, N, P, spd, N, 3 * spd, 2, max_dumps=7)
    assert stats["dumps"] == 6 and V.shape[0] == 6
    V_ref = xengine.correlate_fast(pfb.channelize(x[:, :N * spd * 6], N, P), spd)
    assert vis_err(V.cpu().numpy(), V_ref, n_ant) <= 1e-5
