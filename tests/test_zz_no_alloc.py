"""GPU parity of qc_xcorrelate_noalloc (the fused float32 F+X with its work
memory in the library's fixed device array) against qc_xcorrelate on the
same input, through the C ABI: two calls in a row, the second with a
smaller input, and a stream long enough to need several batches of dumps."""

import numpy as np
import pytest

import synth
from tests.util import vis_err

pytestmark = pytest.mark.gpu


def _pair(qc, x, N, P, spd, hist=None):
    import torch
    xd = torch.from_numpy(x).cuda()
    hd = None if hist is None else torch.from_numpy(hist).cuda()
    ref = qc.xcorrelate(xd, N, P, spd, hist=hd)
    n_dump = (x.shape[1] // N) // spd
    vis = torch.full((n_dump, x.shape[0] * (x.shape[0] + 1) // 2, N // 2), complex(7.0, -3.0),
                     dtype=torch.complex64, device="cuda")
    qc.xcorrelate_noalloc(xd, N, P, spd, vis, hist=hd)
    torch.cuda.synchronize()
    return vis.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_matches_xcorrelate_twice_second_smaller(qc):
    n_ant, N, P = 4, 1024, 4
    x1 = synth.generate(synth.array_spec(n_ant, N * 64 * 6, 11, corr=0.3, max_lag=7))
    V, R = _pair(qc, x1, N, P, 64)
    assert V.shape == R.shape == (6, 10, 512)
    e1 = vis_err(V, R, n_ant)
    x2 = synth.generate(synth.array_spec(n_ant, N * 32 * 2, 12, corr=0.3, max_lag=7))
    V2, R2 = _pair(qc, x2, N, P, 32)
    assert V2.shape == (2, 10, 512)
    e2 = vis_err(V2, R2, n_ant)
    print(f"noalloc vs xcorrelate: {e1:.2e}, {e2:.2e}")
    assert e1 <= 1e-5 and e2 <= 1e-5


@pytest.mark.parametrize("n_ant,N,spd,n_dump", [(4, 4096, 8, 450), (8, 2048, 8, 250), (2, 1024, 1, 6000)])
def test_noalloc_batches_and_history(qc, n_ant, N, spd, n_dump):
    """More dumps than the work array holds partial sums for (399, 222 and
    5333 dumps at one workgroup each), so the call runs several batches: a
    caller history on the first batch, the stream's own samples on the
    later ones."""
    P = 4
    x = synth.generate(synth.array_spec(n_ant, N * spd * n_dump, 13 + n_ant, corr=0.3, max_lag=7))
    hist = np.random.default_rng(5).integers(-60, 60, (n_ant, (P - 1) * N)).astype(np.int8)
    V, R = _pair(qc, x, N, P, spd, hist=hist)
    err = vis_err(V, R, n_ant)
    print(f"noalloc {n_ant} ant N={N}: {err:.2e}")
    assert err <= 1e-5


def test_noalloc_rejects_unfused_shape(qc):
    import torch
    x = torch.zeros((3, 1024 * 4), dtype=torch.int8, device="cuda")
    vis = torch.empty((1, 6, 512), dtype=torch.complex64, device="cuda")
    with pytest.raises(qc.QCError):
        qc.xcorrelate_noalloc(x, 1024, 4, 4, vis)
