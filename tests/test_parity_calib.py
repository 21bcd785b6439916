"""GPU parity: MAD flagging (bit-exact masks and thresholds) and delay/phase
application (within one float32 rounding of the float64 oracle)."""

import numpy as np
import pytest

from oracle import calib, mad

pytestmark = pytest.mark.gpu


def _vis(shape, seed, outliers=0.01, ties=False):
    rng = np.random.default_rng(seed)
    v = (rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(np.complex64)
    n_out = int(outliers * v.size)
    idx = rng.choice(v.size, n_out, replace=False)
    v.flat[idx] *= np.complex64(30.0)
    if ties:   # many exactly equal amplitudes
        v = (np.round(v.real) + 1j * np.round(v.imag)).astype(np.complex64)
    return v


@pytest.mark.parametrize("shape,pop", [
    ((16, 10, 2048), 0),     # real-time dump shape, per baseline plane
    ((7, 3, 33), 0),         # odd counts
    ((8, 3, 32), 0),         # even counts
    ((16, 10, 64), 1),       # per (baseline, channel) over time
    ((5, 6, 31), 2),         # per (baseline, time) over channel
    ((1, 1, 1), 0),          # single value
    ((2, 1, 1), 0),          # two values
    ((9, 2, 8192), 0),       # 73728 per plane: beyond the LDS cache (re-read from HBM)
    ((256, 1, 2048), 0),     # the flagger's plane: 524288 per baseline
])
def test_mad_bit_exact(qc, shape, pop):
    import torch
    for ties in (False, True):
        v = _vis(shape, seed=sum(shape) + pop, ties=ties)
        m_ref, T_ref = mad.mad_flag(v, 5.0, pop)
        m, T = qc.mad_flag(torch.from_numpy(v).cuda(), 5.0, pop)
        assert np.array_equal(m.cpu().numpy(), m_ref)
        assert np.array_equal(T.cpu().numpy(), T_ref)


def test_mad_offset_plane(qc):
    # a plane that starts one visibility past an aligned address takes the
    # scalar amplitude pass, an aligned one the 16-byte pass: both bit-exact
    import torch
    shape = (8, 3, 4096)
    v = _vis(shape, seed=77)
    m_ref, T_ref = mad.mad_flag(v, 5.0, 0)
    buf = torch.zeros(v.size + 1, dtype=torch.complex64, device="cuda")
    for off in (0, 1):
        d = buf[off:off + v.size].view(shape)
        d.copy_(torch.from_numpy(v).cuda())
        assert (d.data_ptr() % 32 == 0) == (off == 0)
        m, T = qc.mad_flag(d, 5.0, 0)
        assert np.array_equal(m.cpu().numpy(), m_ref), off
        assert np.array_equal(T.cpu().numpy(), T_ref), off


def _tie_plane(shape, pop, pattern, rng):
    """Real-valued visibilities (amplitude exactly |v|) with a tie structure
    inside every population:
    0: half the values 1, half 2 (the middle pair straddles two large
       groups of equal keys, every deviation equals 0.5);
    1: 30 % 1, 40 % 2, 30 % 3 (the median inside a group);
    2: half exactly 1, half spread over (1, 2) (the middle pair at the
       edge of a tie group);
    3: a spread with two huge outliers."""
    n_time, n_base, n_chan = shape
    npop = {0: n_base, 1: n_base * n_chan, 2: n_time * n_base}[pop]
    n = {0: n_time * n_chan, 1: n_time, 2: n_chan}[pop]
    A = np.empty((npop, n))
    idx = np.arange(n)
    for q in range(npop):
        if pattern == 0:
            a = np.where(idx < n // 2, 1.0, 2.0)
        elif pattern == 1:
            a = np.where(idx < 3 * n // 10, 1.0, np.where(idx < 7 * n // 10, 2.0, 3.0))
        elif pattern == 2:
            a = np.where(idx < n // 2, 1.0, 1.0 + rng.uniform(0.01, 0.99, n))
        else:
            a = rng.uniform(0.5, 1.5, n)
            a[rng.choice(n, min(2, n), replace=False)] = 1e6
        A[q] = rng.permutation(a) * rng.choice([-1.0, 1.0], n)
    if pop == 0:
        V = A.reshape(n_base, n_time, n_chan).transpose(1, 0, 2)
    elif pop == 1:
        V = A.reshape(n_base, n_chan, n_time).transpose(2, 0, 1)
    else:
        V = A.reshape(n_time, n_base, n_chan)
    return np.ascontiguousarray(V).astype(np.float32).astype(np.complex64)


@pytest.mark.parametrize("shape,pop", [((8, 2, 512), 0), ((4, 3, 4096), 2), ((1, 2, 100), 0),
                                       ((64, 2, 5), 1)])
def test_mad_tie_structures(qc, shape, pop):
    """Bit-exact on populations whose middle order statistics sit at or
    inside large groups of equal amplitudes: the selection resolves every
    bit, or ranks k and k+1 fall in different digits too large to gather,
    and the counting pass finds rank k+1 (single-wave and 1024-thread
    kernels)."""
    import torch
    rng = np.random.default_rng(11)
    for pattern in range(4):
        v = _tie_plane(shape, pop, pattern, rng)
        m_ref, T_ref = mad.mad_flag(v, 5.0, pop)
        m, T = qc.mad_flag(torch.from_numpy(v).cuda(), 5.0, pop)
        assert np.array_equal(T.cpu().numpy(), T_ref), pattern
        assert np.array_equal(m.cpu().numpy(), m_ref), pattern


def test_mad_sigma_zero_and_constant(qc):
    import torch
    v = np.full((4, 2, 16), 3 + 4j, np.complex64)
    v[0, 0, 0] = 30 + 40j
    m_ref, T_ref = mad.mad_flag(v, 0.0, 0)
    m, T = qc.mad_flag(torch.from_numpy(v).cuda(), 0.0, 0)
    assert np.array_equal(m.cpu().numpy(), m_ref) and np.array_equal(T.cpu().numpy(), T_ref)
    assert T_ref[0] == 5.0      # MAD = 0 gives T = median


@pytest.mark.parametrize("n_time,n_ant,n_chan", [(16, 4, 2048), (3, 7, 100), (1, 32, 64)])
def test_apply_matches_oracle(qc, n_time, n_ant, n_chan):
    import torch
    rng = np.random.default_rng(n_ant)
    nb = n_ant * (n_ant + 1) // 2
    v = (rng.normal(size=(n_time, nb, n_chan)) + 1j * rng.normal(size=(n_time, nb, n_chan))).astype(np.complex64)
    tau = rng.uniform(0, 40e-9, n_ant)
    phi = rng.uniform(-np.pi, np.pi, n_ant)
    f0, df = 1.05e9, 1e9 / 4096
    ref = calib.apply_delay_phase(v, n_ant, f0, df, tau, phi)
    vd = torch.from_numpy(v).cuda()
    qc.apply_delay_phase(vd, n_ant, f0, df, tau, phi)
    out = vd.cpu().numpy()
    # float64 rotation, one rounding to float32 per component
    bound = 2.0 ** -23 * np.abs(ref) + 1e-30
    assert np.all(np.abs(out.real - ref.real) <= bound)
    assert np.all(np.abs(out.imag - ref.imag) <= bound)
    # autos untouched, bitwise
    for a in range(n_ant):
        b = a * n_ant - a * (a - 1) // 2
        assert np.array_equal(out[:, b], v[:, b])


def test_apply_zero_is_identity_and_inverse(qc):
    import torch
    n_ant, nb = 4, 10
    rng = np.random.default_rng(2)
    v = (rng.normal(size=(2, nb, 256)) + 1j * rng.normal(size=(2, nb, 256))).astype(np.complex64)
    vd = torch.from_numpy(v).cuda()
    qc.apply_delay_phase(vd, n_ant, 0.0, 1e6, np.zeros(4), np.zeros(4))
    assert np.array_equal(vd.cpu().numpy(), v)
    tau, phi = rng.uniform(0, 4e-8, 4), rng.uniform(-3, 3, 4)
    qc.apply_delay_phase(vd, n_ant, 1.3e9, 2.4e5, tau, phi)
    qc.apply_delay_phase(vd, n_ant, 1.3e9, 2.4e5, -tau, -phi)
    assert np.allclose(vd.cpu().numpy(), v, rtol=0, atol=1e-5 * np.abs(v).max())
