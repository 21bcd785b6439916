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
