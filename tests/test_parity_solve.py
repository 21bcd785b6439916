"""GPU parity: the delay/phase solve (Sec. 7 three-step calibration)."""

import numpy as np
import pytest

import synth
from oracle import calib, mad, pfb, xengine

pytestmark = pytest.mark.gpu


def _noiseless(n_ant, C, f0, df, tau, phi, n_time=2):
    pairs = [(i, j) for i in range(n_ant) for j in range(i, n_ant)]
    f = f0 + df * np.arange(C)
    V = np.zeros((n_time, len(pairs), C), np.complex64)
    for b, (i, j) in enumerate(pairs):
        V[:, b] = 1e3 * np.exp(-1j * (2 * np.pi * f * (tau[i] - tau[j]) + (phi[i] - phi[j])))
    return V


@pytest.mark.parametrize("n_ant,C", [(4, 2048), (5, 512), (32, 256), (2, 64)])
def test_solve_recovers_noiseless(qc, n_ant, C):
    import torch
    rng = np.random.default_rng(n_ant)
    fs = 1e9
    df = fs / (2 * C)
    tau = np.concatenate([[0.0], rng.uniform(-40e-9, 40e-9, n_ant - 1)])
    phi = np.concatenate([[0.0], rng.uniform(-3, 3, n_ant - 1)])
    f0 = 1.05e9
    V = _noiseless(n_ant, C, f0, df, tau, phi)
    lo, hi = C // 8, C - C // 8
    t, p = qc.solve_delay_phase(torch.from_numpy(V).cuda(), n_ant, f0, df, 0, lo, hi)
    # tau within 1e-3 of a sample (1 ps at 1 GS/s), phase within 1e-4 rad
    assert np.max(np.abs(t - tau)) < 1e-3 / fs, np.max(np.abs(t - tau))
    assert np.max(np.abs(calib.wrap(p - phi))) < 1e-4
    to, po = calib.solve_delay_phase(V, None, n_ant, f0, df, 0, lo, hi)
    assert np.max(np.abs(t - to)) < 1e-3 / fs
    assert np.max(np.abs(calib.wrap(p - po))) < 1e-4


@pytest.mark.parametrize("seed,sign", [(7, 1.0), (8, -1.0)])
def test_solve_steep_noisy_phases_need_the_coarse_step(qc, seed, sign):
    """Cross phases stepping up to 0.92 pi per channel (both signs), with
    bounded phase noise that moves each step by up to 0.7 pi: unwrapping
    without the coarse delay (Sec. 7 step 1) mistracks, so agreement with
    the oracle and with the injected delays checks the GPU's coarse argmax."""
    import torch
    n_ant, C = 4, 512
    f0, df = 0.3e9, 1e9 / 4096
    tau = sign * np.array([0.0, 0.22, -0.24, 0.1]) / df
    phi = np.array([0.0, 1.1, -2.5, 0.3])
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(n_ant) for j in range(i, n_ant)]
    f = f0 + df * np.arange(C)
    V = np.zeros((2, len(pairs), C), np.complex64)
    for b, (i, j) in enumerate(pairs):
        eps = rng.uniform(-0.35 * np.pi, 0.35 * np.pi, C) if i != j else 0.0
        V[:, b] = 1e3 * np.exp(-1j * (2 * np.pi * f * (tau[i] - tau[j]) + (phi[i] - phi[j])) + 1j * eps)
    lo, hi = 40, 480
    t, p = qc.solve_delay_phase(torch.from_numpy(V).cuda(), n_ant, f0, df, 0, lo, hi)
    to, po = calib.solve_delay_phase(V, None, n_ant, f0, df, 0, lo, hi)
    assert np.max(np.abs(t - to)) < 1e-3 / 1e9, np.max(np.abs(t - to))
    assert np.max(np.abs(calib.wrap(p - po))) < 1e-4
    assert np.max(np.abs(t - tau)) < 0.5e-9


def test_solve_matches_oracle_on_pipeline_output(qc):
    """Correlated stream with injected lags -> visibilities -> MAD flags ->
    solve: GPU and oracle agree, and the solution matches the lags."""
    import torch
    N, P, spd, n_ant = 1024, 4, 64, 4
    spec = synth.StreamSpec(n_ant, N * spd * 4, 77, corr=1.0, lags=(0, 3, 11, 6))
    x = synth.generate(spec)
    V = qc.xcorrelate(torch.from_numpy(x).cuda(), N, P, spd)
    m, _ = qc.mad_flag(V, 5.0, 0)
    fs = 1e9
    df = fs / N
    lo, hi = 16, 496
    t, p = qc.solve_delay_phase(V, n_ant, 0.0, df, 0, lo, hi, mask=m)
    Vh, mh = V.cpu().numpy(), m.cpu().numpy()
    to, po = calib.solve_delay_phase(Vh, mh, n_ant, 0.0, df, 0, lo, hi)
    assert np.max(np.abs(t - to)) < 1e-3 / fs
    assert np.max(np.abs(calib.wrap(p - po))) < 1e-3
    # the lag differences are recovered (lags are integer samples at fs)
    assert np.max(np.abs(t * fs - np.array([0, 3, 11, 6]))) < 0.05
    # applying the solution flattens the cross phases over the band
    qc.apply_delay_phase(V, n_ant, 0.0, df, t, p)
    W = V.cpu().numpy()[:, :, lo:hi]
    for b in [1, 2, 3, 5, 6, 8]:
        assert np.abs(np.angle(W[:, b].sum())) < 0.05


def test_solve_rejects(qc):
    import torch
    V = torch.zeros((1, 10, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(qc.QCError):
        qc.solve_delay_phase(V, 4, 0.0, 1e6, 0, 10, 10)     # empty band
    with pytest.raises(qc.QCError):
        qc.solve_delay_phase(V, 4, 0.0, 1e6, 4, 0, 64)      # ref out of range
    with pytest.raises(qc.QCError):
        qc.solve_delay_phase(V, 4, 0.0, -1.0, 0, 0, 64)     # df <= 0
