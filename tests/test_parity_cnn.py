"""CNN flagger kernels against the float64 oracle.

Bars (float32 kernels against a float64 reference):
  * logits: |z - z_ref| <= 1e-5 * max(1, max|z_ref|)  (sums of <= 801 float32
    products per layer, four layers);
  * gradients: per parameter tensor, max|g - g_ref| <= 1e-4 * max|g_ref| (each
    weight gradient is a float32 sum over every pixel of the batch);
  * loss: relative 1e-5;  Adam: relative 1e-6;  normalised input: 1e-6 abs;
  * flags: equal wherever the oracle's logit is farther than 1e-3 from the
    threshold (a float32 logit may fall on the other side of it only there).
Half-activation inference (L2/L3 on the matrix cores) is compared with the
oracle's forward pass with the same roundings inserted (L2/L3 weights and
the L1..L3 activations rounded to binary16, round to nearest even): the
remaining difference is float32 accumulation order plus the rare activation
that rounds to the neighbouring half, bounded by 2e-3 * max(1, max|z|);
against the unrounded oracle it is within 3e-2 * max(1, max|z|).
"""

import ctypes

import numpy as np
import pytest

from oracle import cnn

SHAPES = [s for s in cnn.param_shapes()]


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 4:
            fan_in = s[1] * s[2] * s[3]
            parts.append(rng.normal(0, scale * np.sqrt(2.0 / fan_in), s))
        else:
            parts.append(rng.normal(0, 0.05, s))
    return cnn.flatten(parts).astype(np.float32)


def _t(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ---------------------------------------------------------------- CPU checks

def test_cnn_entry_points_reject_bad_arguments():
    import paper_2604_20640_amd as qc
    try:
        L = qc.lib()
    except OSError:
        pytest.skip("library not built")
    assert L.qc_cnn_param_count() == cnn.param_count()
    assert L.qc_cnn_forward(None, None, 1, 8, 8, 0, None, None) == -1
    buf = ctypes.create_string_buffer(64)
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.qc_cnn_forward(p, p, 0, 8, 8, 0, p, None) == -1           # no images
    assert L.qc_cnn_forward(p, p, 1 << 20, 1 << 10, 1 << 10, 0, p, None) == -1   # > 2^31 cells
    assert L.qc_cnn_forward(p, p, 1, 8, 8, 2, p, None) == -1           # unknown activation type
    assert L.qc_cnn_grad(p, p, p, 1, 8, 8, -1.0, p, p, None) == -1     # pos_weight <= 0
    assert L.qc_cnn_adam(p, p, p, p, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -1   # step 0
    assert L.qc_cnn_adam(p, p, p, p, 1, 1e-3, 1.0, 0.999, 1e-8, None) == -1   # beta1 = 1
    assert L.qc_cnn_flag(p, p, 0, 1, 8, 0.0, 0, p, None) == -1
    assert L.qc_cnn_flag(p, p, 4, 1, 8, 0.0, 5, p, None) == -1
    assert L.qc_cnn_normalize(None, 4, 1, 8, p, None) == -1


# ---------------------------------------------------------------- GPU parity

@pytest.fixture(params=[0, 1], ids=["mfma", "valu"])
def cnn_variant(request, qc):
    """Run the test with the float32 convolutions and weight gradients on the
    matrix cores (0) and on the vector ALU (1)."""
    old = qc.cnn_variant()
    qc.cnn_variant(request.param)
    yield request.param
    qc.cnn_variant(old)


@pytest.mark.gpu
@pytest.mark.parametrize("n,H,W", [(2, 13, 37), (1, 8, 32), (3, 5, 70), (1, 1, 1), (2, 21, 9), (130, 3, 40)])
def test_forward_matches_oracle(qc, cnn_variant, n, H, W):
    # 130 x 3 x 40 gives more pixel tiles than the matrix-core kernel's workgroups
    import torch
    p = _params(n * 100 + H)
    x = np.random.default_rng(H * W).normal(0, 1.0, (n, H, W)).astype(np.float32)
    z = qc.cnn_forward(_t(p), _t(x))
    torch.cuda.synchronize()
    z = z.cpu().numpy()
    for i in range(n):
        zr, _ = cnn.forward(p.astype(np.float64), x[i].astype(np.float64))
        assert np.max(np.abs(z[i] - zr)) <= 1e-5 * max(1.0, np.max(np.abs(zr))), i


@pytest.mark.gpu
@pytest.mark.parametrize("n,H,W,pw", [(2, 11, 40, 2.5), (1, 16, 33, 1.0), (3, 6, 7, 7.0)])
def test_grad_matches_oracle(qc, n, H, W, pw):
    import torch
    rng = np.random.default_rng(n + H + W)
    p = _params(H * 7 + W)
    x = rng.normal(0, 1.0, (n, H, W)).astype(np.float32)
    y = (rng.random((n, H, W)) < 0.25).astype(np.uint8)
    g, loss = qc.cnn_grad(_t(p), _t(x), _t(y), pw)
    torch.cuda.synchronize()
    g, loss = g.cpu().numpy(), float(loss.cpu().numpy()[0])
    loss_ref, g_ref = cnn.loss_and_grad(p.astype(np.float64), x.astype(np.float64), y, pw)
    assert abs(loss - loss_ref) <= 1e-5 * abs(loss_ref)
    o = 0
    for s in SHAPES:
        k = int(np.prod(s))
        ref = g_ref[o:o + k]
        assert np.max(np.abs(g[o:o + k] - ref)) <= 1e-4 * np.max(np.abs(ref)) + 1e-12, (s, o)
        o += k


@pytest.mark.gpu
@pytest.mark.parametrize("n,H,W", [(2, 19, 70), (130, 3, 40), (300, 8, 1)])
def test_grad_variants_match_oracle(qc, cnn_variant, n, H, W):
    # both kernel sets; 130 x 3 x 40 and 300 x 8 x 1 give more pixel tiles
    # than workgroups, so workgroups work through several ragged tiles
    import torch
    rng = np.random.default_rng(n * H + W)
    p = _params(n + H + W)
    x = rng.normal(0, 1.0, (n, H, W)).astype(np.float32)
    y = (rng.random((n, H, W)) < 0.2).astype(np.uint8)
    g, loss = qc.cnn_grad(_t(p), _t(x), _t(y), 3.0)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    loss_ref, g_ref = cnn.loss_and_grad(p.astype(np.float64), x.astype(np.float64), y, 3.0)
    assert abs(float(loss.cpu().numpy()[0]) - loss_ref) <= 1e-5 * abs(loss_ref)
    o = 0
    for s in SHAPES:
        k = int(np.prod(s))
        ref = g_ref[o:o + k]
        assert np.max(np.abs(g[o:o + k] - ref)) <= 1e-4 * np.max(np.abs(ref)) + 1e-12, (s, o)
        o += k


@pytest.mark.gpu
def test_grad_is_deterministic(qc):
    import torch
    rng = np.random.default_rng(4)
    p = _t(_params(9))
    x = _t(rng.normal(size=(4, 64, 96)).astype(np.float32))
    y = _t((rng.random((4, 64, 96)) < 0.1).astype(np.uint8))
    g1, l1 = qc.cnn_grad(p, x, y, 3.0)
    g2, l2 = qc.cnn_grad(p, x, y, 3.0)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


@pytest.mark.gpu
def test_adam_matches_oracle(qc):
    import torch
    rng = np.random.default_rng(1)
    P = cnn.param_count()
    w = rng.normal(size=P).astype(np.float32)
    g = rng.normal(size=P).astype(np.float32)
    m = (0.1 * rng.normal(size=P)).astype(np.float32)
    v = np.abs(0.1 * rng.normal(size=P)).astype(np.float32)
    tw, tm, tv = _t(w.copy()), _t(m.copy()), _t(v.copy())
    qc.cnn_adam(tw, _t(g), tm, tv, 7, lr=3e-3, beta1=0.8, beta2=0.99, eps=1e-6)
    torch.cuda.synchronize()
    wr, mr, vr = cnn.adam_step(w, g, m, v, 7, 3e-3, 0.8, 0.99, 1e-6)
    np.testing.assert_allclose(tm.cpu().numpy(), mr, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(tv.cpu().numpy(), vr, rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(tw.cpu().numpy(), wr, rtol=1e-6, atol=1e-7)


@pytest.mark.gpu
@pytest.mark.parametrize("n_time,n_base,n_chan", [(7, 3, 50), (16, 1, 2048), (64, 6, 33)])
def test_normalize_matches_oracle(qc, n_time, n_base, n_chan):
    import torch
    rng = np.random.default_rng(n_chan)
    vis = (rng.normal(size=(n_time, n_base, n_chan)) + 1j * rng.normal(size=(n_time, n_base, n_chan)))
    vis = (vis * np.exp(rng.normal(size=(1, n_base, 1)))).astype(np.complex64)
    vis[0, 0, :3] = 40.0    # outliers
    x = qc.cnn_normalize(_t(vis))
    torch.cuda.synchronize()
    np.testing.assert_allclose(x.cpu().numpy(), cnn.normalize(vis), rtol=0, atol=1e-6)


@pytest.mark.gpu
def test_flag_matches_oracle(qc, cnn_variant):
    import torch
    rng = np.random.default_rng(12)
    n_time, n_base, n_chan = 16, 3, 40
    vis = (rng.normal(size=(n_time, n_base, n_chan)) + 1j * rng.normal(size=(n_time, n_base, n_chan)))
    vis[:, :, 7] *= 30.0          # a line
    vis[5, :, :] *= 20.0          # a burst
    vis = vis.astype(np.complex64)
    p = _params(3)
    thr = 0.0
    mask = qc.cnn_flag(_t(p), _t(vis), thr).cpu().numpy()
    X = cnn.normalize(vis)
    for b in range(n_base):
        zr, _ = cnn.forward(p.astype(np.float64), X[b])
        clear = np.abs(zr - thr) > 1e-3
        assert np.array_equal(mask[:, b, :][clear], (zr > thr)[clear]), b
        assert clear.mean() > 0.95


@pytest.mark.gpu
def test_train_steps_reduce_the_loss(qc):
    """A task the network can learn: flag cells whose input exceeds 1.5."""
    import torch
    rng = np.random.default_rng(8)
    x = rng.normal(size=(8, 32, 64)).astype(np.float32)
    y = (x > 1.5).astype(np.uint8)
    p = _t(_params(21, scale=0.5))
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    tx, ty = _t(x), _t(y)
    losses = []
    for step in range(1, 61):
        loss = qc.cnn_train_step(p, m, v, step, tx, ty, 4.0, lr=3e-3)
        losses.append(float(loss.cpu().numpy()[0]))
    assert losses[-1] < 0.5 * losses[0], (losses[0], losses[-1])
    # one train step is grad followed by Adam
    p2, m2, v2 = p.clone(), m.clone(), v.clone()
    qc.cnn_train_step(p, m, v, 61, tx, ty, 4.0, lr=3e-3)
    g, _ = qc.cnn_grad(p2, tx, ty, 4.0)
    qc.cnn_adam(p2, g, m2, v2, 61, lr=3e-3)
    torch.cuda.synchronize()
    assert torch.equal(p, p2) and torch.equal(m, m2) and torch.equal(v, v2)


def _forward_half_ref(p, x):
    """Oracle forward with the half-activation path's roundings."""
    P = cnn.unflatten(p.astype(np.float64))
    r16 = lambda a: a.astype(np.float16).astype(np.float64)  # noqa: E731
    h = np.asarray(x, np.float64)[None]
    for li, (_, _, _, dil) in enumerate(cnn.LAYERS):
        w = P[2 * li]
        if li in (1, 2):
            w = r16(w)
        z = cnn.conv2d(h, w, P[2 * li + 1], dil)
        h = r16(np.maximum(z, 0.0)) if li < 3 else z
    return h[0]


@pytest.mark.gpu
@pytest.mark.parametrize("n,H,W", [(2, 13, 37), (1, 16, 32), (1, 40, 70), (3, 5, 9), (1, 1, 1)])
def test_forward_half_matches_oracle(qc, n, H, W):
    import torch
    p = _params(n * 31 + H)
    x = np.random.default_rng(H + 7 * W).normal(0, 1.0, (n, H, W)).astype(np.float32)
    z = qc.cnn_forward(_t(p), _t(x), act="f16")
    torch.cuda.synchronize()
    z = z.cpu().numpy()
    for i in range(n):
        zq = _forward_half_ref(p, x[i])
        zr, _ = cnn.forward(p.astype(np.float64), x[i].astype(np.float64))
        scale = max(1.0, np.max(np.abs(zr)))
        assert np.max(np.abs(z[i] - zq)) <= 2e-3 * scale, (i, np.max(np.abs(z[i] - zq)))
        assert np.max(np.abs(z[i] - zr)) <= 3e-2 * scale


@pytest.mark.gpu
def test_flag_half_agrees_with_float(qc):
    import torch
    rng = np.random.default_rng(5)
    vis = (rng.normal(size=(64, 4, 256)) + 1j * rng.normal(size=(64, 4, 256)))
    vis[:, :, 40] *= 25.0
    vis[10, :, :] *= 15.0
    vis = _t(vis.astype(np.complex64))
    p = _t(_params(17))
    m32 = qc.cnn_flag(p, vis, 0.0, act="f32")
    m16 = qc.cnn_flag(p, vis, 0.0, act="f16")
    x = qc.cnn_normalize(vis)
    z = qc.cnn_forward(p, x)
    torch.cuda.synchronize()
    zc = z.cpu().numpy().transpose(1, 0, 2)          # [time][baseline][chan]
    # decided the same way wherever the float32 logit is beyond the half
    # path's error bound (3e-2 * max(1, max|z|)) from the threshold
    clear = np.abs(zc) > 3e-2 * max(1.0, np.abs(zc).max())
    assert np.array_equal(m32.cpu().numpy()[clear], m16.cpu().numpy()[clear])
    assert clear.mean() > 0.5
    assert np.mean(m32.cpu().numpy() == m16.cpu().numpy()) > 0.98
