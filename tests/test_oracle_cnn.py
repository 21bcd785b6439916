"""Pins of the CNN-flagger oracle against routes other than itself:
scipy's 2-D correlation, central finite differences of the loss, the closed
forms of the loss, its gradient and Adam's first steps, and a normalisation
worked by hand."""

import numpy as np
import pytest
from scipy import signal

from oracle import cnn


def _params(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for (co, ci, k, k2) in [s for s in cnn.param_shapes() if len(s) == 4]:
        fan_in = ci * k * k2
        parts.append(rng.normal(0, scale * np.sqrt(2.0 / fan_in), (co, ci, k, k2)))
        parts.append(rng.normal(0, 0.1, co))
    return cnn.flatten(parts)


def test_param_count_matches_architecture():
    # 3x3 1->32, 5x5 32->32 twice, 1x1 32->1, with biases
    assert cnn.param_count() == (9 * 32 + 32) + 2 * (25 * 32 * 32 + 32) + (32 + 1) == 51617


@pytest.mark.parametrize("dil,K", [(1, 3), (1, 5), (2, 5), (1, 1), (3, 3)])
def test_conv2d_equals_scipy_correlate(dil, K):
    rng = np.random.default_rng(dil * 10 + K)
    C, O, H, W = 3, 2, 9, 11
    x = rng.normal(size=(C, H, W))
    w = rng.normal(size=(O, C, K, K))
    b = rng.normal(size=O)
    out = cnn.conv2d(x, w, b, dil)
    E = (K - 1) * dil + 1
    for o in range(O):
        ref = np.full((H, W), b[o])
        for c in range(C):
            kd = np.zeros((E, E))
            kd[::dil, ::dil] = w[o, c]
            ref += signal.correlate2d(x[c], kd, mode="same", boundary="fill")
        np.testing.assert_allclose(out[o], ref, rtol=1e-12, atol=1e-12)


def test_conv2d_offset_is_a_correlation_not_a_convolution():
    # a single off-centre tap picks the neighbour in the +x direction
    x = np.zeros((1, 5, 5))
    x[0, 2, 3] = 1.0
    w = np.zeros((1, 1, 3, 3))
    w[0, 0, 1, 2] = 1.0          # ky = 1 (centre row), kx = 2 (right)
    out = cnn.conv2d(x, w, np.zeros(1), 1)
    assert out[0, 2, 2] == 1.0 and out.sum() == 1.0


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    params = _params(1)
    imgs = rng.normal(size=(2, 5, 6))
    labels = (rng.random((2, 5, 6)) < 0.3).astype(np.float64)
    pw = 2.5
    loss, g = cnn.loss_and_grad(params, imgs, labels, pw)

    def L(p):
        return sum(cnn.bce_loss(cnn.forward(p, imgs[i])[0], labels[i], pw) * labels[i].size
                   for i in range(2)) / labels.size

    assert abs(L(params) - loss) < 1e-13
    # indices spread over every tensor of every layer
    sizes = [int(np.prod(s)) for s in cnn.param_shapes()]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    idx = []
    for t in range(len(sizes)):
        idx += list(rng.choice(np.arange(offs[t], offs[t + 1]), min(6, sizes[t]), replace=False))
    h = 1e-6
    for i in idx:
        e = np.zeros_like(params)
        e[i] = h
        fd = (L(params + e) - L(params - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bce_closed_forms():
    y = np.array([[1.0, 0.0], [0.0, 1.0]])
    z = np.zeros_like(y)
    pw = 3.0
    assert cnn.bce_loss(z, y, pw) == pytest.approx(np.log(2) * (pw * 2 + 2) / 4, rel=1e-14)
    np.testing.assert_allclose(cnn.bce_grad(z, y, pw), np.where(y > 0, -pw * 0.5, 0.5) / 4, rtol=1e-14)
    # far from zero: softplus(z) -> z, softplus(-z) -> 0
    zz = np.array([[40.0, -40.0], [40.0, -40.0]])
    yy = np.array([[1.0, 0.0], [0.0, 1.0]])
    assert cnn.bce_loss(zz, yy, 1.0) == pytest.approx((0 + 0 + 40 + 40) / 4, rel=1e-12)
    assert cnn.sigmoid(np.array(-800.0)) == 0.0 and cnn.sigmoid(np.array(800.0)) == 1.0


def test_adam_first_two_steps():
    w = np.array([1.0, -2.0, 0.5])
    g1 = np.array([0.2, -3.0, 0.0])
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    w1, m, v = cnn.adam_step(w, g1, np.zeros(3), np.zeros(3), 1, lr, b1, b2, eps)
    # step 1: bias-corrected moments are g and g^2
    np.testing.assert_allclose(w1, w - lr * g1 / (np.abs(g1) + eps), rtol=1e-14)
    g2 = np.array([-0.1, 1.0, 2.0])
    w2, _, _ = cnn.adam_step(w1, g2, m, v, 2, lr, b1, b2, eps)
    m2 = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    v2 = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    np.testing.assert_allclose(w2, w1 - lr * m2 / (np.sqrt(v2) + eps), rtol=1e-13)


def test_normalisation_worked_example():
    # amplitudes 1..9 on a 3x3 plane: median 5, |A - 5| = 4,3,2,1,0,1,2,3,4 -> MAD 2
    A = np.arange(1.0, 10.0).reshape(3, 3)
    vis = (A * np.exp(1j * 0.7)).astype(np.complex64)
    x = cnn.normalize_plane(vis)
    r = (A - 5.0) / (1.4826 * 2.0)
    np.testing.assert_allclose(x, np.sign(r) * np.log1p(np.abs(r)), rtol=1e-6)
    assert x[1, 1] == 0.0 and x[0, 0] < 0 < x[2, 2]
    # MAD = 0 falls back to scale 1
    flat = np.full((2, 3), 3.0 + 4.0j, np.complex64)
    flat[0, 0] = 9.0
    np.testing.assert_allclose(cnn.normalize_plane(flat).ravel(), [np.log1p(4.0)] + [0.0] * 5)


def test_zero_last_layer_gives_constant_logits():
    p = cnn.unflatten(_params(5).copy())
    p[6][:] = 0.0
    p[7][:] = -1.25
    z, _ = cnn.forward(cnn.flatten(p), np.random.default_rng(0).normal(size=(4, 7)))
    assert np.all(z == -1.25)
