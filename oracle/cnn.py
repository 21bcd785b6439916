"""Learned RFI flagger: a small convolutional network over per-baseline
dynamic spectra |V_b(t, f)|.

The paper flags RFI with a MAD threshold on visibility amplitude (Sec. 7,
eq. 2) and notes that RFI is structured in time and frequency (Sec. 5:
persistent narrowband lines, intermittent and broadband bursts).  The
network learns that structure from synthetic streams with known injected
RFI; MAD stays the fallback and the judge of its flags.

Readings (the paper defines none of this; every choice is ours):
  * architecture: four 'same'-padded, stride-1 cross-correlation layers
        L1  3x3,              1 -> 32, ReLU
        L2  5x5,             32 -> 32, ReLU
        L3  5x5, dilation 2, 32 -> 32, ReLU
        L4  1x1,             32 ->  1  (logit)
    51,617 parameters, stored flat as W1, b1, W2, b2, W3, b3, W4, b4 with
    W[out][in][ky][kx] (row-major);
  * input: per baseline, A = |V| as float32 (the MAD oracle's amplitude),
    robust z-score r = (A - med) / (1.4826 * MAD) over the baseline's whole
    (time x channel) plane (scale 1 when MAD = 0), then x = sign(r) log1p|r|;
  * loss: binary cross-entropy on the logits, positives weighted by
    pos_weight, averaged over cells;
  * optimiser: Adam (Kingma & Ba) with bias correction;
  * decision: flag iff logit > threshold (0 = probability 0.5).

Everything is float64.  Status: pinned (tests/test_oracle_cnn.py):
correlation against scipy.signal.correlate2d, gradients against central
finite differences, loss and Adam closed forms, normalisation closed form.
"""

from __future__ import annotations

import numpy as np

from .mad import amplitude_f32, median_sorted

# (in, out, kernel, dilation) per layer
LAYERS = ((1, 32, 3, 1), (32, 32, 5, 1), (32, 32, 5, 2), (32, 1, 1, 1))


def param_shapes():
    out = []
    for ci, co, k, _ in LAYERS:
        out.append((co, ci, k, k))
        out.append((co,))
    return out


def param_count() -> int:
    return int(sum(np.prod(s) for s in param_shapes()))


def unflatten(flat):
    """Flat parameter vector -> [W1, b1, W2, b2, W3, b3, W4, b4] (views)."""
    flat = np.asarray(flat, np.float64)
    out, o = [], 0
    for s in param_shapes():
        n = int(np.prod(s))
        out.append(flat[o:o + n].reshape(s))
        o += n
    assert o == flat.size
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in parts])


def conv2d(x, w, b, dil):
    """out[o, y, x] = b[o] + sum_{c, ky, kx} w[o, c, ky, kx] * x[c, y + dil*ky - R, x + dil*kx - R],
    R = dil*(K-1)/2, zero outside the image.  x: [C, H, W]."""
    C, H, W = x.shape
    O, C2, K, _ = w.shape
    assert C == C2
    R = dil * (K - 1) // 2
    xp = np.zeros((C, H + 2 * R, W + 2 * R))
    xp[:, R:R + H, R:R + W] = x
    out = np.zeros((O, H, W)) + np.asarray(b, np.float64)[:, None, None]
    for ky in range(K):
        for kx in range(K):
            patch = xp[:, ky * dil:ky * dil + H, kx * dil:kx * dil + W]
            out += np.einsum("oc,chw->ohw", w[:, :, ky, kx], patch)
    return out


def conv2d_backward(x, w, dil, g):
    """Gradients of sum(g * conv2d(x, w, b, dil)) w.r.t. x, w and b."""
    C, H, W = x.shape
    O, _, K, _ = w.shape
    R = dil * (K - 1) // 2
    xp = np.zeros((C, H + 2 * R, W + 2 * R))
    xp[:, R:R + H, R:R + W] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w, dtype=np.float64)
    for ky in range(K):
        for kx in range(K):
            sl = (slice(None), slice(ky * dil, ky * dil + H), slice(kx * dil, kx * dil + W))
            dw[:, :, ky, kx] = np.einsum("ohw,chw->oc", g, xp[sl])
            dxp[sl] += np.einsum("oc,ohw->chw", w[:, :, ky, kx], g)
    db = g.sum(axis=(1, 2))
    return dxp[:, R:R + H, R:R + W], dw, db


def forward(params, x):
    """Logits [H, W] for one normalised image x [H, W]; also the activations."""
    p = unflatten(params)
    acts = [np.asarray(x, np.float64)[None]]
    h = acts[0]
    for li, (_, _, _, dil) in enumerate(LAYERS):
        z = conv2d(h, p[2 * li], p[2 * li + 1], dil)
        h = np.maximum(z, 0.0) if li < len(LAYERS) - 1 else z
        acts.append(h)
    return acts[-1][0], acts


def softplus(z):
    z = np.asarray(z, np.float64)
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    z = np.asarray(z, np.float64)
    return np.where(z >= 0, 1.0 / (1.0 + np.exp(-np.abs(z))), np.exp(-np.abs(z)) / (1.0 + np.exp(-np.abs(z))))


def bce_loss(logits, labels, pos_weight):
    """mean over cells of  pw*y*softplus(-z) + (1-y)*softplus(z)."""
    z = np.asarray(logits, np.float64)
    y = np.asarray(labels, np.float64)
    return float(np.mean(pos_weight * y * softplus(-z) + (1.0 - y) * softplus(z)))


def bce_grad(logits, labels, pos_weight):
    """d loss / d logits for bce_loss (same shape)."""
    z = np.asarray(logits, np.float64)
    y = np.asarray(labels, np.float64)
    s = sigmoid(z)
    return (-pos_weight * y * (1.0 - s) + (1.0 - y) * s) / z.size


def loss_and_grad(params, images, labels, pos_weight):
    """Mean BCE over every cell of a batch of images [n, H, W] and its
    gradient w.r.t. the flat parameters (explicit backpropagation)."""
    images = np.asarray(images, np.float64)
    labels = np.asarray(labels, np.float64)
    n = images.shape[0]
    p = unflatten(params)
    grads = [np.zeros_like(q) for q in p]
    total = 0.0
    count = labels.size
    for i in range(n):
        z, acts = forward(params, images[i])
        y = labels[i]
        total += float(np.sum(pos_weight * y * softplus(-z) + (1.0 - y) * softplus(z)))
        s = sigmoid(z)
        g = ((-pos_weight * y * (1.0 - s) + (1.0 - y) * s) / count)[None]
        for li in range(len(LAYERS) - 1, -1, -1):
            dil = LAYERS[li][3]
            dx, dw, db = conv2d_backward(acts[li], p[2 * li], dil, g)
            grads[2 * li] += dw
            grads[2 * li + 1] += db
            if li > 0:
                g = dx * (acts[li] > 0.0)     # ReLU of the layer below
    return total / count, flatten(grads)


def adam_step(w, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t >= 1); returns new (w, m, v)."""
    w = np.asarray(w, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def normalize_plane(vis_plane):
    """Network input for one baseline's plane vis[t, f] (complex64)."""
    A = amplitude_f32(vis_plane).astype(np.float64)
    med = median_sorted(A)
    mad = median_sorted(np.abs(A - med))
    scale = 1.4826 * mad
    if scale == 0.0:
        scale = 1.0
    r = (A - med) / scale
    return np.sign(r) * np.log1p(np.abs(r))


def normalize(vis):
    """vis [n_time, n_base, n_chan] -> images [n_base, n_time, n_chan]."""
    V = np.asarray(vis)
    return np.stack([normalize_plane(V[:, b, :]) for b in range(V.shape[1])])


def flag(params, vis, threshold=0.0):
    """Inference mask [n_time, n_base, n_chan] (uint8): logit > threshold."""
    X = normalize(vis)
    out = np.zeros(np.asarray(vis).shape, np.uint8)
    for b in range(X.shape[0]):
        z, _ = forward(params, X[b])
        out[:, b, :] = (z > threshold).astype(np.uint8)
    return out
