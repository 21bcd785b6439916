"""Training and evaluation of the learned RFI flagger.

The flagger is trained on visibilities the correlator itself produces from
synthetic streams with known injected RFI (persistent lines, broadband
bursts, linear chirps; per-channel SNR log-uniform in [1, 50]) and judged
against the truth and against MAD (Sec. 7, eq. 2, sigma = 5), which stays
the fallback flagger.  Every numerical step runs in the library's kernels
(correlation, normalisation, forward, backward, Adam, flagging); this
module only draws training tiles and counts agreements.

    python -m paper_2604_20640_amd.flagger --out weights.npy --metrics m.json
    python -m paper_2604_20640_amd.flagger --train-seeds 200 --train-ant 32 \
        --test-seeds 50 --test-ant 32 --tiles-per-set 64 --steps 1500
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

import paper_2604_20640_amd as qc

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)
import synth  # noqa: E402


def realise(seed, n_ant, n_samp=1 << 24, device="cuda"):
    """(vis [n_int, n_base, n_chan] complex64, truth [n_int, n_chan] uint8, params)."""
    spec, truth, params = synth.rfi_realisation(seed, n_ant=n_ant, n_samp=n_samp)
    x = torch.from_numpy(synth.generate(spec)).to(device)
    vis = qc.xcorrelate(x, params["n_fft"], params["n_taps"], params["spec_per_dump"])
    del x
    return vis, torch.from_numpy(truth).to(device), params


def init_params(seed=0, device="cuda"):
    """He-normal weights, zero biases, in the library's flat layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for (ci, co, k) in ((1, 32, 3), (32, 32, 5), (32, 32, 5), (32, 1, 1)):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (ci * k * k)), (co, ci, k, k)).ravel())
        parts.append(np.zeros(co))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == qc.cnn_param_count()
    return torch.from_numpy(flat).to(device)


class TileSampler:
    """Random (time x channel) tiles of normalised planes and their truth."""

    def __init__(self, sets, tile=(64, 256), seed=0):
        self.images, self.truth = [], []
        for vis, truth, _ in sets:
            self.images.append(qc.cnn_normalize(vis))   # [n_base, n_int, n_chan]
            self.truth.append(truth)                     # [n_int, n_chan]
        self.tile = tile
        self.g = torch.Generator(device="cpu").manual_seed(seed)
        pos = sum(float(t.float().sum()) for t in self.truth)
        tot = sum(t.numel() for t in self.truth)
        self.pos_frac = pos / tot

    def batch(self, n):
        th, tw = self.tile
        xs, ys = [], []
        for _ in range(n):
            k = int(torch.randint(len(self.images), (1,), generator=self.g))
            img, tr = self.images[k], self.truth[k]
            nb, T, F = img.shape
            b = int(torch.randint(nb, (1,), generator=self.g))
            t0 = int(torch.randint(T - th + 1, (1,), generator=self.g))
            f0 = int(torch.randint(F - tw + 1, (1,), generator=self.g))
            xs.append(img[b, t0:t0 + th, f0:f0 + tw])
            ys.append(tr[t0:t0 + th, f0:f0 + tw])
        return torch.stack(xs).contiguous(), torch.stack(ys).contiguous()


class TilePool:
    """A fixed pool of training tiles: each realisation contributes
    `per_set` random (time x channel) tiles of random baselines of its
    normalised plane, and the plane is then freed, so many realisations fit
    in device memory.  Batches are drawn from the pool with replacement."""

    def __init__(self, per_set, tile=(64, 256), seed=0):
        self.per_set, self.tile = per_set, tile
        self.g = torch.Generator(device="cpu").manual_seed(seed)
        self.xs, self.ys = [], []
        self.X = self.Y = None

    def add(self, vis, truth):
        img = qc.cnn_normalize(vis)          # [n_base, n_int, n_chan]
        th, tw = self.tile
        nb, T, F = img.shape
        for _ in range(self.per_set):
            b = int(torch.randint(nb, (1,), generator=self.g))
            t0 = int(torch.randint(T - th + 1, (1,), generator=self.g))
            f0 = int(torch.randint(F - tw + 1, (1,), generator=self.g))
            self.xs.append(img[b, t0:t0 + th, f0:f0 + tw].clone())
            self.ys.append(truth[t0:t0 + th, f0:f0 + tw].clone())
        del img

    def finalize(self):
        self.X = torch.stack(self.xs).contiguous()
        self.Y = torch.stack(self.ys).contiguous()
        self.xs, self.ys = [], []
        self.pos_frac = float(self.Y.float().mean())

    def batch(self, n):
        idx = torch.randint(self.X.shape[0], (n,), generator=self.g).to(self.X.device)
        return self.X[idx].contiguous(), self.Y[idx].contiguous()


def summarise(results):
    """Mean, standard deviation, minimum and maximum of every rate over the
    held-out realisations."""
    out = {}
    for group in results[0]:
        out[group] = {}
        for key in results[0][group]:
            v = np.array([r[group][key] for r in results], np.float64)
            out[group][key] = {"mean": round(float(v.mean()), 4), "std": round(float(v.std()), 4),
                               "min": round(float(v.min()), 4), "max": round(float(v.max()), 4)}
    return out


def train(sampler, steps=400, batch=32, lr=1e-3, seed=0, log_every=50, log=print):
    params = init_params(seed)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    pw = float(min(30.0, max(1.0, (1.0 - sampler.pos_frac) / max(sampler.pos_frac, 1e-6))))
    losses = []
    for step in range(1, steps + 1):
        x, y = sampler.batch(batch)
        loss = qc.cnn_train_step(params, m, v, step, x, y, pw, lr=lr)
        if step % log_every == 0 or step == steps:
            losses.append((step, float(loss.item())))
            log(f"[flagger] step {step}: loss {losses[-1][1]:.4f}")
    return params, {"pos_weight": pw, "losses": losses}


def _rates(pred, ref):
    tp = float((pred & ref).sum())
    fp = float((pred & ~ref).sum())
    fn = float((~pred & ref).sum())
    prec = tp / (tp + fp) if tp + fp else 0.0
    rec = tp / (tp + fn) if tp + fn else 0.0
    f1 = 2 * prec * rec / (prec + rec) if prec + rec else 0.0
    return {"precision": round(prec, 4), "recall": round(rec, 4), "f1": round(f1, 4),
            "flagged_frac": round(float(pred.float().mean()), 5)}


def evaluate(params, vis, truth, sigma=5.0, threshold=0.0, act="f32"):
    """CNN and MAD masks against the truth, and the CNN judged by MAD."""
    cnn = qc.cnn_flag(params, vis, threshold, act=act).bool()
    mad, _ = qc.mad_flag(vis, sigma, 0)
    mad = mad.bool()
    tr = truth.bool()[:, None, :].expand_as(cnn)
    out = {"cnn_vs_truth": _rates(cnn, tr), "mad_vs_truth": _rates(mad, tr)}
    n_cnn, n_mad = float(cnn.sum()), float(mad.sum())
    out["cnn_judged_by_mad"] = {
        # flags MAD does not raise, as a fraction of the CNN's flags
        "false_flag_rate": round(float((cnn & ~mad).sum()) / n_cnn, 4) if n_cnn else 0.0,
        # MAD flags the CNN misses, as a fraction of MAD's flags
        "missed_flag_rate": round(float((~cnn & mad).sum()) / n_mad, 4) if n_mad else 0.0,
    }
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-seeds", type=int, default=8)
    ap.add_argument("--test-seeds", type=int, default=2)
    ap.add_argument("--train-ant", type=int, default=8)
    ap.add_argument("--test-ant", type=int, default=32)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", type=str, default=None)
    ap.add_argument("--metrics", type=str, default=None)
    ap.add_argument("--tiles-per-set", type=int, default=0,
                    help="keep this many random tiles per training realisation (0: whole planes)")
    ap.add_argument("--act", type=str, default="f32", help="inference activations for the test set")
    a = ap.parse_args(argv)
    t0 = time.time()
    if a.tiles_per_set > 0:
        sampler = TilePool(a.tiles_per_set, seed=1)
        for s in range(a.train_seeds):
            vis, truth, _ = realise(s, a.train_ant)
            sampler.add(vis, truth)
            del vis, truth
            if (s + 1) % 10 == 0:
                print(f"[flagger] {s + 1} training realisations in {time.time() - t0:.1f}s", flush=True)
        sampler.finalize()
    else:
        sets = [realise(s, a.train_ant) for s in range(a.train_seeds)]
        sampler = TileSampler(sets, seed=1)
        del sets
    print(f"[flagger] {a.train_seeds} training realisations in {time.time() - t0:.1f}s", flush=True)
    t0 = time.time()
    params, info = train(sampler, a.steps, a.batch, a.lr, log=lambda s: print(s, flush=True))
    torch.cuda.synchronize()
    info["train_s"] = round(time.time() - t0, 2)
    del sampler
    results = []
    t0 = time.time()
    for s in range(200, 200 + a.test_seeds):
        vis, truth, _ = realise(s, a.test_ant)
        results.append(evaluate(params, vis, truth, act=a.act))
        print(f"[flagger] test seed {s}: {results[-1]}", flush=True)
        del vis
    info["test_s"] = round(time.time() - t0, 2)
    info["config"] = {"train_seeds": a.train_seeds, "train_ant": a.train_ant, "test_seeds": a.test_seeds,
                      "test_ant": a.test_ant, "steps": a.steps, "batch": a.batch, "lr": a.lr,
                      "tiles_per_set": a.tiles_per_set, "act": a.act}
    info["test"] = results
    info["test_summary"] = summarise(results)
    if a.out:
        np.save(a.out, params.cpu().numpy())
    if a.metrics:
        with open(a.metrics, "w") as f:
            json.dump(info, f, indent=1)
    print(json.dumps(info), flush=True)


if __name__ == "__main__":
    main()
