"""Training and evaluation of the surrogate on runs of the coupled method.

Features: mu_s, mu_r, drop radius, log10(body force), particle contact angle,
particle radius, each standardised with the training set's mean and standard
deviation; targets: the outcome class and the 48 displacement values, the
latter standardised per output.  The surrogate's answer for a run is accepted
when its largest softmax probability is at least `confidence`; otherwise the
run falls back to the plain method.
"""
from __future__ import annotations

import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DATA = os.path.join(HERE, "data")
TRAIN_FILES = ("surrogate_runs_train.npz",)
HELDOUT_FILES = ("surrogate_runs_heldout.npz",)


def load(files):
    parts = [np.load(os.path.join(DATA, f)) for f in files]
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0].files}


def features(params):
    f = np.asarray(params, np.float64).copy()
    f[:, 3] = np.log10(f[:, 3])
    return f


class Scaler:
    def __init__(self, a):
        self.mean = a.mean(axis=0)
        self.std = a.std(axis=0) + 1e-12

    def __call__(self, a):
        return (a - self.mean) / self.std

    def inverse(self, a):
        return a * self.std + self.mean


def train_and_evaluate(train, held, epochs=200, batch=256, lr=1e-3, w_traj=1.0, seed=0,
                       confidence=0.9, infer_batch=65536, init_seed=1):
    import torch
    from .surrogate import Surrogate, flatten, he_init
    xs = Scaler(features(train["params"]))
    tr_flat = train["traj"].reshape(len(train["traj"]), -1)
    ts = Scaler(tr_flat)
    Xt = xs(features(train["params"]))
    Yt = ts(tr_flat)
    n_train = (len(Xt) // batch) * batch
    s = Surrogate(max_batch=max(infer_batch, batch), max_train=len(Xt))
    s.set_params(flatten(he_init(init_seed)))
    s.set_train(Xt, train["label"], Yt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = s.train(epochs, batch=batch, lr=lr, w_traj=w_traj, seed=seed)
    t_train = time.perf_counter() - t0
    # held-out runs
    Xh = xs(features(held["params"]))
    y = s.predict(Xh)
    logits = y[:, :3].astype(np.float64)
    p = np.exp(logits - logits.max(axis=1, keepdims=True))
    p /= p.sum(axis=1, keepdims=True)
    pred = np.argmax(p, axis=1)
    conf = p.max(axis=1)
    lab = held["label"]
    traj_pred = ts.inverse(y[:, 3:].astype(np.float64)).reshape(held["traj"].shape)
    err = traj_pred - held["traj"]
    rmse = float(np.sqrt(np.mean(err ** 2)))
    base_rmse = float(np.sqrt(np.mean((held["traj"] - train["traj"].mean(axis=0)) ** 2)))
    final_err = np.sqrt(np.sum(err[:, -1, :] ** 2, axis=1))
    accept = conf >= confidence
    counts = np.bincount(train["label"], minlength=3)
    out = dict(
        n_train=int(n_train), epochs=epochs, train_s=round(t_train, 2),
        loss_first=float(losses[0]), loss_last=float(losses[-1]),
        accuracy=float(np.mean(pred == lab)),
        majority_accuracy=float(np.mean(lab == np.argmax(counts))),
        per_class_recall=[float(np.mean(pred[lab == c] == c)) if np.any(lab == c) else None
                          for c in range(3)],
        traj_rmse_lu=rmse, traj_rmse_constant_lu=base_rmse,
        final_disp_err_median_lu=float(np.median(final_err)),
        fallback_fraction=float(1.0 - accept.mean()),
        accepted_accuracy=float(np.mean(pred[accept] == lab[accept])) if accept.any() else None,
    )
    # inference throughput, device-resident batch
    g = torch.Generator(device="cpu").manual_seed(0)
    Xd = torch.randn(infer_batch, 6, generator=g).to("cuda")
    Yd = torch.empty(infer_batch, 51, device="cuda")
    s.predict_device(Xd, Yd)
    s.sync()
    reps = 20
    st = s.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        s.predict_device(Xd, Yd)
    e1.record(st)
    s.sync()
    ms = e0.elapsed_time(e1) / reps
    flops = 2.0 * infer_batch * sum(a * b for a, b in ((6, 256), (256, 256), (256, 256),
                                                       (256, 256), (256, 51)))
    out.update(infer_batch=infer_batch, infer_us=round(ms * 1e3, 1),
               infer_tflops=round(flops / (ms * 1e-3) / 1e12, 2))
    s.close()
    return out
