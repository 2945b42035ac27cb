"""FP64 CPU reference of the outcome/trajectory surrogate network.

TEST INFRASTRUCTURE ONLY: used by the test suite to check the GPU kernels'
forward pass, gradients and optimiser step.  Nothing in the product library
imports it.

The network maps the six run parameters (mu_s, mu_r, drop radius, body force,
particle contact angle, particle radius; standardised by the caller) to three
outcome logits (picked up / pushed / left behind, the outcome classes of the
section on particle removal) and the particle's displacement at 16 times
(48 values, standardised).  Layers: 6 -> 256 -> 256 -> 256 -> 256 -> 51, ReLU
between layers, none after the last.

Loss per batch of B samples:
    L = mean_b CE(softmax(y_b[0:3]), label_b) + w * mean_{b,j} (y_b[3+j] - t_b[j])^2
with CE the cross-entropy.  Optimiser: Adam (Kingma and Ba, 2015) with bias
correction, lr, beta1 = 0.9, beta2 = 0.999, eps = 1e-8.

Parameters are lists [W1, b1, ..., W5, b5] with W_l of shape (in, out).
"""
from __future__ import annotations

import numpy as np

SIZES = (6, 256, 256, 256, 256, 51)
N_CLASS = 3
N_TRAJ = 48


def init_params(seed: int, sizes=SIZES):
    """He-normal weights, zero biases (numpy Generator(PCG64(seed)))."""
    g = np.random.Generator(np.random.PCG64(seed))
    ps = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        ps.append(g.normal(0.0, np.sqrt(2.0 / a), size=(a, b)))
        ps.append(np.zeros(b))
    return ps


def forward(params, X):
    """Returns the output y (B, 51) and the per-layer activations (inputs of
    each layer: X, h1, ..., h4)."""
    acts = [np.asarray(X, np.float64)]
    h = acts[0]
    n = len(params) // 2
    for l in range(n):
        z = h @ params[2 * l] + params[2 * l + 1]
        if l < n - 1:
            h = np.maximum(z, 0.0)
            acts.append(h)
        else:
            h = z
    return h, acts


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss(y, label, traj, w_traj=1.0):
    B = y.shape[0]
    p = softmax(y[:, :N_CLASS])
    ce = -np.log(p[np.arange(B), label]).mean()
    mse = ((y[:, N_CLASS:] - traj) ** 2).mean()
    return ce + w_traj * mse


def output_gradient(y, label, traj, w_traj=1.0):
    """dL/dy: (softmax - onehot)/B on the logits, 2 w (y - t)/(B * 48) on the
    trajectory outputs."""
    B = y.shape[0]
    g = np.zeros_like(y)
    p = softmax(y[:, :N_CLASS])
    p[np.arange(B), label] -= 1.0
    g[:, :N_CLASS] = p / B
    g[:, N_CLASS:] = 2.0 * w_traj * (y[:, N_CLASS:] - traj) / (B * N_TRAJ)
    return g


def gradients(params, X, label, traj, w_traj=1.0):
    """Backpropagation: list of dL/dparam in the order of params, and L."""
    y, acts = forward(params, X)
    L = loss(y, label, traj, w_traj)
    dz = output_gradient(y, label, traj, w_traj)
    n = len(params) // 2
    grads = [None] * len(params)
    for l in range(n - 1, -1, -1):
        grads[2 * l] = acts[l].T @ dz
        grads[2 * l + 1] = dz.sum(axis=0)
        if l > 0:
            dh = dz @ params[2 * l].T
            dz = dh * (acts[l] > 0.0)
    return grads, L


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new params, m, v."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1.0 - b1) * g
        vv = b2 * vv + (1.0 - b2) * g * g
        mh = mm / (1.0 - b1 ** t)
        vh = vv / (1.0 - b2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v
