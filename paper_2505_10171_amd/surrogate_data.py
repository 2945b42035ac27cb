"""Training data for the surrogate, produced by the coupled method itself.

Each run is an ensemble member of the uneven-box drop-particle distribution
(workloads.ensemble_member_c4 with index 0 and its own seed), advanced for its
5,000 steps in batched contexts of up to 256 runs.  Recorded per run:

* the six parameters (mu_s, mu_r, drop radius, body force, particle contact
  angle, particle radius);
* the particle's displacement from its start at steps round(k * 5000 / 16),
  k = 1..16, unwrapped across the periodic boundaries (48 values);
* the outcome class from the final state (the outcome taxonomy of the section on
  particle removal; thresholds are this project's): with dx_d the drop-centroid
  displacement along the drive and dx_p the particle's, the particle was
  *left behind* (2) if dx_p < 0.25 dx_d; otherwise *pushed* (1) if it ends
  ahead of the drop centroid (minimum-image x_p - x_d > 0), else *picked up* (0).

The drop centroid is the circular mean along x of the fluid-a fraction
(1 + phi)/2 over fluid nodes, unwrapped from sample to sample like the
particle position.

    python -m paper_2505_10171_amd.surrogate_data --seed-start 1000 --count 4096 --out FILE.npz
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np

PARAM_KEYS = ("mu_s", "mu_r", "R_d", "f_x", "theta_p", "R_p")
N_SAMPLES = 16
LABELS = ("picked up", "pushed", "left behind")


def drop_centroid_x(phi, mask):
    """Circular-mean x of the fluid-a fraction over fluid nodes (phi: nz,ny,nx)."""
    nx = phi.shape[2]
    w = np.where(mask == 0, 0.5 * (1.0 + phi.astype(np.float64)), 0.0).sum(axis=(0, 1))
    ang = 2.0 * np.pi * np.arange(nx) / nx
    a = np.arctan2((w * np.sin(ang)).sum(), (w * np.cos(ang)).sum())
    return (a % (2.0 * np.pi)) * nx / (2.0 * np.pi)


def minimage(d, L):
    return d - L * np.round(d / L)


def label_of(dxp, dxd, xp_end, xd_end, L):
    if dxp < 0.25 * dxd:
        return 2
    return 1 if minimage(xp_end - xd_end, L) > 0.0 else 0


def run_batch(seeds, storage="fp32", log=print):
    import torch
    from . import workloads as W
    from .lbm import Context
    members = [W.ensemble_member_c4(int(s), 0, storage=storage) for s in seeds]
    steps = members[0]["steps"]
    marks = [int(round(k * steps / N_SAMPLES)) for k in range(1, N_SAMPLES + 1)]
    stream = torch.cuda.Stream()
    ctx = Context(members, stream=stream)
    ctx.use_graph(True)
    n = len(members)
    L = np.array([m["cfg"]["nx"] for m in members], np.float64)
    x0 = np.array([m["particles"][0]["x"] for m in members], np.float64)
    xd_prev = np.array([drop_centroid_x(*ctx.phi_mask(i)) for i in range(n)])
    dxd = np.zeros(n)
    prev = x0.copy()
    disp = np.zeros((n, 3), np.float64)
    traj = np.zeros((n, N_SAMPLES, 3), np.float64)
    done = 0
    t0 = time.perf_counter()
    for k, t in enumerate(marks):
        ctx.step(t - done)
        done = t
        for i in range(n):
            x = np.array(ctx.particles(i)[0]["x"])
            d = x - prev[i]
            d[:2] = minimage(d[:2], L[i])  # periodic in x and y; z is bounded by the wall
            disp[i] += d
            prev[i] = x
            traj[i, k] = disp[i]
            # drop centroid, unwrapped mark to mark (it moves far less than L/2
            # between marks)
            xd = drop_centroid_x(*ctx.phi_mask(i))
            dxd[i] += minimage(xd - xd_prev[i], L[i])
            xd_prev[i] = xd
        log(f"  step {t}/{steps} ({time.perf_counter() - t0:.0f} s)")
    lab = np.array([label_of(traj[i, -1, 0], dxd[i], prev[i, 0], xd_prev[i], L[i])
                    for i in range(n)], np.int32)
    params = np.array([[m["params"][k] for k in PARAM_KEYS] for m in members], np.float64)
    ctx.close()
    return dict(seeds=np.asarray(seeds, np.int64), params=params, traj=traj, label=lab,
                drop_dx=dxd, L=L)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed-start", type=int, required=True)
    ap.add_argument("--count", type=int, required=True)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    parts = []
    for s0 in range(a.seed_start, a.seed_start + a.count, a.batch):
        seeds = list(range(s0, min(s0 + a.batch, a.seed_start + a.count)))
        t0 = time.perf_counter()
        print(f"batch of {len(seeds)} runs from seed {s0}", flush=True)
        parts.append(run_batch(seeds, a.storage, log=lambda m: print(m, flush=True)))
        lab = parts[-1]["label"]
        print(f"  done in {time.perf_counter() - t0:.0f} s; labels "
              f"{np.bincount(lab, minlength=3).tolist()}", flush=True)
        out = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
        np.savez_compressed(a.out, **out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
