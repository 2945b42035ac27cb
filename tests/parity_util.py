"""Comparison helpers of the GPU parity tests (GPU fields and particle records
against the FP64 oracle's).

Bars: masks bit-exact; FP32-storage fields rho, u, phi within 1e-5 relative L2
over the fluid nodes, and at every fluid node next to a solid (wetting nodes,
particle link nodes, freshly uncovered nodes) within 1e-4 of the field's
largest magnitude, so that a wrong value at a few branch nodes cannot hide in
the global norm; FP16 storage: relative L2 within 1e-3.
"""
import numpy as np

C19 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
       (1, 1, 0), (1, -1, 0), (-1, 1, 0), (-1, -1, 0), (1, 0, 1), (1, 0, -1), (-1, 0, 1),
       (-1, 0, -1), (0, 1, 1), (0, 1, -1), (0, -1, 1), (0, -1, -1)]


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def boundary_nodes(mask):
    """Fluid nodes (mask 0) with at least one solid D3Q19 neighbour (periodic
    indexing), mask shaped (nz, ny, nx)."""
    solid = mask != 0
    nb = np.zeros_like(solid)
    for cx, cy, cz in C19[1:]:
        nb |= np.roll(solid, shift=(-cz, -cy, -cx), axis=(0, 1, 2))
    return (~solid) & nb


def compare_fields(g, o, tol=1e-5, node_tol=1e-4, label="", fields=None, open_x=False):
    """GPU context g against oracle o (or precomputed oracle fields).  Returns
    the relative L2 errors and the boundary-node errors.  open_x: the planes
    x = 0 and x = nx - 1 (pressure-boundary nodes) count as boundary nodes."""
    rg, ug, pg, mg = g.fields()
    ro, uo, po, mo = fields if fields is not None else o.fields()
    assert np.array_equal(mg, mo), f"{label}: masks differ at {np.argwhere(mg != mo)[:5]}"
    fl = mo == 0
    e = dict(rho=rel_l2(rg[fl], ro[fl]), u=rel_l2(ug[:, fl], uo[:, fl]),
             phi=rel_l2(pg[fl], po[fl]))
    bn = boundary_nodes(mo)
    if open_x:
        bn[:, :, 0] |= fl[:, :, 0]
        bn[:, :, -1] |= fl[:, :, -1]
    en = {}
    if bn.any():
        for k, a, b in (("rho", rg, ro), ("u", ug, uo), ("phi", pg, po)):
            sel = (slice(None), bn) if k == "u" else bn
            allf = (slice(None), fl) if k == "u" else fl
            scale = np.abs(np.asarray(b, np.float64)[allf]).max()
            en[k] = float(np.abs(np.asarray(a, np.float64)[sel] - b[sel]).max() / scale)
    print(label, "rel-L2", {k: f"{v:.2e}" for k, v in e.items()},
          f"| {int(bn.sum())} boundary nodes, max error / field max",
          {k: f"{v:.2e}" for k, v in en.items()}, flush=True)
    for k, v in e.items():
        assert v <= tol, (label, k, v)
    if node_tol is not None:
        for k, v in en.items():
            assert v <= node_tol, (label, "boundary node", k, v)
    return e, en


def compare_particles(pg, po, keys, label="", tol=1e-5, R=None):
    """Per quantity, max |gpu - oracle| over the particles within tol of the
    largest oracle magnitude.  Torques are also reported against R max|F| of
    the force of the same kind; that scale is used only where the torque is
    much smaller than it (|T| < 0.1 R |F|: a residual of cancelling moments)."""
    out = {}
    for k in keys:
        a = np.array([p[k] for p in pg], np.float64)
        b = np.array([p[k] for p in po], np.float64)
        err = np.abs(a - b).max()
        scale = np.abs(b).max()
        out[k] = err / scale if scale > 0 else err
        if k.startswith("T_") and R is not None:
            fk = "F_" + k[2:]
            rF = R * np.abs(np.array([p[fk] for p in po])).max()
            print(f"{label} {k}: err/max|T| {out[k]:.2e}, err/(R max|F|) {err / rF:.2e}, "
                  f"max|T|/(R max|F|) {scale / rF:.3f}", flush=True)
            if scale < 0.1 * rF:
                out[k] = err / rF
        else:
            print(f"{label} {k}: err/max {out[k]:.2e}", flush=True)
        assert out[k] <= tol, (label, k, out[k])
    return out


def compare_history(hg, ho, names, R, label="", tol=1e-5):
    """Per-step particle histories (steps x 3 per quantity), the same policy."""
    out = {}
    for k, name in enumerate(names):
        a, b = hg[:, 3 * k:3 * k + 3], ho[:, 3 * k:3 * k + 3]
        err = np.abs(a - b).max()
        scale = np.abs(b).max()
        e = err / scale if scale > 0 else err
        if name.startswith("T_"):
            kf = names.index("F_" + name[2:])
            rF = R * np.abs(ho[:, 3 * kf:3 * kf + 3]).max()
            print(f"{label} {name}: err/max|T| {e:.2e}, err/(R max|F|) {err / rF:.2e}, "
                  f"max|T|/(R max|F|) {scale / rF:.3f}", flush=True)
            if scale < 0.1 * rF:
                e = err / rF
        else:
            print(f"{label} {name}: err/max {e:.2e}", flush=True)
        out[name] = e
        assert e <= tol, (label, name, e)
    return out


def oracle_fields_at(args):
    """Worker for a process pool: (cfg, phi0, particles, marks, threads,
    probe) -> the oracle's (rho, u, phi, mask, particle centres) after each
    step count in marks.
    probe "f32" (or True): the state's departures from rest are rounded to
    single precision after every step; "f16": every total population is
    rounded as a 16-bit store relative to its node's density would round it
    (sensitivity probes of the method to the storage, not the method)."""
    cfg, phi0, parts, marks, threads, probe = args
    round_f32 = probe in (True, "f32", "f16")
    from oracle import oracle as O
    from oracle.oracle import OracleSim
    O.set_num_threads(threads)
    o = OracleSim(cfg, phi0, parts)
    out, t = [], 0
    for mk in marks:
        while t < mk:
            if round_f32:
                o.step(1)
                if probe == "f16":
                    o.round_state_f16()
                else:
                    o.round_state_f32()
                t += 1
            else:
                o.step(mk - t)
                t = mk
        out.append(tuple(o.fields()) + (np.array([q["x"] for q in o.particles()]),))
    o.close()
    return out


def oracle_runs_parallel(jobs):
    """Oracle runs of several (cfg, phi0, particles, marks, probe) jobs in
    parallel processes, the host's cores split between them."""
    import multiprocessing as mp
    import os
    threads = max(1, (len(os.sched_getaffinity(0)) or 2) // len(jobs))
    ctx = mp.get_context("spawn")
    with ctx.Pool(len(jobs)) as pool:
        return pool.map(oracle_fields_at, [(c, p, q, m, threads, r) for c, p, q, m, r in jobs])
