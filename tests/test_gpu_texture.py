"""GPU against the FP64 oracle on a textured wall (LBM_WALL_BOXES: the plane
z = 0 with boxes of solid nodes; the paper names textured walls as future
work).

- a drop on a 2 x 2 array of pillars with a free sphere between them (the
  boxes' masks, bounce-back, the nearest-surface wetting normal at faces, edges
  and corners, the sphere's contacts with the pillars), FP32 and FP16;
- spheres held against a box's face, edge and corner: the contact force;
- a layer of packed spheres pressing on pillars, in the DEM placement that
  keeps everything in LDS and in the one that spreads over the GPU.

Bars as in tests/parity_util.py.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSim
from paper_2505_10171_amd import workloads as W
from parity_util import compare_fields, compare_history, compare_particles

pytestmark = pytest.mark.gpu

PILLARS = [(6, 6, 1, 9, 9, 5), (16, 6, 1, 19, 9, 5), (6, 16, 1, 9, 19, 5), (16, 16, 1, 19, 19, 5)]


def _gpu(cfg, phi0=None, parts=(), hist=0):
    from paper_2505_10171_amd.lbm import Simulation
    return Simulation(cfg, phi0, parts, history_steps=hist)


def _row(p, names):
    return np.concatenate([np.asarray(p[k], np.float64) for k in names])


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_drop_on_pillars_with_a_sphere(storage):
    """26 x 26 x 24, four pillars 4 x 4 x 5, wall angle 110 degrees, a drop of
    radius 8 sitting on the pillars and pushed along x, a free sphere of radius
    2.5 resting between two pillars, in front of the drop: 150 steps."""
    n = 26
    cfg = W.config(n, n, 24, has_wall=3, boxes=PILLARS, theta_wall_deg=110.0,
                   body_force=(4e-6, 0.0, 0.0), storage=storage)
    phi0 = W.drop_phi0(n, n, 24, (8.0, 12.5, 6.0), 8.0)
    R = 2.5
    p = W.particle((21.0, 12.6, 0.5 + R + cfg["delta_R"] + 0.02), R, theta_deg=70.0)
    steps = 150
    names = ("F_hyd", "T_hyd", "F_cap", "T_cap", "F_con", "T_con", "x", "v", "w")
    o = OracleSim(dict(cfg, storage="fp32"), phi0, [p])
    g = _gpu(cfg, phi0, [p], hist=steps)
    ho = []
    for _ in range(steps):
        o.step(1)
        ho.append(_row(o.particles()[0], names))
    g.step(steps)
    ho = np.array(ho)
    if storage == "fp32":
        compare_fields(g, o, label="drop on pillars, FP32")
        _, h = g.particles(history=True)
        compare_history(h[:, 0, :], ho, names, R, label="sphere between pillars")
    else:
        compare_fields(g, o, tol=1e-3, node_tol=None, label="drop on pillars, FP16")


@pytest.mark.parametrize("where", ["face", "edge", "corner"])
def test_held_sphere_against_a_box(where):
    """A sphere held (prescribed velocity zero) at overlap 0.2 with a box's side
    face, top edge or top corner: its contact force against the oracle's."""
    box = (10, 6, 1, 15, 13, 6)
    cfg = W.config(28, 20, 20, has_wall=3, boxes=[box])
    R, d0 = 3.0, 0.2
    Rc = R + cfg["delta_R"]
    q, n = {"face": ((9.5, 9.5, 5.0), (-1.0, 0.0, 0.0)),
            "edge": ((9.5, 9.5, 6.5), (-1.0, 0.0, 1.0)),
            "corner": ((9.5, 5.5, 6.5), (-1.0, -1.0, 1.0))}[where]
    n = np.array(n) / np.linalg.norm(n)
    x0 = np.array(q) + n * (Rc - d0)
    parts = [W.particle(tuple(x0), R, g_p=0.0, kinematic=1)]
    o = OracleSim(cfg, None, parts)
    g = _gpu(cfg, None, parts)
    o.step(2)
    g.step(2)
    fo, fg = np.array(o.particles()[0]["F_con"]), np.array(g.particles()[0]["F_con"])
    assert np.abs(fo - cfg["kn"] * d0 * n).max() <= 1e-12
    assert np.abs(fg - fo).max() <= 1e-9 * np.abs(fo).max()
    assert np.array_equal(g.fields()[3], o.fields()[3])  # masks (fluid at rest)


@pytest.mark.parametrize("n_side", [5, 8])
def test_packed_spheres_on_pillars(n_side):
    """A layer of n_side^2 spheres (R = 2, contact radius 3) packed closer than
    their contact diameter over a wall with four pillars of height 2, jittered
    and moving: 25 spheres run the DEM in LDS, 64 spread it over the GPU (a
    lane per candidate, one per wall face and one per pillar)."""
    g0 = W.rng(78, n_side)
    L = 6 * n_side - 2
    q = L // 4
    boxes = [(q - 2, q - 2, 1, q + 1, q + 1, 2), (3 * q - 2, q - 2, 1, 3 * q + 1, q + 1, 2),
             (q - 2, 3 * q - 2, 1, q + 1, 3 * q + 1, 2), (3 * q - 2, 3 * q - 2, 1, 3 * q + 1, 3 * q + 1, 2)]
    cfg = W.config(L, L, 18, has_wall=3, boxes=boxes, theta_wall_deg=90.0)
    phi0 = W.slab_phi0(L, L, 18, 10.0)
    R = 2.0
    Rc = R + cfg["delta_R"]
    sp = L / n_side
    parts = []
    for a in range(n_side):
        for b in range(n_side):
            x = ((a + 0.5) * sp + g0.uniform(-0.1, 0.1), (b + 0.5) * sp + g0.uniform(-0.1, 0.1),
                 2.5 + Rc - 0.1 + g0.uniform(-0.05, 0.05))
            parts.append(W.particle(x, R, theta_deg=90.0, mu_s=0.5, mu_r=0.05, sigma=cfg["sigma"],
                                    v=tuple(g0.uniform(-0.01, 0.01, 3)),
                                    w=tuple(g0.uniform(-0.005, 0.005, 3))))
    g = _gpu(cfg, phi0, parts)
    o = OracleSim(cfg, phi0, parts)
    g.step(3)
    o.step(3)
    compare_fields(g, o, label=f"{n_side}^2 packed spheres on pillars, 3 steps")
    pg, po = g.particles(), o.particles()
    assert np.abs(np.array([p["F_con"] for p in po])).max() > 0.1
    compare_particles(pg, po, ("F_con", "T_con", "x", "v", "w"),
                      label=f"{n_side}^2 packed spheres on pillars", R=R)


def test_mixed_geometry_ensemble():
    """One context holding a drop and sphere on the plane, a plug in a tube, a
    channel with open ends and a drop on pillars (the general instances of the
    interface and fused kernels run for all of them): 60 steps, each member
    against the oracle."""
    from paper_2505_10171_amd.lbm import Context
    import torch
    x = np.arange(40, dtype=np.float64)
    plug = np.broadcast_to(np.tanh(np.minimum(x - 10, 30 - x) / 2.0), (15, 15, 40))
    members = [
        dict(cfg=W.config(24, 20, 16, theta_wall_deg=80.0, body_force=(3e-6, 0.0, 0.0)),
             phi0=W.drop_phi0(24, 20, 16, (10.0, 10.0, 0.5), 7.0),
             particles=[W.particle((17.3, 9.8, 4.5), 3.0, theta_deg=70.0, kinematic=1,
                                   v=(0.002, 0.0, 0.0))]),
        dict(cfg=W.config(40, 15, 15, has_wall=2, tube_R=6.0, sigma=0.01, theta_wall_deg=60.0),
             phi0=plug.astype(np.float32).copy(), particles=[]),
        dict(cfg=W.config(32, 4, 17, has_wall=1, rho0=1.0, sigma=0.0, open_x=1, rho_in=1.0025,
                          rho_out=0.9975), phi0=None, particles=[]),
        dict(cfg=W.config(26, 26, 24, has_wall=3, boxes=PILLARS, theta_wall_deg=110.0,
                          body_force=(4e-6, 0.0, 0.0)),
             phi0=W.drop_phi0(26, 26, 24, (8.0, 12.5, 6.0), 8.0), particles=[]),
    ]
    ens = Context(members, stream=torch.cuda.Stream())
    ens.step(60)
    ens.sync()
    for i, m in enumerate(members):
        o = OracleSim(m["cfg"], m["phi0"], m["particles"])
        o.step(60)
        compare_fields(_Member(ens, i), o, label=f"mixed ensemble member {i}",
                       open_x=bool(m["cfg"].get("open_x", 0)))


class _Member:
    """One simulation of a context, seen as a single simulation."""

    def __init__(self, ctx, i):
        self.ctx, self.i = ctx, i

    def fields(self):
        return self.ctx.fields(self.i)
