"""Seeded synthetic inputs for the drop-particle workloads.

This module only builds inputs: configuration dictionaries (lattice units), the
initial order parameter phi0 and the particle records.  It holds none of the
method's arithmetic; both the GPU library and the CPU oracle receive exactly the
arrays made here.  Every random draw comes from
``numpy.random.Generator(PCG64([seed, index]))``.

Defaults follow the paper's parameter table (Table 1: rho_f = 0.05, beta = 0.7,
k_n = 2.5, k_t = 1.0, k_r = 0.5, particle density 0.125, damping zero in the
systematic runs, delta R = 1, capillary k = 0.134 on a 2-degree grid).  The
surface tension 0.01 is the lower end of the table's range; the downward force
on a particle is 5.23 sigma R_p, which keeps mu g_p / (sigma R_p) <= 5.2.
"""
from __future__ import annotations

import numpy as np

DEFAULTS = dict(
    rho0=0.05, tau_a=1.0, tau_b=1.0, sigma=0.01, beta=0.7, theta_wall_deg=90.0,
    body_force=(0.0, 0.0, 0.0), kn=2.5, kt=1.0, kr=0.5, gn=0.0, gt=0.0, gr=0.0,
    delta_R=1.0, cap_k=0.134, cap_dang_deg=2.0, has_wall=1, storage="fp32",
)


def rng(seed: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(index)]))


def config(nx: int, ny: int, nz: int, **kw) -> dict:
    c = dict(DEFAULTS)
    c.update(nx=int(nx), ny=int(ny), nz=int(nz))
    c.update(kw)
    c["body_force"] = tuple(float(v) for v in c["body_force"])
    return c


def particle(x, R, theta_deg=90.0, mu_s=0.5, mu_r=0.05, rho_p=0.125, g_p=None, sigma=0.01,
             v=(0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0), kinematic=0) -> dict:
    return dict(x=tuple(float(a) for a in x), v=tuple(float(a) for a in v),
                w=tuple(float(a) for a in w), q=(1.0, 0.0, 0.0, 0.0), R=float(R),
                rho_p=float(rho_p), theta_deg=float(theta_deg), mu_s=float(mu_s),
                mu_r=float(mu_r), g_p=float(5.23 * sigma * R if g_p is None else g_p),
                kinematic=int(kinematic))


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def _wrap(d, L):
    return d - L * np.round(d / L)


def drop_phi0(nx, ny, nz, centre, radius, width=2.0, periodic=True) -> np.ndarray:
    """phi0 = tanh((R - r) / width), shape (nz, ny, nx), float32; +1 inside the drop."""
    x, y, z = _grid(nx, ny, nz)
    dx, dy, dz = x - centre[0], y - centre[1], z - centre[2]
    if periodic:
        dx, dy = _wrap(dx, nx), _wrap(dy, ny)
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    return np.tanh((radius - r) / width).astype(np.float32)


def slab_phi0(nx, ny, nz, z_int, width=2.0) -> np.ndarray:
    """phi0 = tanh((z_int - z) / width): liquid (fluid a) below z_int."""
    x, y, z = _grid(nx, ny, nz)
    return np.tanh((z_int - z) / width).astype(np.float32)


def _place(g, n, lo, hi, spacing, L, tries=200000):
    """n points uniform in the box [lo, hi] with min-image spacing >= spacing."""
    pts = []
    for _ in range(tries):
        if len(pts) == n:
            break
        p = g.uniform(lo, hi)
        ok = True
        for q in pts:
            d = _wrap(np.asarray(p) - np.asarray(q), np.asarray(L, dtype=float))
            if np.dot(d, d) < spacing * spacing:
                ok = False
                break
        if ok:
            pts.append(p)
    if len(pts) < n:
        raise RuntimeError("could not place the particles")
    return pts


def sessile_drop_c1(seed: int = 1):
    """32^3, hemisphere R_d = 10 on a 90-degree wall, one R_p = 4 sphere with a
    60-degree contact angle at the drop edge with +-0.5 lu jitter; 200 steps."""
    g = rng(seed, 0)
    cfg = config(32, 32, 32, theta_wall_deg=90.0)
    phi0 = drop_phi0(32, 32, 32, (16.0, 16.0, 0.5), 10.0)
    R = 4.0
    x = (26.0 + g.uniform(-0.5, 0.5), 16.0 + g.uniform(-0.5, 0.5), 0.5 + R + cfg["delta_R"])
    parts = [particle(x, R, theta_deg=60.0, mu_s=0.5, mu_r=0.05, sigma=cfg["sigma"])]
    return dict(name="sessile drop 32^3, 1 sphere R=4", cfg=cfg, phi0=phi0, particles=parts,
                steps=200)


def drop_sweep_c2(seed: int = 2):
    """256x128x96, 110-degree wall, hemisphere R_d = 30 pushed along x by a body
    force 5e-6, 20 spheres R_p = 5 resting on the dry wall at seeded uniform
    positions outside the drop footprint (as the paper starts its particles in
    front of the drop), downward force 10 sigma R_p; 10,000 steps."""
    g = rng(seed, 0)
    nx, ny, nz = 256, 128, 96
    Rd, xc = 30.0, (64.0, 64.0)
    cfg = config(nx, ny, nz, theta_wall_deg=110.0, body_force=(5e-6, 0.0, 0.0))
    phi0 = drop_phi0(nx, ny, nz, (xc[0], xc[1], 0.5), Rd)
    R, Rc = 5.0, 5.0 + cfg["delta_R"]
    parts, pts = [], []
    while len(pts) < 20:
        q = _place(g, 1, [0.0, 0.0], [nx, ny], 0.0, [nx, ny])[0]
        d = _wrap(np.asarray(q) - np.asarray(xc), np.asarray([nx, ny], float))
        if np.hypot(*d) < Rd + Rc + 4.0:
            continue
        if any(np.hypot(*_wrap(np.asarray(q) - np.asarray(o), np.asarray([nx, ny], float)))
               < 2 * Rc + 1 for o in pts):
            continue
        pts.append(q)
    for p in pts:
        parts.append(particle((p[0] % nx, p[1] % ny, 0.5 + Rc), R,
                              theta_deg=g.uniform(30.0, 120.0), mu_s=g.uniform(0.0, 1.0),
                              mu_r=g.uniform(0.0, 0.1), g_p=10.0 * cfg["sigma"] * R,
                              sigma=cfg["sigma"]))
    return dict(name="drop sweeping particles 256x128x96, 20 spheres R=5", cfg=cfg, phi0=phi0,
                particles=parts, steps=10000)


def slab_c3(seed: int = 3, storage: str = "fp32"):
    """512x256x192, liquid slab filling 40% of the height, 500 spheres R_p = 4
    at non-overlapping random positions; 500 steps."""
    g = rng(seed, 0)
    nx, ny, nz = 512, 256, 192
    cfg = config(nx, ny, nz, theta_wall_deg=90.0, storage=storage)
    phi0 = slab_phi0(nx, ny, nz, 0.4 * nz)
    R, Rc = 4.0, 4.0 + cfg["delta_R"]
    pts = _place(g, 500, [0.0, 0.0, 0.5 + Rc], [nx, ny, nz - 0.5 - Rc], 2 * Rc + 1,
                 [nx, ny, 1e9])
    parts = [particle((p[0] % nx, p[1] % ny, p[2]), R, theta_deg=90.0, mu_s=0.5, mu_r=0.05,
                      sigma=cfg["sigma"]) for p in pts]
    return dict(name="liquid slab 512x256x192, 500 spheres R=4", cfg=cfg, phi0=phi0,
                particles=parts, steps=500)


def ensemble_member_c4(seed: int, index: int, storage: str = "fp32"):
    """One member of the batched ensemble: cubic box of side L in {48,64,80,96},
    drop radius 12-24, body force 1e-6..1e-5, one sphere of radius 3-6 in front
    of the drop; 5,000 steps."""
    g = rng(seed, index)
    L = int(g.choice([48, 64, 80, 96]))
    cfg = config(L, L, L, theta_wall_deg=90.0, storage=storage)
    Rp = g.uniform(3.0, 6.0)
    Rc = Rp + cfg["delta_R"]
    Rd = g.uniform(12.0, min(24.0, (L - 2 * Rc - 8) / 2.0))
    fx = g.uniform(1e-6, 1e-5)
    cfg["body_force"] = (fx, 0.0, 0.0)
    mu_s, mu_r, th = g.uniform(0.0, 1.0), g.uniform(0.0, 0.1), g.uniform(30.0, 150.0)
    xc = L / 4.0
    phi0 = drop_phi0(L, L, L, (xc, L / 2.0, 0.5), Rd)
    px = (xc + Rd + Rc + 2.0, L / 2.0 + g.uniform(-0.5, 0.5), 0.5 + Rc)
    parts = [particle(px, Rp, theta_deg=th, mu_s=mu_s, mu_r=mu_r, sigma=cfg["sigma"])]
    return dict(name=f"ensemble member {index}: L={L}", cfg=cfg, phi0=phi0, particles=parts,
                steps=5000, params=dict(mu_s=mu_s, mu_r=mu_r, R_d=Rd, f_x=fx, theta_p=th, R_p=Rp))


# Relaxation times of the paper's drop-particle runs (Table 1): rho_f = 0.05,
# eta = 0.0273 for the drop and 0.00273 for the air, tau = 1/2 + 3 eta / rho_f.
# Fluid a (phi = +1) is the drop here, fluid b the air.
TAU_DROP = 0.5 + 3.0 * 0.0273 / 0.05   # 2.138
TAU_AIR = 0.5 + 3.0 * 0.00273 / 0.05   # 0.6638


def table1_n1(seed: int = 5, R_p: float = 10.0, drop_ratio: float = 5.0, bond: float = 1.25,
              theta_p: float = 92.0, theta_s: float = 100.0, mu_s: float = 0.5,
              mu_r: float = 0.05, sigma: float = 0.01, nx: int = 400, ny: int = 181,
              nz: int = 71, storage: str = "fp32"):
    """The paper's drop-particle workload (section "Simulation setup and
    parameters", Table 1): 400x181x71 lattice, particle radius 10, drop radius
    5 R_p as a hemisphere on the wall, viscosity ratio 10 (drop tau 2.138, air
    0.664), particle contact angle 90-95 degrees, wall 90-110 degrees, body
    force on the drop from the Bond number Bo = f R_d^2 / sigma, downward force
    5.23 sigma R_p on the particle; the particle rests on the wall in front of
    the drop, offset in y by a seeded jitter of +-0.5."""
    g = rng(seed, 0)
    R_d = drop_ratio * R_p
    f_x = bond * sigma / (R_d * R_d)
    cfg = config(nx, ny, nz, tau_a=TAU_DROP, tau_b=TAU_AIR, sigma=sigma,
                 theta_wall_deg=theta_s, body_force=(f_x, 0.0, 0.0), storage=storage)
    xd, yd = 0.25 * nx, 0.5 * (ny - 1)
    phi0 = drop_phi0(nx, ny, nz, (xd, yd, 0.5), R_d)
    Rc = R_p + cfg["delta_R"]
    x = (xd + R_d + Rc + 2.0, yd + g.uniform(-0.5, 0.5), 0.5 + Rc)
    parts = [particle(x, R_p, theta_deg=theta_p, mu_s=mu_s, mu_r=mu_r, sigma=sigma)]
    return dict(name=f"drop-particle (Table 1) {nx}x{ny}x{nz}, R_p={R_p:g}, R_d={R_d:g}",
                cfg=cfg, phi0=phi0, particles=parts, steps=20000,
                params=dict(Bo=bond, f_x=f_x, R_d=R_d))


def table1_reduced(seed: int = 6, storage: str = "fp32"):
    """The Table 1 fluids and angles on a 64x48x32 box with R_p = 6 and a drop
    of radius 2 R_p whose contact line touches the particle: a parity case at
    viscosity ratio 10 that the oracle finishes in seconds."""
    w = table1_n1(seed=seed, R_p=6.0, drop_ratio=2.0, nx=64, ny=48, nz=32, storage=storage)
    # the particle starts at the drop's contact line, so that the interface
    # meets it within the compared steps
    p = w["particles"][0]
    xd = 0.25 * 64
    p["x"] = (xd + 12.0 + 4.0, p["x"][1], p["x"][2])
    w["steps"] = 100
    return w


def drop_meets_sphere(seed: int = 7, storage: str = "fp32"):
    """The drop-sweeping workload reduced to 96x64x40: a 110-degree wall, a drop
    of radius 15 pushed along x by 5e-6, and one free sphere of radius 5 (contact
    angle 60 degrees, mu_s 0.4, mu_r 0.04) placed where the drop's advancing
    contact line reaches it within the first steps."""
    g = rng(seed, 0)
    nx, ny, nz = 96, 64, 40
    cfg = config(nx, ny, nz, theta_wall_deg=110.0, body_force=(5e-6, 0.0, 0.0), storage=storage)
    R_d, xd, yd = 15.0, 30.0, 32.0
    phi0 = drop_phi0(nx, ny, nz, (xd, yd, 0.5), R_d)
    R, Rc = 5.0, 5.0 + cfg["delta_R"]
    x = (xd + R_d + 2.0, yd + g.uniform(-1.0, 1.0), 0.5 + Rc)
    parts = [particle(x, R, theta_deg=60.0, mu_s=0.4, mu_r=0.04, g_p=10.0 * cfg["sigma"] * R,
                      sigma=cfg["sigma"])]
    return dict(name="drop meets sphere 96x64x40", cfg=cfg, phi0=phi0, particles=parts, steps=200)


def tube_segre(seed: int = 8, R_t: float = 40.0, R_p: float = 12.2, length: float = 8.0,
               l_frac: float = 0.21, rho_f: float = 1.05, nu: float = 0.457,
               v_in: float = 0.0113, storage: str = "fp32"):
    """The hydrodynamic-force benchmark (section "Benchmarking hydrodynamic
    force"): a neutrally buoyant sphere of radius R_p = 12.2 in pressure-driven
    Poiseuille flow through a tube of radius R_t = 40, fluid density 1.05,
    kinematic viscosity 0.457 (tau = 1.871), mean velocity 0.0113 set by the
    Hagen-Poiseuille pressure drop 8 rho nu v_in L / R_t^2 between the open
    ends; the sphere starts 0.21 R_t off the axis, two tube radii behind the
    inlet plane's clearance.  The tube length, which the paper does not give,
    is `length` radii.  The off-axis direction is drawn from the seed."""
    g = rng(seed, 0)
    ny = nz = int(2 * R_t) + 3
    nx = int(length * R_t)
    tau = 0.5 + 3.0 * nu
    dp = 8.0 * rho_f * nu * v_in * nx / (R_t * R_t)
    drho = 3.0 * dp
    cfg = config(nx, ny, nz, has_wall=2, tube_R=R_t, open_x=1, rho0=rho_f,
                 rho_in=rho_f + 0.5 * drho, rho_out=rho_f - 0.5 * drho, tau_a=tau, tau_b=tau,
                 sigma=0.0, storage=storage)
    a = g.uniform(0.0, 2.0 * np.pi)
    l = l_frac * R_t
    x = (2.0 * R_t, 0.5 * (ny - 1) + l * np.cos(a), 0.5 * (nz - 1) + l * np.sin(a))
    parts = [particle(x, R_p, rho_p=rho_f, g_p=0.0, mu_s=0.0, mu_r=0.0)]
    return dict(name=f"sphere in tube flow {nx}x{ny}x{nz}, R_t={R_t:g}, R_p={R_p:g}",
                cfg=cfg, phi0=None, particles=parts, steps=20000,
                params=dict(drho=drho, v_in=v_in, l0=l))


def tube_reduced(seed: int = 9, storage: str = "fp32"):
    """tube_segre scaled to R_t = 8, R_p = 3 on a 48-node tube (the same
    viscosity, mean velocity 0.005 so that the pressure drop stays a few per
    cent of the density): a parity case the oracle finishes in seconds."""
    w = tube_segre(seed=seed, R_t=8.0, R_p=3.0, length=6.0, v_in=0.005, storage=storage)
    p = w["particles"][0]
    p["x"] = (16.0, p["x"][1], p["x"][2])
    w["steps"] = 200
    return w


def textured_wall(seed: int = 10, storage: str = "fp32"):
    """A textured wall (the future work of the paper's conclusions): a
    256x128x64 box whose floor carries eight square pillars (12 x 12 nodes, 8
    high, in a 4 x 2 array), a drop of radius 24 resting on the pillar tops and
    pushed along x by 4e-6 (wall 110 degrees), and six spheres of radius 4 on
    the floor between the pillars at seeded positions (contact angle 60-120
    degrees)."""
    g = rng(seed, 0)
    nx, ny, nz = 256, 128, 64
    boxes = [(cx - 6, cy - 6, 1, cx + 5, cy + 5, 8) for cx in (48, 96, 144, 192) for cy in (40, 88)]
    cfg = config(nx, ny, nz, has_wall=3, boxes=boxes, theta_wall_deg=110.0,
                 body_force=(4e-6, 0.0, 0.0), storage=storage)
    phi0 = drop_phi0(nx, ny, nz, (72.0, 64.0, 8.5), 24.0)
    R = 4.0
    Rc = R + cfg["delta_R"]
    parts = []
    tries = 0
    while len(parts) < 6 and tries < 100000:
        tries += 1
        x = (g.uniform(110.0, 250.0), g.uniform(Rc, ny - Rc), 0.5 + Rc)
        clear = all(max(b[0] - 0.5 - x[0], x[0] - b[3] - 0.5, b[1] - 0.5 - x[1], x[1] - b[4] - 0.5)
                    > Rc + 1.0 for b in boxes)
        apart = all(np.hypot(x[0] - q["x"][0], x[1] - q["x"][1]) > 2 * Rc + 1.0 for q in parts)
        if clear and apart:
            parts.append(particle(x, R, theta_deg=g.uniform(60.0, 120.0), sigma=cfg["sigma"]))
    return dict(name=f"textured wall {nx}x{ny}x{nz}, 8 pillars, drop R=24, 6 spheres",
                cfg=cfg, phi0=phi0, particles=parts, steps=5000)
