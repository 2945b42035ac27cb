"""The paper's capillary-force benchmark (section "Benchmarking capillary
force") run by the FP64 oracle.  TEST INFRASTRUCTURE ONLY: nothing in the
product library imports it.

A sphere of radius R_p with contact angle theta (measured through fluid a) sits
at a flat interface between a layer of fluid a on the wall (below) and fluid b
(above), at the height where the flat interface meets it at theta:
z_p = z_int - R_p cos(theta).  After the colour profile has relaxed, the sphere
is pulled upward at the constant velocity v_p (a prescribed-velocity particle)
and the vertical capillary force is recorded every step.  Its largest downward
magnitude is the detachment force, which the paper compares with Scheludko's
closed form F_max = 2 pi sigma R_p cos^2(theta/2) (detachment-force eq.): the
vertical surface-tension force of a contact line held at angle theta on the
sphere, maximised over the contact line's position.  The paper states errors up
to 30 % for R_p = 10 at theta = 30 degrees, within 5 % at R_p = 25.

The fluid-a layer rests on the wall (node plane z = 0), so that pulling the
sphere stretches a meniscus instead of lifting a free-floating layer; the box is
periodic in x and y.
"""
import numpy as np


def scheludko(sigma, R, theta_deg):
    """Detachment force of a sphere held at contact angle theta (detachment-force eq.)."""
    return 2.0 * np.pi * sigma * R * np.cos(np.radians(theta_deg) / 2.0) ** 2


def setup(theta_deg, R=10.0, nxy=32, nz=52, z_int=22.5, sigma=0.01):
    """(cfg, phi0, particle) of the benchmark box: fluid a below z_int on the
    wall, the sphere centred in x, y at its flat-interface equilibrium height."""
    from paper_2505_10171_amd import workloads as W
    cfg = W.config(nxy, nxy, nz, has_wall=1, sigma=sigma, theta_wall_deg=90.0)
    z = np.arange(nz, dtype=np.float64)
    phi0 = np.broadcast_to(np.tanh((z_int - z) / 2.0)[:, None, None],
                           (nz, nxy, nxy)).astype(np.float32).copy()
    zc = z_int - R * np.cos(np.radians(theta_deg))
    p = W.particle((nxy / 2.0, nxy / 2.0, zc), R, theta_deg=theta_deg, kinematic=1)
    return cfg, phi0, p


def run(theta_deg, R=10.0, v=0.01, relax=100, min_pull=250, max_pull=2600, stop_frac=0.6, threads=0,
        **box):
    """Relax `relax` steps at rest, then pull at v along +z until, after at
    least min_pull steps, the downward capillary force has fallen below
    stop_frac of its largest value (or max_pull steps).  Returns a dict with the per-step history of the pull
    (rise of the centre, F_cap, T_cap) and F_max."""
    from oracle import oracle as O
    from oracle.oracle import OracleSim
    if threads:
        O.set_num_threads(threads)
    cfg, phi0, p = setup(theta_deg, R=R, **box)
    sim = OracleSim(cfg, phi0, [p])
    sim.step(relax)
    sim.set_particles([dict(p, v=(0.0, 0.0, v))])
    z0 = p["x"][2]
    rise, Fc, Tc = [], [], []
    best = 0.0
    for _ in range(max_pull):
        sim.step(1)
        q = sim.particles()[0]
        rise.append(q["x"][2] - z0)
        Fc.append(q["F_cap"])
        Tc.append(q["T_cap"])
        best = max(best, -q["F_cap"][2])
        if len(rise) >= min_pull and -q["F_cap"][2] < stop_frac * best:
            break
    sim.close()
    Fc = np.array(Fc)
    return dict(theta=theta_deg, R=R, sigma=cfg["sigma"], rise=np.array(rise), F_cap=Fc,
                T_cap=np.array(Tc), F_max=float(-Fc[:, 2].min()),
                rise_at_max=float(rise[int(np.argmin(Fc[:, 2]))]))
