"""Pins of the oracle's textured wall: the plane z = 0 with boxes of solid nodes
(the paper names textured walls as future work; the surface of a box is the
box of its nodes grown by half a node, as half-way bounce-back places it).

X1  a box covering the whole x-y plane at heights 1..h is the plane wall raised
    by h: a drop and a resting sphere on it give the plane run's fields, forces
    and path, shifted (mask, bounce-back, the top face's wetting normal and its
    DEM contact surface);
X2  a sphere pressed against a box's side face, and against its top edge along
    the edge's diagonal, comes to rest at the overlap F / k_n along the force
    (the nearest-point contact of a face and of an edge);
X3  a drop centred over a square pillar keeps the mirror symmetries of the set-up
    (x -> -x and x <-> y about the pillar's axis): a wrong sign or axis in a side
    face's wetting normal breaks them.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSim
from paper_2505_10171_amd import workloads as W


def test_X1_full_width_box_is_a_raised_plane():
    nx, ny, nzp, h = 24, 20, 16, 3
    nz = nzp + h
    plane = W.config(nx, ny, nzp, has_wall=1, theta_wall_deg=70.0, body_force=(2e-6, 0, 0))
    boxed = W.config(nx, ny, nz, has_wall=3, theta_wall_deg=70.0, body_force=(2e-6, 0, 0),
                     boxes=[(0, 0, 1, nx - 1, ny - 1, h)])
    phi_p = W.drop_phi0(nx, ny, nzp, (10.0, 10.0, 0.5), 6.0)
    phi_b = np.full((nz, ny, nx), -1.0, np.float32)
    phi_b[h:] = phi_p
    R = 3.0
    Rc = R + plane["delta_R"]
    pp = W.particle((17.3, 9.6, 0.5 + Rc + 0.05), R, theta_deg=60.0)
    pb = dict(pp, x=(pp["x"][0], pp["x"][1], pp["x"][2] + h))
    a = OracleSim(plane, phi_p, [pp])
    b = OracleSim(boxed, phi_b, [pb])
    a.step(60)
    b.step(60)
    ra, ua, fa, ma = a.fields()
    rb, ub, fb, mb = b.fields()
    assert np.array_equal(mb[h:] != 0, ma != 0)
    assert np.all(mb[:h + 1] != 0)
    fl = ma == 0
    assert np.abs(rb[h:][fl] - ra[fl]).max() <= 1e-13
    assert np.abs(fb[h:][fl] - fa[fl]).max() <= 1e-11
    assert np.abs(ub[:, h:][:, fl] - ua[:, fl]).max() <= 1e-12
    qa, qb = a.particles()[0], b.particles()[0]
    assert abs(qb["x"][2] - h - qa["x"][2]) <= 1e-11
    for k in ("F_hyd", "F_cap", "F_con"):
        assert np.abs(np.array(qb[k]) - np.array(qa[k])).max() <= 1e-11 * max(1.0, np.abs(qa[k]).max())
    assert np.abs(qa["F_con"]).max() > 0  # the sphere rests on the surface


def test_X2_contact_with_a_box_face():
    """Pressed against a side face, the sphere comes to rest at F / k_n."""
    box = (10, 6, 1, 15, 13, 6)      # nodes; surface x in [9.5, 15.5], z up to 6.5
    cfg = W.config(28, 20, 20, has_wall=3, boxes=[box], gn=0.6)
    R, F = 3.0, 0.4
    Rc = R + cfg["delta_R"]
    n = np.array([-1.0, 0.0, 0.0])      # from the face x = 9.5 to the centre
    q = np.array([9.5, 9.5, 5.0])
    x0 = q + n * (Rc + 0.3)
    s = OracleSim(cfg, None, [W.particle(tuple(x0), R, g_p=0.0, mu_s=0.0, mu_r=0.0)])
    s.dem_run(4000, Fext=np.array([(-F * n)]))
    p = s.particles()[0]
    expect = q + n * (Rc - F / cfg["kn"])
    assert np.abs(np.array(p["x"]) - expect).max() <= 1e-8
    assert np.abs(np.array(p["F_con"]) - F * n).max() <= 1e-8


@pytest.mark.parametrize("case", ["edge", "corner"])
def test_X2_contact_with_a_box_edge_and_corner(case):
    """A sphere held at overlap 0.2 with a box's top edge or corner is pushed
    along the line from the nearest point of the box to its centre, with
    k_n times the overlap (a ridge is no resting place, so the sphere is held)."""
    box = (10, 6, 1, 15, 13, 6)
    cfg = W.config(28, 20, 20, has_wall=3, boxes=[box])
    R, d0 = 3.0, 0.2
    Rc = R + cfg["delta_R"]
    if case == "edge":
        q = np.array([9.5, 9.5, 6.5])
        n = np.array([-1.0, 0.0, 1.0]) / np.sqrt(2.0)
    else:
        q = np.array([9.5, 5.5, 6.5])
        n = np.array([-1.0, -1.0, 1.0]) / np.sqrt(3.0)
    x0 = q + n * (Rc - d0)
    s = OracleSim(cfg, None, [W.particle(tuple(x0), R, g_p=0.0, kinematic=1)])
    s.dem_run(2)
    p = s.particles()[0]
    assert np.abs(np.array(p["F_con"]) - cfg["kn"] * d0 * n).max() <= 1e-12


def test_X3_pillar_mirror_symmetry():
    L = 21
    c = (L - 1) / 2.0
    cfg = W.config(L, L, 18, has_wall=3, theta_wall_deg=60.0, boxes=[(8, 8, 1, 12, 12, 4)])
    phi0 = W.drop_phi0(L, L, 18, (c, c, 4.5), 6.0)
    s = OracleSim(cfg, phi0)
    s.step(80)
    rho, u, phi, mask = s.fields()
    assert np.abs(phi - phi[:, :, ::-1]).max() <= 1e-11
    assert np.abs(phi - phi.transpose(0, 2, 1)).max() <= 1e-11
    assert np.abs(u[0] + u[0][:, :, ::-1]).max() <= 1e-13
    assert np.abs(u[0] - u[1].transpose(0, 2, 1)).max() <= 1e-13
    assert np.abs(u).max() > 1e-5  # the drop moves over the pillar's edges
