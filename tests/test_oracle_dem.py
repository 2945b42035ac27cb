"""Pins of the oracle's DEM against the paper's contact benchmarks (no fluid).

T14 a sphere bouncing on the wall: with no damping the apex height stays h0
    (energy conservation); with normal damping the n-th apex is r^(2n) h0 with
    restitution r = exp(-eta_n t_c), eta_n = gamma_n/(2m), t_c = pi/omega_c,
    omega_c = sqrt(k_n/m - eta_n^2) (restitution and rebound-height eqs.);
T15 a sphere on a 45-degree incline (gravity tilted instead of the wall):
    without friction it slides with a = g sin 45 and never turns; with sliding
    friction it rolls, a -> 5/7 g sin 45, slip ratio omega R / v - 1 ~ 0, and its
    rotation angle matches the distance travelled (cycloid marker); rolling
    friction lowers the acceleration.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSim
from paper_2505_10171_amd import workloads as W


def _mass(R, rho_p=0.125):
    return rho_p * 4.0 / 3.0 * np.pi * R ** 3


def _bounce(gn, steps, h0=10.0, g=2e-4, R=4.0):
    cfg = W.config(8, 8, 48, gn=gn)
    m = _mass(R)
    Rc = R + cfg["delta_R"]
    z0 = 0.5 + Rc + h0
    s = OracleSim(cfg, None, [W.particle((4.0, 4.0, z0), R, g_p=m * g)])
    z = [z0]
    for _ in range(steps):
        s.dem_run(1)
        z.append(s.particles()[0]["x"][2])
    h = np.array(z) - 0.5 - Rc
    apex = [h[k] for k in range(1, len(h) - 1) if h[k] >= h[k - 1] and h[k] > h[k + 1] and h[k] > 0.5]
    return cfg, m, np.array(apex)


def test_T14_elastic_bounce_keeps_height():
    cfg, m, apex = _bounce(0.0, 2600)
    assert len(apex) >= 3
    # velocity Verlet on the switched-on spring keeps the energy to the order
    # (omega_c dt_s)^2 ~ (pi/45)^2 of one contact
    assert np.abs(apex / 10.0 - 1).max() < 0.5 * (np.pi / 45) ** 2


def test_T14_damped_rebound_heights():
    # the restitution law is that of a free collision; a weak gravity keeps its
    # effect during the ~t_c contact negligible (overlap m g / k_n << v0 / omega_c)
    gn = 1.0
    cfg, m, apex = _bounce(gn, 10400, g=1.25e-5)
    eta = gn / (2 * m)
    tc = np.pi / np.sqrt(cfg["kn"] / m - eta ** 2)
    r = np.exp(-eta * tc)
    assert len(apex) >= 3
    for n, hn in enumerate(apex[:4], start=1):
        assert abs(hn / (r ** (2 * n) * 10.0) - 1) < 0.005, (n, hn)


def _incline(mu, mur, steps=1500, g=1e-3, R=4.0):
    cfg = W.config(8, 8, 32, delta_R=0.0)
    m = _mass(R)
    s45 = np.sin(np.pi / 4)
    Fext = np.array([m * g * s45, 0.0, -m * g * s45])
    dz = m * g * s45 / cfg["kn"]          # static overlap, so the sphere starts at rest in z
    s = OracleSim(cfg, None, [W.particle((4.0, 4.0, 0.5 + R - dz), R, mu_s=mu, mu_r=mur, g_p=0.0)])
    V, Wy, Q = [], [], []
    for _ in range(steps):
        s.dem_run(1, Fext)
        p = s.particles()[0]
        V.append(p["v"][0])
        Wy.append(p["w"][1])
        Q.append(p["q"])
    return g * s45, np.array(V), np.array(Wy), np.array(Q), R


def test_T15_frictionless_slide():
    a, V, Wy, Q, R = _incline(0.0, 0.0, steps=400)
    t = np.arange(1, len(V) + 1)
    assert np.allclose(V, a * t, rtol=1e-12, atol=0)
    assert np.abs(Wy).max() == 0.0


def test_T15_rolling_with_friction():
    a, V, Wy, Q, R = _incline(0.5, 0.0)
    k0, k1 = 1000, 1499
    acc = (V[k1] - V[k0]) / (k1 - k0)
    assert abs(acc / (5.0 / 7.0 * a) - 1) < 0.01
    slip = Wy[k1] * R / V[k1] - 1
    assert abs(slip) < 0.01
    # rotation angle about +y (from the orientation quaternion) vs distance:
    # the contact marker traces a cycloid when x = R alpha
    alpha = np.unwrap(2 * np.arctan2(Q[:, 2], Q[:, 0]))
    dist = np.cumsum(V)
    assert abs(R * alpha[-1] / dist[-1] - 1) < 0.02


def test_T15_rolling_resistance_slows():
    a, V0, _, _, _ = _incline(0.5, 0.0)
    a, V1, _, _, _ = _incline(0.5, 0.05)
    assert V1[-1] < V0[-1]


def test_table1_time_step_rule():
    """Table 1 values (R_p = 10, particle density 0.125, k_n = 2.5) give the
    paper's DEM step dt ~ t_c/45 with one sub-step per lattice step; smaller
    particles get proportionally more sub-steps."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_parameters.json")))
    cfg = W.config(24, 24, 24, kn=g["k_n"], kt=g["k_t"], kr=g["k_r"])
    s = OracleSim(cfg, None, [W.particle((12.0, 12.0, 12.0), g["R_p"], rho_p=g["rho_p"])])
    assert s.n_sub == 1
    m = _mass(g["R_p"], g["rho_p"])
    tc = np.pi / np.sqrt(g["k_n"] / m)
    assert abs(1.0 / tc - g["dt_over_tc"]) < 0.001
    s4 = OracleSim(cfg, None, [W.particle((12.0, 12.0, 12.0), 4.0, rho_p=g["rho_p"])])
    assert s4.n_sub == 4
    # the table's viscosities at rho_f = 0.05 are the relaxation times 0.664 / 2.138
    from oracle import oracle as O
    for eta, tau in ((g["eta_a"], 0.664), (g["eta_b"], 2.138)):
        c = W.config(4, 4, 4, tau_a=tau, tau_b=tau)
        assert abs(1.0 / O.omega(c, 1.0) - (0.5 + 3 * eta / g["rho_f"])) < 1e-3
