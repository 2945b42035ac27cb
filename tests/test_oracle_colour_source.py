"""T18: the colour populations after a step are a function of the total
populations and of per-node quantities of the state that collided.

The recolouring (recolouring eqs.) gives the population leaving x' in
direction i the colour difference f^a_i - f^b_i = phi' f*_i + r' w_i (c_i . n'),
r' = beta rho' (1 - phi'^2) / 2.  After streaming, f_i(x) came from
x' = x - c_i, or, when x - c_i was solid, is f*_opp(i)(x) bounced back, whose
colour difference is phi(x) f_i(x) - r(x) w_i (c_i . n(x)) (the moving-wall
term of the bounce-back eqs. splits between the fluids as rho_a : rho_b).
The GPU path stores only f and rebuilds the colour this way; this test checks
the identity on the oracle's own step, at fluid and wall links, at the links
of a moving, spinning particle and across a wetting interface.
"""
import numpy as np

from oracle import oracle as O
from oracle.oracle import OracleSim
from paper_2505_10171_amd import workloads as W


def test_T18_colour_rebuilt_from_sources():
    nx, ny, nz = 20, 18, 16
    cfg = W.config(nx, ny, nz, sigma=0.01, theta_wall_deg=70.0, body_force=(3e-6, 0, 0),
                   tau_a=0.8, tau_b=1.3)
    phi0 = W.drop_phi0(nx, ny, nz, (9.0, 9.0, 1.0), 6.5)
    parts = [W.particle((13.2, 9.6, 5.4), 3.0, theta_deg=60.0, v=(0.01, -0.004, 0.002),
                        w=(0.0, 0.003, 0.002), kinematic=1)]
    s = OracleSim(cfg, phi0, parts)
    s.step(20)
    c, w, _ = O.lattice()
    beta = cfg["beta"]
    # the state about to collide
    rho, _, phi, mask0 = s.fields()
    G = s.grad_force()[0]
    g = np.sqrt((G ** 2).sum(axis=-1))
    n = G / np.maximum(g, 1e-4)[..., None]          # interface normal after wetting
    r = 0.5 * beta * rho * (1.0 - phi ** 2)
    s.step(1)
    fa, fb = s.pops()
    mask1 = s.fields()[3]
    s.close()
    shp = (nz, ny, nx, 19)
    f = (fa + fb).reshape(shp)
    gcol = (fa - fb).reshape(shp)
    keep = (mask0 == 0) & (mask1 == 0)   # fluid before and after (no refill)
    assert keep.sum() > 0.8 * keep.size
    n_bounced = 0
    err = 0.0
    for i in range(1, 19):
        sh = (c[i, 2], c[i, 1], c[i, 0])
        src = lambda a: np.roll(a, shift=sh, axis=(0, 1, 2))     # value at x - c_i
        solid = src(mask0) != 0
        cn_src = (src(n) @ c[i]).astype(float)
        cn_own = (n @ c[i]).astype(float)
        expect = np.where(solid, phi * f[..., i] - r * w[i] * cn_own,
                          src(phi) * f[..., i] + src(r) * w[i] * cn_src)
        d = np.abs(expect - gcol[..., i])[keep]
        err = max(err, d.max())
        n_bounced += int((solid & keep).sum())
    assert n_bounced > 100          # wall and particle links were exercised
    assert err <= 1e-12 * np.abs(f[keep]).max(), err
    # rest population: colour phi(x) f_0
    d0 = np.abs(phi * f[..., 0] - gcol[..., 0])[keep].max()
    assert d0 <= 1e-12 * np.abs(f[keep]).max(), d0
