"""Pin of the oracle's capillary force (capillary-force eq.) by the paper's
detachment benchmark (section "Benchmarking capillary force"): a sphere of
radius 10 pulled out of a fluid-a layer at v_p = 0.01.  Its largest downward
capillary force is compared with Scheludko's F_max = 2 pi sigma R cos^2(theta/2)
(detachment-force eq.).

The paper states errors up to 30 % at R_p = 10 for theta = 30 degrees.  That
band holds here for 30, 60, 90 and 120 degrees.  At 150 degrees the contact line
at the force maximum is a ring of radius R sin(15 deg) = 2.6 lattice units on the
sphere, narrower than the diffuse interface, and F_max is 7 % of the 30-degree
value; there the bound is on the error in units of 2 pi sigma R (the force scale
of the closed form), 5 %.  A wrong prefactor, area element, k, sin(theta) factor
or direction of m fails the band at one angle or more (e.g. without sin(theta)
the 30-degree ratio is about 1.9, with m reversed F_max has the wrong sign).
The torque about the centre must vanish for the axisymmetric pull: an arm taken
from any point other than the centre gives a torque |X x F| of the order R |F|.
"""
import multiprocessing as mp
import os

import numpy as np
import pytest

ANGLES = (30.0, 60.0, 90.0, 120.0, 150.0)


def _one(theta):
    from oracle import detachment as D
    threads = max(1, (os.cpu_count() or 5) // len(ANGLES))
    r = D.run(theta, threads=threads)
    return theta, r["F_max"], r["rise_at_max"], float(np.abs(r["T_cap"]).max()), \
        float(np.abs(r["F_cap"]).max()), len(r["rise"])


@pytest.fixture(scope="module")
def sweep():
    ctx = mp.get_context("spawn")
    with ctx.Pool(len(ANGLES)) as pool:
        out = pool.map(_one, ANGLES)
    return {t: dict(F_max=f, rise=z, T_max=tm, F_abs=fa, steps=n) for t, f, z, tm, fa, n in out}


@pytest.mark.slow
def test_detachment_force_against_closed_form(sweep):
    from oracle.detachment import scheludko
    sigma, R = 0.01, 10.0
    scale = 2 * np.pi * sigma * R
    for theta in ANGLES:
        r = sweep[theta]
        pred = scheludko(sigma, R, theta)
        ratio = r["F_max"] / pred
        print(f"theta {theta:5.1f}: F_max {r['F_max']:.4f} closed form {pred:.4f} ratio {ratio:.3f} "
              f"(rise {r['rise']:.2f}, {r['steps']} pull steps)", flush=True)
        assert r["F_max"] > 0.0
        if theta <= 120.0:
            assert abs(ratio - 1.0) <= 0.30, (theta, ratio)
        else:
            assert abs(r["F_max"] - pred) <= 0.05 * scale, (theta, r["F_max"], pred)
    # the force falls with the angle, as the closed form does
    fm = [sweep[t]["F_max"] for t in ANGLES]
    assert all(a > b for a, b in zip(fm, fm[1:])), fm


@pytest.mark.slow
def test_detachment_torque_vanishes(sweep):
    for theta in ANGLES:
        r = sweep[theta]
        assert r["T_max"] <= 1e-9 * 10.0 * r["F_abs"], (theta, r["T_max"], r["F_abs"])
