"""Pins of the oracle's single-node arithmetic against the mathematics.

* D3Q19 isotropy (the lattice tensors that fix the weights and c_s^2 = 1/3);
* equilibrium moments (second-order Maxwellian truncation, refilling eq.);
* Guo forcing moments (forcing eq.) and the MRT collision (collision-operator
  eq. with the printed relaxation vector S) against an independently written
  two-relaxation-time form, which the printed S reduces to because every even
  non-conserved moment relaxes with omega and every odd one with omega';
* the harmonic-mean viscosity (viscosity eq.).
"""
import numpy as np
import pytest

from oracle import oracle as O


@pytest.fixture(scope="module")
def lat():
    return O.lattice()


def test_lattice_isotropy(lat):
    c, w, opp = lat
    assert c.shape == (19, 3)
    assert np.isclose(w.sum(), 1.0, atol=1e-15)
    # odd tensors vanish
    assert np.allclose(w @ c, 0.0, atol=1e-16)
    # second-order tensor = c_s^2 I with c_s^2 = 1/3
    T2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(T2, np.eye(3) / 3.0, atol=1e-15)
    # fourth-order tensor = c_s^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    T4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(T4, iso, atol=1e-15)
    # opposite directions
    for i in range(19):
        assert np.array_equal(c[opp[i]], -c[i])
    # the documented order: rest, axes, then xy, xz, yz pairs in ++,+-,-+,-- order
    assert np.array_equal(c[1], [1, 0, 0]) and np.array_equal(c[6], [0, 0, -1])
    assert np.array_equal(c[8], [1, -1, 0]) and np.array_equal(c[13], [-1, 0, 1])
    assert np.array_equal(c[18], [0, -1, -1])


def test_mrt_matrix(lat):
    c, w, opp = lat
    M, Mi = O.mrt_matrix()
    assert np.allclose(M @ Mi, np.eye(19), atol=1e-13)
    # rows are mutually orthogonal (the basis is an orthogonal polynomial basis)
    G = M @ M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-12)
    # conserved rows: density and momentum
    assert np.array_equal(M[0], np.ones(19))
    for k, row in ((0, 3), (1, 5), (2, 7)):
        assert np.array_equal(M[row], c[:, k].astype(float))
    # parity: rows 1,2,9..15 even in c, rows 4,6,8,16..18 odd
    for r in (1, 2, 9, 10, 11, 12, 13, 14, 15):
        assert np.array_equal(M[r], M[r][opp])
    for r in (4, 6, 8, 16, 17, 18):
        assert np.array_equal(M[r], -M[r][opp])


def test_equilibrium_moments(lat):
    c, w, opp = lat
    g = np.random.default_rng(1)
    for _ in range(20):
        rho = g.uniform(0.03, 0.08)
        u = g.uniform(-0.1, 0.1, 3)
        feq = O.equilibrium(rho, u)
        assert np.isclose(feq.sum(), rho, rtol=1e-15, atol=0)
        assert np.allclose(c.T @ feq, rho * u, rtol=0, atol=1e-17)
        P = np.einsum("i,ia,ib->ab", feq, c, c)
        assert np.allclose(P, rho * np.eye(3) / 3.0 + rho * np.outer(u, u), rtol=0, atol=1e-16)


def _trt(f, feq, Fb, om, opp):
    """Two-relaxation-time collision written from its definition: symmetric
    parts relax with omega, antisymmetric parts with omega'."""
    om2 = 8.0 * (2.0 - om) / (8.0 - om)
    s = lambda a: 0.5 * (a + a[opp])
    a = lambda a: 0.5 * (a - a[opp])
    d = f - feq
    return f - om * s(d) - om2 * a(d) + (1 - om / 2) * s(Fb) + (1 - om2 / 2) * a(Fb)


def test_mrt_equals_trt(lat):
    c, w, opp = lat
    g = np.random.default_rng(2)
    worst = 0.0
    for _ in range(200):
        rho = g.uniform(0.03, 0.08)
        f = rho * w * (1 + g.uniform(-0.3, 0.3, 19))
        F = g.uniform(-1e-3, 1e-3, 3)
        rho = f.sum()
        u = (c.T @ f + 0.5 * F) / rho
        feq = O.equilibrium(rho, u)
        Fb = O.guo_source(u, F)
        om = g.uniform(0.3, 1.9)
        a = O.collide(f, feq, Fb, om)
        b = _trt(f, feq, Fb, om, opp)
        worst = max(worst, np.abs(a - b).max() / np.abs(f).max())
    assert worst < 1e-14


def test_guo_forcing_moments(lat):
    c, w, opp = lat
    g = np.random.default_rng(3)
    for _ in range(50):
        rho = g.uniform(0.03, 0.08)
        u = g.uniform(-0.05, 0.05, 3)
        F = g.uniform(-1e-3, 1e-3, 3)
        Fb = O.guo_source(u, F)
        assert abs(Fb.sum()) < 1e-18
        assert np.allclose(c.T @ Fb, F, rtol=0, atol=1e-18)
        assert np.allclose(np.einsum("i,ia,ib->ab", Fb, c, c), np.outer(u, F) + np.outer(F, u),
                           rtol=0, atol=1e-18)
        # the collision adds F to momentum and (1 - omega/2)(uF + Fu) to the
        # second moment of an equilibrium state (forcing eq. with S)
        feq = O.equilibrium(rho, u)
        om = g.uniform(0.3, 1.9)
        d = O.collide(feq, feq, Fb, om) - feq
        # (d is the difference of two O(1e-3) arrays: rounding ~1e-19 per entry)
        assert abs(d.sum()) < 1e-17
        assert np.allclose(c.T @ d, F, rtol=0, atol=1e-17)
        assert np.allclose(np.einsum("i,ia,ib->ab", d, c, c),
                           (1 - om / 2) * (np.outer(u, F) + np.outer(F, u)), rtol=0, atol=1e-17)


def test_collision_relaxes_stress(lat):
    """A shear-stress perturbation decays by (1 - omega) per collision; the
    heat-flux-like odd moment by (1 - omega')."""
    c, w, opp = lat
    M, Mi = O.mrt_matrix()
    rho, u = 0.05, np.array([0.01, -0.02, 0.005])
    feq = O.equilibrium(rho, u)
    for om in (0.5, 1.0, 1.6):
        om2 = 8 * (2 - om) / (8 - om)
        f = feq + 1e-5 * Mi[:, 13] / np.linalg.norm(Mi[:, 13])  # pxy perturbation
        out = O.collide(f, feq, np.zeros(19), om)
        assert np.isclose((M @ (out - feq))[13], (1 - om) * (M @ (f - feq))[13], rtol=1e-12)
        f = feq + 1e-5 * Mi[:, 4] / np.linalg.norm(Mi[:, 4])  # qx perturbation
        out = O.collide(f, feq, np.zeros(19), om)
        assert np.isclose((M @ (out - feq))[4], (1 - om2) * (M @ (f - feq))[4], rtol=1e-12)
        # magic combination (1/omega - 1/2)(1/omega' - 1/2) = 3/16
        assert np.isclose((1 / om - 0.5) * (1 / om2 - 0.5), 3 / 16, rtol=1e-14)


def test_harmonic_viscosity():
    from paper_2505_10171_amd import workloads as W
    cfg = W.config(4, 4, 4, tau_a=0.664, tau_b=2.138)
    assert np.isclose(O.omega(cfg, 1.0), 1 / 0.664, rtol=1e-14)
    assert np.isclose(O.omega(cfg, -1.0), 1 / 2.138, rtol=1e-14)
    nua, nub = (0.664 - 0.5) / 3, (2.138 - 0.5) / 3
    for phi in (-0.5, 0.0, 0.3):
        nu = 1.0 / ((1 + phi) / (2 * nua) + (1 - phi) / (2 * nub))
        assert np.isclose(O.omega(cfg, phi), 1 / (0.5 + 3 * nu), rtol=1e-14)
    cfg = W.config(4, 4, 4, tau_a=1.0, tau_b=1.0)
    for phi in (-1, -0.3, 0.0, 0.9, 1):
        assert O.omega(cfg, phi) == 1.0
