"""GPU (HIP library through the C ABI) against the FP64 CPU oracle.

Bars (tests/parity_util.py): masks and link lists bit-exact; FP32-storage
fields rho, u, phi within 1e-5 relative L2 over the fluid nodes and within 1e-4
of the field's largest magnitude at every fluid node next to a solid; FP64
particle force histories (and positions, velocities) within 1e-5 of their
largest magnitude; a torque within 1e-5 of its largest magnitude, or, where it
is a small residual of cancelling moments (|T| < 0.1 R_p |F|), of R_p max|F|;
FP16 storage within 1e-3.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSim
from paper_2505_10171_amd import workloads as W
from parity_util import compare_fields, compare_history, compare_particles, rel_l2

pytestmark = pytest.mark.gpu

HIST_NAMES = ("F_hyd", "T_hyd", "F_cap", "T_cap", "F_con", "T_con", "x", "v", "w")


def _gpu(cfg, phi0, parts, hist=0):
    from paper_2505_10171_amd.lbm import Simulation
    return Simulation(cfg, phi0, parts, history_steps=hist)


def _compare_fields(g, o, tol=1e-5, label=""):
    return compare_fields(g, o, tol=tol, label=label)[0]


def test_c1_sessile_drop_with_sphere():
    w = W.sessile_drop_c1()
    steps = w["steps"]
    g = _gpu(w["cfg"], w["phi0"], w["particles"], hist=steps)
    o = OracleSim(w["cfg"], w["phi0"], w["particles"])
    assert g.dem_substeps() == o.n_sub
    hist_o = []
    for t in range(steps):
        o.step(1)
        p = o.particles()[0]
        hist_o.append(np.concatenate([p[k] for k in ("F_hyd", "T_hyd", "F_cap", "T_cap", "F_con",
                                                      "T_con", "x", "v", "w")]))
    g.step(steps)
    _compare_fields(g, o, label="C1 200 steps")
    parts, hist_g = g.particles(history=True)
    hist_o = np.array(hist_o)
    assert hist_g.shape == (steps, 1, 27)
    compare_history(hist_g[:, 0, :], hist_o, HIST_NAMES, w["particles"][0]["R"], label="C1")
    lg, pg = g.links()
    lo, po = o.links()
    assert np.array_equal(lg, lo) and np.array_equal(pg, po)


def test_drop_ragged_lattice_no_particles():
    cfg = W.config(37, 29, 23, theta_wall_deg=70.0, sigma=0.02, body_force=(4e-6, -1e-6, 0.0))
    phi0 = W.drop_phi0(37, 29, 23, (15.3, 14.1, 0.5), 9.0)
    g = _gpu(cfg, phi0, [])
    o = OracleSim(cfg, phi0, [])
    g.step(80)
    o.step(80)
    _compare_fields(g, o, label="ragged 37x29x23")


@pytest.mark.parametrize("shape", [(10, 6, 5), (12, 3, 7), (70, 9, 9)])
def test_tiny_and_partial_boxes(shape):
    """Boxes narrower than every block tile (x < 16, y < 4), a z extent that
    leaves a partial plane march, and an x extent one past the widest tile."""
    nx, ny, nz = shape
    cfg = W.config(nx, ny, nz, theta_wall_deg=70.0, sigma=0.01, body_force=(3e-6, 0.0, 0.0))
    phi0 = W.drop_phi0(nx, ny, nz, (0.45 * nx, 0.5 * ny, 0.5), 0.4 * min(nx, 2 * nz))
    g = _gpu(cfg, phi0, [])
    o = OracleSim(cfg, phi0, [])
    g.step(40)
    o.step(40)
    _compare_fields(g, o, label=f"box {shape}")


def test_drop_free_periodic():
    cfg = W.config(24, 20, 28, has_wall=0, sigma=0.01, tau_a=0.8, tau_b=1.4)
    phi0 = W.drop_phi0(24, 20, 28, (11.5, 9.5, 13.5), 7.0)
    g = _gpu(cfg, phi0, [])
    o = OracleSim(cfg, phi0, [])
    g.step(100)
    o.step(100)
    _compare_fields(g, o, label="free drop, viscosity ratio")


@pytest.mark.parametrize("seed", range(4))
def test_mask_and_links_bitexact(seed):
    g_ = np.random.default_rng(500 + seed)
    L = (26, 22, 24)
    cfg = W.config(*L, has_wall=seed % 2)
    parts = []
    for k in range(5):
        R = float(g_.choice([1.5, 2.0, 2.5, 3.0, 4.0]))
        if k % 3 == 0:
            x = (L[0] - 0.5, 0.5, float(g_.integers(6, L[2] - 6)) + 0.5)
        elif k % 3 == 1:
            x = (float(g_.integers(0, L[0])), float(g_.integers(0, L[1])), 10.0)
            R = 3.0
        else:
            x = (g_.uniform(0, L[0]), g_.uniform(0, L[1]), g_.uniform(6, L[2] - 6))
        parts.append(W.particle(x, R, kinematic=1))
    g = _gpu(cfg, None, parts)
    o = OracleSim(cfg, None, parts)
    _, _, _, mg = g.fields()
    _, _, _, mo = o.fields()
    assert np.array_equal(mg, mo)
    lg, pg = g.links()
    lo, po = o.links()
    assert np.array_equal(lg, lo) and np.array_equal(pg, po)
    # moved state pushed to both sides: still bit-exact, fresh nodes refilled
    moved = [dict(p, x=tuple(np.array(p["x"]) + g_.uniform(-1.5, 1.5, 3))) for p in parts]
    for p in moved:
        p["x"] = (p["x"][0] % L[0], p["x"][1] % L[1], p["x"][2])
    g.push_particles(moved)
    o.set_particles(moved)
    _, _, _, mg = g.fields()
    _, _, _, mo = o.fields()
    assert np.array_equal(mg, mo)


def test_moving_particle_refill_and_bounce():
    """A particle with prescribed velocity and spin through a two-fluid box:
    moving bounce-back, momentum exchange and refilling against the oracle."""
    L = 24
    cfg = W.config(L, L, L, has_wall=0, sigma=0.01)
    # a liquid layer with two smooth interfaces (periodic in z)
    z = np.arange(L, dtype=float)
    prof = np.tanh((z - 5.7) / 2.0) * np.tanh((17.9 - z) / 2.0)
    phi0 = np.broadcast_to(prof[:, None, None], (L, L, L)).astype(np.float32)
    parts = [W.particle((6.2, 11.7, 17.4), 3.5, theta_deg=70.0, v=(0.03, 0.01, -0.005),
                        w=(0.0, 0.002, 0.001), kinematic=1)]
    g = _gpu(cfg, phi0, parts, hist=60)
    o = OracleSim(cfg, phi0, parts)
    Fo = []
    for _ in range(60):
        o.step(1)
        Fo.append(o.particles()[0]["F_hyd"])
    g.step(60)
    _compare_fields(g, o, label="moving particle")
    _, h = g.particles(history=True)
    Fo = np.array(Fo)
    err = np.abs(h[:, 0, 0:3] - Fo).max() / np.abs(Fo).max()
    assert err <= 1e-5, err


def test_mass_conservation_static_solids_gpu():
    cfg = W.config(32, 32, 24, sigma=0.01, theta_wall_deg=75.0)
    phi0 = W.drop_phi0(32, 32, 24, (16.0, 16.0, 0.5), 9.0)
    g = _gpu(cfg, phi0, [W.particle((24.0, 16.0, 5.5), 3.0, kinematic=1)])
    m0 = g.mass()
    g.step(500)
    m1 = g.mass()
    assert np.all(np.abs(m1 - m0) <= 2e-6 * m0.sum()), (m0, m1)


def test_poiseuille_gpu():
    nz, f, tau = 17, 1e-6, 0.8
    cfg = W.config(4, 4, nz, tau_a=tau, tau_b=tau, sigma=0.0, body_force=(f, 0, 0))
    g = _gpu(cfg, np.ones((nz, 4, 4), np.float32), [])
    g.step(6000)
    rho, u, phi, mask = g.fields()
    z = np.arange(1, nz, dtype=float)
    nu = (tau - 0.5) / 3.0
    exact = f / (2 * cfg["rho0"] * nu) * (z - 0.5) * (nz - 0.5 - z)
    assert np.abs(u[0, 1:, 0, 0] - exact).max() <= 1e-4 * exact.max()


def test_unstable_flow_is_reported():
    from paper_2505_10171_amd.lbm import LbmError, LBM_EUNSTABLE
    cfg = W.config(8, 8, 8, has_wall=0, body_force=(2e-2, 0, 0), sigma=0.0)
    g = _gpu(cfg, None, [])
    g.step(50)
    with pytest.raises(LbmError) as e:
        g.sync()
    assert e.value.code == LBM_EUNSTABLE
    with pytest.raises(LbmError):
        g.step(1)  # sticky error state


@pytest.mark.parametrize("n_cube", [3, 5])
def test_candidate_list_overflow_is_reported(n_cube):
    """A cubic cluster of n_cube^3 spheres (R = 1.5, contact radius 2.5) at
    spacing 3.2: every interior sphere has 26 partners within the candidate
    range (2.5 + 2.5 + 1.5 = 6.5 > 2 x 3.2), more than the 24 a list holds, so
    the step reports the overflow.  The spheres are held in place (prescribed
    zero velocity), so the overlapping contacts move nothing.  27 spheres take
    the DEM placement with all data in LDS; 125 the LDS contact view with the
    pair tests spread over the GPU."""
    from paper_2505_10171_amd.lbm import LbmError, LBM_ERANGE
    cfg = W.config(28, 28, 24)
    parts = [W.particle((6.0 + 3.2 * a, 6.0 + 3.2 * b, 4.0 + 3.2 * c), 1.5, sigma=cfg["sigma"],
                        kinematic=1)
             for a in range(n_cube) for b in range(n_cube) for c in range(n_cube)]
    g = _gpu(cfg, None, parts)
    g.step(1)
    with pytest.raises(LbmError) as e:
        g.sync()
    assert e.value.code == LBM_ERANGE


def _full_size(work_fn, steps, label, keys):
    """FP32 and FP16 storage of one workload against one oracle run."""
    w = work_fn()
    o = OracleSim(w["cfg"], w["phi0"], w["particles"])
    o.step(steps)
    fo, po = o.fields(), o.particles()
    o.close()
    R = max(p["R"] for p in w["particles"])
    for storage in ("fp32", "fp16"):
        g = _gpu(dict(w["cfg"], storage=storage), w["phi0"], w["particles"])
        g.step(steps)
        if storage == "fp32":
            compare_fields(g, None, label=f"{label}, {steps} steps, FP32", fields=fo)
            compare_particles(g.particles(), po, keys, label=f"{label} FP32", R=R)
        else:
            compare_fields(g, None, tol=1e-3, node_tol=None, label=f"{label}, {steps} steps, FP16",
                           fields=fo)
            compare_particles(g.particles(), po, ("x",), label=f"{label} FP16", tol=1e-3)
        g.close()


def test_full_size_drop_sweep_c2_parity():
    """The 256x128x96 drop-sweeping workload with its 20 spheres, in the launch
    configuration the benchmark times, 20 steps against the oracle, in FP32 and
    FP16 storage."""
    _full_size(W.drop_sweep_c2, 20, "C2 full size",
               ("F_hyd", "T_hyd", "F_cap", "T_cap", "F_con", "x", "v"))


def test_full_size_slab_c3_parity():
    """The 512x256x192 slab with its 500 spheres (the throughput-at-scale
    workload) at full size for two steps against the oracle, in FP32 and FP16
    storage: masks bit-exact, fields within 1e-5 (FP32) and 1e-3 (FP16),
    particle forces within 1e-5 of their scale."""
    _full_size(W.slab_c3, 2, "C3 full size", ("F_hyd", "T_hyd", "F_cap", "F_con", "x", "v"))


def test_mass_against_oracle():
    """Global FP64 masses of both fluids (lbm_mass) against the oracle's sums of
    its colour populations, after the 200 steps of the sessile drop with a
    sphere: within 1e-6 relative."""
    w = W.sessile_drop_c1()
    g = _gpu(w["cfg"], w["phi0"], w["particles"])
    o = OracleSim(w["cfg"], w["phi0"], w["particles"])
    for steps in (0, 200):
        g.step(steps)
        o.step(steps)
        mg, mo = g.mass(), o.mass()
        err = np.abs(mg - mo) / mo
        print(f"mass after {steps} steps: gpu {mg} oracle {mo} rel {err}", flush=True)
        assert np.all(err <= 1e-6), (steps, mg, mo)


def test_device_fields_match_host_fields():
    w = W.sessile_drop_c1()
    g = _gpu(w["cfg"], w["phi0"], w["particles"])
    g.step(10)
    rho, u, phi, mask = g.fields()
    rd, ud, pd = g.fields_device()
    assert np.array_equal(rd.cpu().numpy().reshape(rho.shape), rho)
    assert np.array_equal(pd.cpu().numpy().reshape(phi.shape), phi)
    assert np.array_equal(ud.cpu().numpy().reshape(u.shape), u)


def test_fp16_storage_c1_against_oracle():
    """FP16 population storage (scaled offsets, FP32 arithmetic) on the C1
    workload: masks bit-exact, velocity within 1e-3 relative L2 of the FP64
    oracle after 200 steps; rho and phi errors reported."""
    w = W.sessile_drop_c1()
    cfg = dict(w["cfg"], storage="fp16")
    g = _gpu(cfg, w["phi0"], w["particles"])
    o = OracleSim(w["cfg"], w["phi0"], w["particles"])
    g.step(w["steps"])
    o.step(w["steps"])
    rg, ug, pg, mg = g.fields()
    ro, uo, po, mo = o.fields()
    assert np.array_equal(mg, mo)
    fl = mo == 0
    e = dict(rho=rel_l2(rg[fl], ro[fl]), u=rel_l2(ug[:, fl], uo[:, fl]), phi=rel_l2(pg[fl], po[fl]))
    print("FP16 C1 200 steps", {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    pgp, pop_ = g.particles()[0], o.particles()[0]
    for k in ("F_hyd", "F_cap", "x"):
        print(k, np.abs(np.array(pgp[k]) - np.array(pop_[k])).max(), np.abs(pop_[k]).max())
    assert e["u"] <= 1e-3, e
    assert e["rho"] <= 1e-3 and e["phi"] <= 1e-3, e


def test_fp16_storage_free_drop():
    cfg = W.config(24, 20, 28, has_wall=0, sigma=0.01, tau_a=0.8, tau_b=1.4, storage="fp16")
    phi0 = W.drop_phi0(24, 20, 28, (11.5, 9.5, 13.5), 7.0)
    g = _gpu(cfg, phi0, [])
    o = OracleSim(dict(cfg, storage="fp32"), phi0, [])
    g.step(100)
    o.step(100)
    rg, ug, pg, mg = g.fields()
    ro, uo, po, mo = o.fields()
    e = dict(rho=rel_l2(rg, ro), u=rel_l2(ug, uo), phi=rel_l2(pg, po))
    print("FP16 free drop", {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    assert e["u"] <= 1e-3, e


@pytest.mark.parametrize("n_side", [5, 8, 28, 35])
def test_packed_spheres_in_contact(n_side):
    """A layer of n_side^2 spheres (R = 2, contact radius 3) on the wall, packed
    closer than their contact diameter, with jittered positions and random
    velocities and spins: every sphere presses on its neighbours and on the
    wall from the first sub-step, so normal, sliding and rolling springs all
    act.  25 spheres keep the DEM's data in LDS; 64 keep the contact view
    there, their pair tests spread over the GPU; 784 keep the contact view and
    search in one workgroup; 1,225 keep everything in global memory."""
    g0 = W.rng(77, n_side)
    L = 6 * n_side - 2                    # spacing L / n_side < 2 Rc = 6
    cfg = W.config(L, L, 16, theta_wall_deg=90.0)
    phi0 = W.slab_phi0(L, L, 16, 8.0)
    R = 2.0
    Rc = R + cfg["delta_R"]
    sp = L / n_side
    parts = []
    for a in range(n_side):
        for b in range(n_side):
            x = ((a + 0.5) * sp + g0.uniform(-0.1, 0.1), (b + 0.5) * sp + g0.uniform(-0.1, 0.1),
                 0.5 + Rc - 0.1 + g0.uniform(-0.05, 0.05))
            parts.append(W.particle(x, R, theta_deg=90.0, mu_s=0.5, mu_r=0.05, sigma=cfg["sigma"],
                                    v=tuple(g0.uniform(-0.01, 0.01, 3)),
                                    w=tuple(g0.uniform(-0.005, 0.005, 3))))
    g = _gpu(cfg, phi0, parts)
    o = OracleSim(cfg, phi0, parts)
    g.step(3)
    o.step(3)
    _compare_fields(g, o, label=f"{n_side}^2 packed spheres, 3 steps")
    pg, po = g.particles(), o.particles()
    assert np.abs(np.array([p["F_con"] for p in po])).max() > 0.1  # the contacts do act
    for k in ("F_con", "T_con", "x", "v", "w"):
        a = np.array([p[k] for p in pg])
        b = np.array([p[k] for p in po])
        scale = np.abs(b).max()
        if k == "T_con":
            scale = max(scale, R * np.abs(np.array([p["F_con"] for p in po])).max())
        assert np.abs(a - b).max() <= 1e-5 * scale, (k, np.abs(a - b).max(), scale)
    g.close()
    o.close()
