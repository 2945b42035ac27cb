"""GPU against the FP64 oracle with open x ends (anti-bounce-back pressure
boundaries, section "Benchmarking hydrodynamic force", pressure inlet/outlet
eq.) and the tube wall of that benchmark.

- pressure-driven flow between the wall plane's faces, FP32 and FP16 storage;
- a layer of fluid a cut by both open ends (the colour of the populations that
  enter there);
- a liquid plug in a wetting tube (the tube's wall normal in the wetting rule);
- the benchmark's sphere in tube flow, reduced, with its force and path
  histories, and at full size (320x83x83, R_t = 40, R_p = 12.2);
- the guard that stops a run whose particle reaches an open end.

Bars as in tests/parity_util.py; the planes next to the open ends count as
boundary nodes.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSim
from paper_2505_10171_amd import workloads as W
from parity_util import compare_fields, compare_history, compare_particles

pytestmark = pytest.mark.gpu


def _gpu(cfg, phi0=None, parts=(), hist=0):
    from paper_2505_10171_amd.lbm import Simulation
    return Simulation(cfg, phi0, parts, history_steps=hist)


def _row(p, names):
    return np.concatenate([np.asarray(p[k], np.float64) for k in names])


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_channel_open_ends(storage):
    """32x4x17 between the wall plane's two faces, density 1.0025 at the inlet
    and 0.9975 at the outlet, from rest: 300 steps."""
    cfg = W.config(32, 4, 17, has_wall=1, rho0=1.0, sigma=0.0, open_x=1, rho_in=1.0025,
                   rho_out=0.9975, storage=storage)
    o = OracleSim(dict(cfg, storage="fp32"))
    g = _gpu(cfg)
    o.step(300)
    g.step(300)
    if storage == "fp32":
        compare_fields(g, o, label="channel, open ends, FP32", open_x=True)
    else:
        compare_fields(g, o, tol=1e-3, node_tol=None, label="channel, open ends, FP16")


def test_layer_cut_by_open_ends():
    """Between the wall plane's faces, a layer of fluid a (viscosity ratio
    1.25) 12 nodes thick whose flat interfaces run along x through both open
    ends, driven by a pressure difference of 2e-4: 100 steps.  The populations
    that enter through the ends carry the colour of the boundary nodes,
    interface nodes included.  (Thinner layers are no test case: with bands of
    7 nodes the two interfaces overlap and a one-ulp change of phi0 grows to an
    O(1) change of u within 30 steps, in the oracle alone, periodic or not; a
    drop cut by an open end neither: its Laplace pressure, which the boundary
    cannot hold, blows its liquid out of the box.)"""
    ny = 24
    cfg = W.config(24, ny, 12, has_wall=1, theta_wall_deg=90.0, sigma=0.01, tau_a=1.0,
                   tau_b=0.8, open_x=1, rho_in=0.0501, rho_out=0.0499)
    y = np.arange(ny, dtype=np.float64)
    prof = np.tanh(np.minimum(y - 5.5, 17.5 - y) / 2.0)
    phi0 = np.broadcast_to(prof[None, :, None], (12, ny, 24)).astype(np.float32).copy()
    o = OracleSim(cfg, phi0)
    g = _gpu(cfg, phi0)
    o.step(100)
    g.step(100)
    rho, u, phi, mask = o.fields()
    assert phi[1:, :, 0].max() > 0.99 and phi[1:, :, 0].min() < -0.99
    assert np.abs(phi[1:, :, 0]).min() < 0.5  # interface nodes on the inlet plane
    compare_fields(g, o, label="layer cut by the open ends", open_x=True)


@pytest.mark.parametrize("theta", [60.0, 120.0])
def test_tube_plug_wetting(theta):
    """A plug of fluid a in a tube of radius 6 (periodic x), wall angle theta:
    200 steps as its menisci curve."""
    cfg = W.config(40, 15, 15, has_wall=2, tube_R=6.0, sigma=0.01, theta_wall_deg=theta)
    x = np.arange(40, dtype=np.float64)
    prof = np.tanh(np.minimum(x - 10, 30 - x) / 2.0)
    phi0 = np.broadcast_to(prof, (15, 15, 40)).astype(np.float32).copy()
    o = OracleSim(cfg, phi0)
    g = _gpu(cfg, phi0)
    o.step(200)
    g.step(200)
    compare_fields(g, o, label=f"plug in a tube, {theta:g} deg")


def test_tube_sphere_reduced():
    """The benchmark's neutrally buoyant sphere in pressure-driven tube flow,
    reduced (R_t = 8, R_p = 3, 48 nodes): 200 steps, fields and the per-step
    hydrodynamic force, torque and path histories."""
    w = W.tube_reduced()
    steps = w["steps"]
    names = ("F_hyd", "T_hyd", "x", "v", "w")
    o = OracleSim(w["cfg"], None, w["particles"])
    g = _gpu(w["cfg"], None, w["particles"], hist=steps)
    ho = []
    for _ in range(steps):
        o.step(1)
        ho.append(_row(o.particles()[0], names))
    g.step(steps)
    ho = np.array(ho)
    assert ho[-1, 9] > 1e-3  # the sphere is carried downstream
    compare_fields(g, o, label="sphere in tube flow, reduced", open_x=True)
    _, h = g.particles(history=True)
    hg = np.concatenate([h[:, 0, 0:6], h[:, 0, 18:27]], axis=1)
    compare_history(hg, ho, names, w["particles"][0]["R"], label="sphere in tube flow")


def test_tube_segre_full_size():
    """The benchmark at the paper's sizes (tube radius 40, sphere radius 12.2,
    density 1.05, viscosity 0.457, 320 nodes long), 160 steps from rest (the
    pressure wave from the inlet has passed the sphere) in FP32 and FP16
    storage against one oracle run."""
    w = W.tube_segre()
    steps = 160
    o = OracleSim(w["cfg"], None, w["particles"])
    o.step(steps)
    fo, po = o.fields(), o.particles()
    o.close()
    assert np.abs(po[0]["F_hyd"]).max() > 1e-3  # the flow acts on the sphere
    for storage in ("fp32", "fp16"):
        g = _gpu(dict(w["cfg"], storage=storage), None, w["particles"])
        g.step(steps)
        if storage == "fp32":
            compare_fields(g, None, label="tube benchmark full size, FP32", fields=fo, open_x=True)
            compare_particles(g.particles(), po, ("F_hyd", "T_hyd", "x", "v"),
                              label="tube benchmark FP32", R=w["particles"][0]["R"])
        else:
            compare_fields(g, None, tol=1e-3, node_tol=None, fields=fo,
                           label="tube benchmark full size, FP16")
        g.close()


def test_open_end_guard():
    """A particle placed within R + 4 nodes of an open end is refused at
    creation; one carried there stops the run with LBM_ERANGE."""
    from paper_2505_10171_amd.lbm import LbmError
    cfg = W.config(30, 12, 12, has_wall=0, open_x=1, rho_in=0.05, rho_out=0.05)
    R = 3.0
    with pytest.raises(LbmError, match="open x end"):
        _gpu(cfg, None, [W.particle((5.0, 6.0, 6.0), R)])
    x0 = 30 - 1 - R - 4.0 - 0.25
    g = _gpu(cfg, None, [W.particle((x0, 6.0, 6.0), R, v=(0.1, 0, 0), kinematic=1)])
    g.step(2)
    g.sync()
    g.step(2)
    with pytest.raises(LbmError, match="open x end") as e:
        g.sync()
    assert e.value.code == -5


def test_march_depth_gives_identical_results():
    """The marching depth of the interface and moments passes (lbm_set_march)
    changes the blocks, not the arithmetic: fields after 30 steps of the
    reduced tube benchmark are bit-identical at depths 3, 5 and 12."""
    w = W.tube_reduced()
    out = []
    for planes in (3, 5, 12):
        g = _gpu(w["cfg"], None, w["particles"])
        g.set_march(0, planes)
        g.step(30)
        out.append(g.fields())
        g.close()
    for f in out[1:]:
        for a, b in zip(out[0], f):
            assert np.array_equal(a, b)


def test_held_sphere_against_the_tube():
    """A sphere held (prescribed velocity zero) at overlap 0.2 with the tube's
    wall, off-axis along a diagonal of the section: its contact force against
    the oracle's (the cylinder as a DEM contact surface)."""
    Rt, R, d0 = 8.0, 3.0, 0.2
    cfg = W.config(20, 19, 19, has_wall=2, tube_R=Rt)
    Rc = R + cfg["delta_R"]
    c = 9.0
    e = np.array([0.0, 1.0, -1.0]) / np.sqrt(2.0)   # from the axis towards the wall
    x0 = np.array([10.0, c, c]) + e * (Rt - Rc + d0)
    parts = [W.particle(tuple(x0), R, g_p=0.0, kinematic=1)]
    o = OracleSim(cfg, None, parts)
    g = _gpu(cfg, None, parts)
    o.step(2)
    g.step(2)
    fo, fg = np.array(o.particles()[0]["F_con"]), np.array(g.particles()[0]["F_con"])
    assert np.abs(fo + cfg["kn"] * d0 * e).max() <= 1e-12
    assert np.abs(fg - fo).max() <= 1e-9 * np.abs(fo).max()
