"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

The oracle is a plain, slow FP64 implementation of the coupled colour-gradient
lattice Boltzmann + DEM step of arXiv 2505.10171 (see lbm_oracle.c for the step
list and every reading of the paper it takes).  Nothing in the product library
imports this module.

The capillary-force sum (capillary-force eq.) is pinned by the paper's
detachment benchmark (oracle/detachment.py): the largest force on a sphere
pulled out of a liquid layer against Scheludko's closed form.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

Q = 19


class OrcConfig(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("has_wall", C.c_int32),
                ("rho0", C.c_double), ("tau_a", C.c_double), ("tau_b", C.c_double),
                ("sigma", C.c_double), ("beta", C.c_double), ("theta_wall_deg", C.c_double),
                ("body_force", C.c_double * 3),
                ("kn", C.c_double), ("kt", C.c_double), ("kr", C.c_double),
                ("gn", C.c_double), ("gt", C.c_double), ("gr", C.c_double),
                ("delta_R", C.c_double), ("cap_k", C.c_double), ("cap_dang_deg", C.c_double),
                ("n_particles", C.c_int32), ("pad0", C.c_int32),
                ("open_x", C.c_int32), ("pad1", C.c_int32),
                ("rho_in", C.c_double), ("rho_out", C.c_double), ("tube_R", C.c_double),
                ("n_boxes", C.c_int32), ("pad2", C.c_int32), ("boxes", C.c_int32 * 48)]


class OrcParticle(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("v", C.c_double * 3), ("w", C.c_double * 3),
                ("q", C.c_double * 4),
                ("R", C.c_double), ("rho_p", C.c_double), ("theta_deg", C.c_double),
                ("mu_s", C.c_double), ("mu_r", C.c_double), ("g_p", C.c_double),
                ("kinematic", C.c_int32), ("pad0", C.c_int32),
                ("F_hyd", C.c_double * 3), ("T_hyd", C.c_double * 3),
                ("F_cap", C.c_double * 3), ("T_cap", C.c_double * 3),
                ("F_con", C.c_double * 3), ("T_con", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcConfig), C.POINTER(C.c_float), C.POINTER(OrcParticle)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_dem_run.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_n_sub.argtypes = [C.c_void_p]
        L.orc_n_fresh.argtypes = [C.c_void_p]
        L.orc_n_fresh.restype = C.c_int64
        L.orc_fields.argtypes = [C.c_void_p, dp, dp, dp, C.POINTER(C.c_uint16)]
        L.orc_grad_force.argtypes = [C.c_void_p, dp, dp]
        L.orc_get_pops.argtypes = [C.c_void_p, dp, dp]
        L.orc_set_pops.argtypes = [C.c_void_p, dp, dp]
        L.orc_get_particles.argtypes = [C.c_void_p, C.POINTER(OrcParticle)]
        L.orc_set_particles.argtypes = [C.c_void_p, C.POINTER(OrcParticle)]
        L.orc_links.restype = C.c_int64
        L.orc_links.argtypes = [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_int32), C.c_int64]
        L.orc_mass.argtypes = [C.c_void_p, dp]
        L.orc_lattice.argtypes = [C.POINTER(C.c_int32), dp, C.POINTER(C.c_int32)]
        L.orc_mrt_matrix.argtypes = [dp, dp]
        L.orc_equilibrium.argtypes = [C.c_double, dp, dp]
        L.orc_guo_source.argtypes = [dp, dp, dp]
        L.orc_collide.argtypes = [dp, dp, dp, C.c_double, dp]
        L.orc_omega.restype = C.c_double
        L.orc_omega.argtypes = [C.POINTER(OrcConfig), C.c_double]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_round_state_f32.argtypes = [C.c_void_p]
        L.orc_round_state_f16.argtypes = [C.c_void_p]
        L.orc_set_regularisation.argtypes = [C.c_double, C.c_double, C.c_int]
        L.orc_get_regularisation.argtypes = [dp, dp, C.POINTER(C.c_int)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_config(cfg: dict, n_particles: int) -> OrcConfig:
    c = OrcConfig()
    c.nx, c.ny, c.nz = cfg["nx"], cfg["ny"], cfg["nz"]
    c.has_wall = int(cfg.get("has_wall", 1))
    for k in ("rho0", "tau_a", "tau_b", "sigma", "beta", "theta_wall_deg", "kn", "kt", "kr",
              "gn", "gt", "gr", "delta_R", "cap_k", "cap_dang_deg"):
        setattr(c, k, float(cfg[k]))
    for k in range(3):
        c.body_force[k] = float(cfg["body_force"][k])
    c.n_particles = n_particles
    c.open_x = int(cfg.get("open_x", 0))
    c.rho_in = float(cfg.get("rho_in", cfg["rho0"]))
    c.rho_out = float(cfg.get("rho_out", cfg["rho0"]))
    c.tube_R = float(cfg.get("tube_R", 0.0))
    boxes = list(cfg.get("boxes", ()))
    c.n_boxes = len(boxes)
    for b, box in enumerate(boxes[:8]):
        for k in range(6):
            c.boxes[6 * b + k] = int(box[k])
    return c


def make_particles(parts) -> "C.Array":
    arr = (OrcParticle * max(1, len(parts)))()
    for i, p in enumerate(parts):
        o = arr[i]
        for k in range(3):
            o.x[k] = p["x"][k]
            o.v[k] = p.get("v", (0, 0, 0))[k]
            o.w[k] = p.get("w", (0, 0, 0))[k]
        q = p.get("q", (1.0, 0.0, 0.0, 0.0))
        for k in range(4):
            o.q[k] = q[k]
        o.R, o.rho_p, o.theta_deg = p["R"], p["rho_p"], p["theta_deg"]
        o.mu_s, o.mu_r, o.g_p = p["mu_s"], p["mu_r"], p["g_p"]
        o.kinematic = int(p.get("kinematic", 0))
    return arr


def particle_dict(o: OrcParticle) -> dict:
    d = {k: np.array(getattr(o, k)[:]) for k in ("x", "v", "w", "q", "F_hyd", "T_hyd", "F_cap",
                                                  "T_cap", "F_con", "T_con")}
    for k in ("R", "rho_p", "theta_deg", "mu_s", "mu_r", "g_p"):
        d[k] = getattr(o, k)
    d["kinematic"] = o.kinematic
    return d


class OracleSim:
    """One simulation on the CPU in FP64."""

    def __init__(self, cfg: dict, phi0=None, particles=()):
        L = lib()
        self.cfg = dict(cfg)
        self.nx, self.ny, self.nz = cfg["nx"], cfg["ny"], cfg["nz"]
        self.N = self.nx * self.ny * self.nz
        self.np = len(particles)
        self._c = make_config(cfg, self.np)
        self._p = make_particles(particles)
        if phi0 is not None:
            self._phi0 = np.ascontiguousarray(phi0, dtype=np.float32).reshape(-1)
            assert self._phi0.size == self.N
            pp = self._phi0.ctypes.data_as(C.POINTER(C.c_float))
        else:
            pp = None
        self.h = L.orc_create(C.byref(self._c), pp, self._p)
        if not self.h:
            raise ValueError("oracle rejected the configuration")

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        rc = lib().orc_step(self.h, int(n))
        if rc != 0:
            raise RuntimeError(f"oracle step failed ({rc})")

    def dem_run(self, n, Fext=None):
        fe = None
        if Fext is not None:
            self._fe = np.ascontiguousarray(Fext, dtype=np.float64).reshape(-1)
            fe = _dp(self._fe)
        rc = lib().orc_dem_run(self.h, int(n), fe)
        if rc != 0:
            raise RuntimeError(f"oracle DEM failed ({rc})")

    @property
    def n_sub(self):
        return lib().orc_n_sub(self.h)

    @property
    def n_fresh(self):
        return lib().orc_n_fresh(self.h)

    def fields(self):
        """rho (nz,ny,nx), u (3,nz,ny,nx), phi (nz,ny,nx), mask (nz,ny,nx) uint16."""
        shp = (self.nz, self.ny, self.nx)
        rho = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        phi = np.zeros(self.N)
        mask = np.zeros(self.N, dtype=np.uint16)
        lib().orc_fields(self.h, _dp(rho), _dp(u), _dp(phi),
                         mask.ctypes.data_as(C.POINTER(C.c_uint16)))
        return rho.reshape(shp), u.reshape((3,) + shp), phi.reshape(shp), mask.reshape(shp)

    def grad_force(self):
        G = np.zeros(3 * self.N)
        F = np.zeros(3 * self.N)
        lib().orc_grad_force(self.h, _dp(G), _dp(F))
        shp = (self.nz, self.ny, self.nx, 3)
        return G.reshape(shp), F.reshape(shp)

    def pops(self):
        fa = np.zeros(self.N * Q)
        fb = np.zeros(self.N * Q)
        lib().orc_get_pops(self.h, _dp(fa), _dp(fb))
        return fa.reshape(self.N, Q), fb.reshape(self.N, Q)

    def set_pops(self, fa, fb):
        fa = np.ascontiguousarray(fa, dtype=np.float64).reshape(-1)
        fb = np.ascontiguousarray(fb, dtype=np.float64).reshape(-1)
        lib().orc_set_pops(self.h, _dp(fa), _dp(fb))

    def particles(self):
        arr = (OrcParticle * max(1, self.np))()
        lib().orc_get_particles(self.h, arr)
        return [particle_dict(arr[i]) for i in range(self.np)]

    def set_particles(self, parts):
        arr = make_particles(parts)
        lib().orc_set_particles(self.h, arr)

    def links(self):
        L = lib()
        cnt = L.orc_links(self.h, None, None, 0)
        out = np.zeros(max(1, cnt), dtype=np.uint32)
        pid = np.zeros(max(1, cnt), dtype=np.int32)
        L.orc_links(self.h, out.ctypes.data_as(C.POINTER(C.c_uint32)),
                    pid.ctypes.data_as(C.POINTER(C.c_int32)), cnt)
        return out[:cnt], pid[:cnt]

    def round_state_f32(self):
        """Sensitivity probe: round the state's departures from rest to FP32."""
        lib().orc_round_state_f32(self.h)

    def round_state_f16(self):
        """Sensitivity probe: round each total population as a 16-bit store
        relative to the node's density would (the colour difference kept)."""
        lib().orc_round_state_f16(self.h)

    def mass(self):
        out = np.zeros(2)
        lib().orc_mass(self.h, _dp(out))
        return out


def lattice():
    c = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    lib().orc_lattice(c.ctypes.data_as(C.POINTER(C.c_int32)), _dp(w),
                      opp.ctypes.data_as(C.POINTER(C.c_int32)))
    return c.reshape(19, 3), w, opp


def mrt_matrix():
    M = np.zeros(Q * Q)
    Mi = np.zeros(Q * Q)
    lib().orc_mrt_matrix(_dp(M), _dp(Mi))
    return M.reshape(Q, Q), Mi.reshape(Q, Q)


def equilibrium(rho, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(Q)
    lib().orc_equilibrium(float(rho), _dp(u), _dp(out))
    return out


def guo_source(u, F):
    u = np.ascontiguousarray(u, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(Q)
    lib().orc_guo_source(_dp(u), _dp(F), _dp(out))
    return out


def collide(f, feq, Fb, omega):
    f, feq, Fb = (np.ascontiguousarray(a, dtype=np.float64) for a in (f, feq, Fb))
    out = np.zeros(Q)
    lib().orc_collide(_dp(f), _dp(feq), _dp(Fb), float(omega), _dp(out))
    return out


def omega(cfg, phi):
    c = make_config(cfg, 0)
    return lib().orc_omega(C.byref(c), float(phi))


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


def get_regularisation():
    """(eps_g, eps_gt, blend): the normal's threshold, the wetting rotation's
    tangential threshold, and whether the rotation fades in."""
    g, gt, b = C.c_double(), C.c_double(), C.c_int()
    lib().orc_get_regularisation(C.byref(g), C.byref(gt), C.byref(b))
    return g.value, gt.value, b.value


class regularisation:
    """Context manager that runs the oracle with other interface thresholds
    (for instance the plain method: thresholds near zero, no fade-in) and
    restores the previous ones on exit.  Applies to every simulation stepped
    inside the block."""

    def __init__(self, eps_g, eps_gt, blend):
        self.new = (float(eps_g), float(eps_gt), int(blend))

    def __enter__(self):
        self.old = get_regularisation()
        lib().orc_set_regularisation(*self.new)
        return self

    def __exit__(self, *exc):
        lib().orc_set_regularisation(*self.old)
        return False
