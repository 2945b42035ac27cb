"""Thin ctypes binding of liblbm (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides the device workspace (a uint8 tensor on the GPU) and the HIP
stream.  The library is loaded from this package's csrc/ directory; if it is
missing the import fails loudly (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "csrc", "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EUNSTABLE, LBM_ERANGE, LBM_ESTATE = 0, -1, -2, -3, -4, -5, -6
LBM_STORE_FP32, LBM_STORE_FP16 = 0, 1
LBM_F_RHO, LBM_F_U, LBM_F_PHI, LBM_F_MASK, LBM_F_POPS, LBM_F_FORCE = 1, 2, 4, 8, 16, 32
HIST_DOUBLES = 27

EXPORTS = ["lbm_workspace_bytes", "lbm_create", "lbm_step", "lbm_sync", "lbm_particles_sync",
           "lbm_fields", "lbm_fields2", "lbm_links", "lbm_mass", "lbm_dem_substeps", "lbm_destroy",
           "lbm_last_error", "lbm_profile", "lbm_profile_read", "lbm_use_graph",
           "lbm_autotune", "lbm_set_tile", "lbm_set_march", "lbm_mass_all_noalloc"]
PROFILE_KINDS = ("fused", "particles", "moments", "interface", "links")


class LbmConfig(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("has_wall", C.c_int32),
                ("rho0", C.c_double), ("tau_a", C.c_double), ("tau_b", C.c_double),
                ("sigma", C.c_double), ("beta", C.c_double), ("theta_wall_deg", C.c_double),
                ("body_force", C.c_double * 3),
                ("kn", C.c_double), ("kt", C.c_double), ("kr", C.c_double),
                ("gn", C.c_double), ("gt", C.c_double), ("gr", C.c_double),
                ("delta_R", C.c_double), ("cap_k", C.c_double), ("cap_dang_deg", C.c_double),
                ("storage", C.c_int32), ("n_particles", C.c_int32),
                ("open_x", C.c_int32), ("pad0", C.c_int32),
                ("rho_in", C.c_double), ("rho_out", C.c_double), ("tube_R", C.c_double),
                ("n_boxes", C.c_int32), ("pad1", C.c_int32), ("boxes", C.c_int32 * 48)]


class LbmParticle(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("v", C.c_double * 3), ("w", C.c_double * 3),
                ("q", C.c_double * 4), ("R", C.c_double), ("rho_p", C.c_double),
                ("theta_deg", C.c_double), ("mu_s", C.c_double), ("mu_r", C.c_double),
                ("g_p", C.c_double), ("kinematic", C.c_int32), ("pad0", C.c_int32),
                ("F_hyd", C.c_double * 3), ("T_hyd", C.c_double * 3),
                ("F_cap", C.c_double * 3), ("T_cap", C.c_double * 3),
                ("F_con", C.c_double * 3), ("T_con", C.c_double * 3)]


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load liblbm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"liblbm.so not found at {path}: build it with "
                          "`python -m paper_2505_10171_amd.build` (hipcc, gfx950)")
    # torch first: it may bring its own HIP runtime, and the library must bind
    # to that same runtime (device pointers and streams come from torch).
    # Loaded the other way round, a process holds two runtimes and the first
    # copy into torch memory fails.
    import torch  # noqa: F401
    L = C.CDLL(path)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    L.lbm_workspace_bytes.restype = sz
    L.lbm_workspace_bytes.argtypes = [C.POINTER(LbmConfig), i32, C.POINTER(C.POINTER(LbmParticle)), i32]
    L.lbm_create.restype = C.c_int
    L.lbm_create.argtypes = [C.POINTER(LbmConfig), i32, C.POINTER(C.POINTER(C.c_float)),
                             C.POINTER(C.POINTER(LbmParticle)), i32, vp, sz, vp, C.POINTER(vp)]
    L.lbm_step.argtypes = [vp, i32]
    L.lbm_sync.argtypes = [vp]
    L.lbm_particles_sync.argtypes = [vp, i32, i32, C.POINTER(LbmParticle), i32,
                                     C.POINTER(C.c_double), i32, C.POINTER(i32)]
    L.lbm_fields.argtypes = [vp, i32, C.c_uint32, vp, vp, vp, vp, vp, i32]
    L.lbm_fields2.argtypes = [vp, i32, C.c_uint32, vp, vp, vp, vp, vp, vp, i32]
    L.lbm_links.argtypes = [vp, i32, C.POINTER(C.c_uint32), C.POINTER(i32), i64, C.POINTER(i64)]
    L.lbm_mass.argtypes = [vp, i32, C.POINTER(C.c_double)]
    L.lbm_mass_all_noalloc.argtypes = [vp, C.POINTER(C.c_double), i32]
    L.lbm_dem_substeps.argtypes = [vp, i32, C.POINTER(i32)]
    L.lbm_profile.argtypes = [vp, i32]
    L.lbm_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64), i32]
    L.lbm_use_graph.argtypes = [vp, i32]
    L.lbm_autotune.argtypes = [vp, i32, C.POINTER(i32)]
    L.lbm_set_tile.argtypes = [vp, i32, i32]
    L.lbm_set_march.argtypes = [vp, i32, i32]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = None
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = C.c_char_p
    _lib = L
    return L


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblbm error {code}: {msg}")
        self.code = code


def make_config(cfg: dict, n_particles: int) -> LbmConfig:
    c = LbmConfig()
    c.nx, c.ny, c.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg["nz"])
    c.has_wall = int(cfg.get("has_wall", 1))
    for k in ("rho0", "tau_a", "tau_b", "sigma", "beta", "theta_wall_deg", "kn", "kt", "kr",
              "gn", "gt", "gr", "delta_R", "cap_k", "cap_dang_deg"):
        setattr(c, k, float(cfg[k]))
    for k in range(3):
        c.body_force[k] = float(cfg["body_force"][k])
    st = cfg.get("storage", "fp32")
    c.storage = LBM_STORE_FP16 if st in ("fp16", LBM_STORE_FP16) else LBM_STORE_FP32
    c.n_particles = int(n_particles)
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


def make_particles(parts):
    arr = (LbmParticle * max(1, len(parts)))()
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


def particle_dict(o: LbmParticle) -> dict:
    d = {k: np.array(getattr(o, k)[:]) for k in ("x", "v", "w", "q", "F_hyd", "T_hyd", "F_cap",
                                                  "T_cap", "F_con", "T_con")}
    for k in ("R", "rho_p", "theta_deg", "mu_s", "mu_r", "g_p"):
        d[k] = getattr(o, k)
    d["kinematic"] = o.kinematic
    return d


class Context:
    """A set of independent simulations advanced together on one GPU stream."""

    def __init__(self, sims, history_steps: int = 0, device: str = "cuda:0", stream=None):
        """sims: list of dicts with keys cfg (workloads.config), phi0 (array or
        None), particles (list of workloads.particle dicts)."""
        import torch
        L = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.n = len(sims)
        self.sims = sims
        self._cfg = (LbmConfig * self.n)()
        self._parts = []
        self._phi = []
        pp = (C.POINTER(LbmParticle) * self.n)()
        ph = (C.POINTER(C.c_float) * self.n)()
        for i, s in enumerate(sims):
            parts = list(s.get("particles", ()))
            self._cfg[i] = make_config(s["cfg"], len(parts))
            arr = make_particles(parts)
            self._parts.append(arr)
            pp[i] = C.cast(arr, C.POINTER(LbmParticle)) if parts else None
            if s.get("phi0") is not None:
                a = np.ascontiguousarray(s["phi0"], dtype=np.float32).reshape(-1)
                self._phi.append(a)
                ph[i] = a.ctypes.data_as(C.POINTER(C.c_float))
            else:
                self._phi.append(None)
                ph[i] = None
        nbytes = L.lbm_workspace_bytes(self._cfg, self.n, pp, int(history_steps))
        if nbytes == 0:
            raise LbmError(LBM_EINVAL, "invalid configuration")
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.history_steps = int(history_steps)
        h = C.c_void_p()
        rc = L.lbm_create(self._cfg, self.n, ph, pp, int(history_steps),
                          C.c_void_p(self.workspace.data_ptr()), C.c_size_t(nbytes),
                          C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self.h = h
        if rc != 0:
            msg = L.lbm_last_error(h)
            self.close()
            raise LbmError(rc, msg.decode() if msg else "create failed")

    # ------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load_library().lbm_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            msg = load_library().lbm_last_error(self.h)
            raise LbmError(rc, msg.decode() if msg else "")

    # ---------------------------------------------------------------- calls
    def step(self, n: int = 1):
        self._check(load_library().lbm_step(self.h, int(n)))

    def sync(self):
        self._check(load_library().lbm_sync(self.h))

    def _np(self, sim):
        return len(self.sims[sim].get("particles", ()))

    def particles(self, sim: int = 0, history: bool = False):
        n = self._np(sim)
        arr = (LbmParticle * max(1, n))()
        nh = C.c_int32(0)
        hbuf = None
        hptr = None
        if history and self.history_steps > 0 and n > 0:
            hbuf = np.zeros(self.history_steps * n * HIST_DOUBLES)
            hptr = hbuf.ctypes.data_as(C.POINTER(C.c_double))
        self._check(load_library().lbm_particles_sync(self.h, sim, 0, arr, n, hptr,
                                                      self.history_steps if hptr else 0,
                                                      C.byref(nh)))
        parts = [particle_dict(arr[i]) for i in range(n)]
        if history:
            h = (hbuf[: nh.value * n * HIST_DOUBLES].reshape(nh.value, n, HIST_DOUBLES)
                 if hbuf is not None else np.zeros((0, n, HIST_DOUBLES)))
            return parts, h
        return parts

    def push_particles(self, parts, sim: int = 0):
        arr = make_particles(parts)
        self._check(load_library().lbm_particles_sync(self.h, sim, 1, arr, len(parts), None, 0,
                                                      None))

    def fields(self, sim: int = 0):
        """rho (nz,ny,nx), u (3,nz,ny,nx), phi (nz,ny,nx) as float32; mask uint16."""
        c = self._cfg[sim]
        N = c.nx * c.ny * c.nz
        shp = (c.nz, c.ny, c.nx)
        rho = np.zeros(N, np.float32)
        u = np.zeros(3 * N, np.float32)
        phi = np.zeros(N, np.float32)
        mask = np.zeros(N, np.uint16)
        self._check(load_library().lbm_fields(
            self.h, sim, LBM_F_RHO | LBM_F_U | LBM_F_PHI | LBM_F_MASK,
            rho.ctypes.data, u.ctypes.data, phi.ctypes.data, mask.ctypes.data, None, 0))
        return rho.reshape(shp), u.reshape((3,) + shp), phi.reshape(shp), mask.reshape(shp)

    def phi_mask(self, sim: int = 0):
        """Order parameter and solid mask only (nz, ny, nx)."""
        c = self._cfg[sim]
        shp = (c.nz, c.ny, c.nx)
        N = c.nx * c.ny * c.nz
        phi = np.zeros(N, np.float32)
        mask = np.zeros(N, np.uint16)
        self._check(load_library().lbm_fields(self.h, sim, LBM_F_PHI | LBM_F_MASK, None, None,
                                              phi.ctypes.data, mask.ctypes.data, None, 0))
        return phi.reshape(shp), mask.reshape(shp)

    def force(self, sim: int = 0):
        """Force per volume (CSF + body force), shape (nz, ny, nx, 3), float32."""
        c = self._cfg[sim]
        N = c.nx * c.ny * c.nz
        F = np.zeros(3 * N, np.float32)
        self._check(load_library().lbm_fields2(self.h, sim, LBM_F_FORCE, None, None, None,
                                               F.ctypes.data, None, None, 0))
        return np.moveaxis(F.reshape(3, c.nz, c.ny, c.nx), 0, -1)

    def fields_device(self, sim: int = 0):
        """rho, u, phi as torch tensors on the device (no host copy)."""
        torch = self.torch
        c = self._cfg[sim]
        N = c.nx * c.ny * c.nz
        rho = torch.empty(N, dtype=torch.float32, device=self.device)
        u = torch.empty(3 * N, dtype=torch.float32, device=self.device)
        phi = torch.empty(N, dtype=torch.float32, device=self.device)
        self._check(load_library().lbm_fields(self.h, sim, LBM_F_RHO | LBM_F_U | LBM_F_PHI,
                                              rho.data_ptr(), u.data_ptr(), phi.data_ptr(),
                                              None, None, 1))
        return rho, u, phi

    def pops(self, sim: int = 0):
        c = self._cfg[sim]
        N = c.nx * c.ny * c.nz
        dt = np.float16 if c.storage == LBM_STORE_FP16 else np.float32
        Np = (N + 63) // 64 * 64
        out = np.zeros(19 * Np, dt)
        self._check(load_library().lbm_fields(self.h, sim, LBM_F_POPS, None, None, None, None,
                                              out.ctypes.data, 0))
        # blocks of 64 nodes, 19 runs of 64 values each -> 19 planes of N
        return out.reshape(Np // 64, 19, 64).transpose(1, 0, 2).reshape(19, Np)[:, :N]

    def links(self, sim: int = 0):
        L = load_library()
        cnt = C.c_int64(0)
        self._check(L.lbm_links(self.h, sim, None, None, 0, C.byref(cnt)))
        out = np.zeros(max(1, cnt.value), np.uint32)
        pid = np.zeros(max(1, cnt.value), np.int32)
        self._check(L.lbm_links(self.h, sim, out.ctypes.data_as(C.POINTER(C.c_uint32)),
                                pid.ctypes.data_as(C.POINTER(C.c_int32)), cnt.value,
                                C.byref(cnt)))
        return out[: cnt.value], pid[: cnt.value]

    def mass(self, sim: int = 0):
        out = np.zeros(2)
        self._check(load_library().lbm_mass(self.h, sim, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def mass_all_noalloc(self):
        """FP64 masses (a, b) of every simulation, (n_sims, 2), through the
        entry point that allocates nothing."""
        out = np.zeros((self.n, 2))
        self._check(load_library().lbm_mass_all_noalloc(
            self.h, out.ctypes.data_as(C.POINTER(C.c_double)), 0))
        return out

    def profile(self, enable: bool = True, every: int = 1):
        """Time the phases of every `every`-th step with HIP events (off: enable=False)."""
        self._check(load_library().lbm_profile(self.h, int(every) if enable else 0))

    def profile_read(self):
        """{kind: (total_ms, launches)} for the fused, particle (other than
        the links), moments, interface and link phases."""
        n = len(PROFILE_KINDS)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        self._check(load_library().lbm_profile_read(self.h, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(PROFILE_KINDS)}

    def autotune(self, reps: int = 5):
        """Pick the per-node block shape of every box class; returns the tile
        width chosen per simulation (0 = consecutive nodes)."""
        out = (C.c_int32 * self.n)()
        self._check(load_library().lbm_autotune(self.h, int(reps), out))
        return list(out)

    def set_tile(self, sim: int, tile_x: int):
        self._check(load_library().lbm_set_tile(self.h, int(sim), int(tile_x)))

    def set_march(self, sim: int, planes: int):
        self._check(load_library().lbm_set_march(self.h, int(sim), int(planes)))

    def use_graph(self, enable: bool = True):
        """Replay pairs of steps from a captured HIP graph (needs a non-null stream)."""
        self._check(load_library().lbm_use_graph(self.h, int(bool(enable))))

    def dem_substeps(self, sim: int = 0):
        v = C.c_int32(0)
        self._check(load_library().lbm_dem_substeps(self.h, sim, C.byref(v)))
        return v.value


def Simulation(cfg, phi0=None, particles=(), **kw) -> Context:
    """One simulation in its own context."""
    return Context([dict(cfg=cfg, phi0=phi0, particles=list(particles))], **kw)
