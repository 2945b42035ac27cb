"""ctypes binding of the surrogate C ABI (include/srg.h): argument marshalling
only; training and inference run in the HIP kernels of liblbm.so."""
from __future__ import annotations

import ctypes as C

import numpy as np

from .lbm import LBM_EINVAL, LbmError, load_library

SRG_IN, SRG_OUT, SRG_PARAMS = 6, 51, 212275
SRG_EXPORTS = ["srg_workspace_bytes", "srg_create", "srg_set_params", "srg_get_params",
               "srg_set_train", "srg_train", "srg_gradients", "srg_predict", "srg_sync",
               "srg_destroy", "srg_last_error"]
_ready = False


def library():
    global _ready
    L = load_library()
    if not _ready:
        vp, i32, u64, sz = C.c_void_p, C.c_int32, C.c_uint64, C.c_size_t
        fp = C.POINTER(C.c_float)
        ip = C.POINTER(C.c_int32)
        L.srg_workspace_bytes.restype = sz
        L.srg_workspace_bytes.argtypes = [i32, i32]
        L.srg_create.argtypes = [vp, sz, i32, i32, vp, C.POINTER(vp)]
        L.srg_set_params.argtypes = [vp, fp]
        L.srg_get_params.argtypes = [vp, fp]
        L.srg_set_train.argtypes = [vp, fp, ip, fp, i32]
        L.srg_train.argtypes = [vp, i32, i32, C.c_float, C.c_float, u64, fp]
        L.srg_gradients.argtypes = [vp, fp, ip, fp, i32, C.c_float, fp, fp]
        L.srg_predict.argtypes = [vp, vp, i32, vp, i32, i32]
        L.srg_sync.argtypes = [vp]
        L.srg_destroy.argtypes = [vp]
        L.srg_destroy.restype = None
        L.srg_last_error.argtypes = [vp]
        L.srg_last_error.restype = C.c_char_p
        _ready = True
    return L


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Surrogate:
    """MLP 6 -> 256 x4 -> 51 trained and evaluated with BF16 MFMA kernels."""

    def __init__(self, max_batch: int = 1024, max_train: int = 4096, device: str = "cuda:0",
                 stream=None):
        import torch
        L = library()
        self.torch = torch
        nbytes = L.srg_workspace_bytes(int(max_batch), int(max_train))
        if nbytes == 0:
            raise LbmError(LBM_EINVAL, "max_batch must be a multiple of 64")
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = L.srg_create(C.c_void_p(self.workspace.data_ptr()), C.c_size_t(nbytes), int(max_batch),
                          int(max_train), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self.h = h
        self.max_batch = max_batch
        if rc != 0:
            raise LbmError(rc, "srg_create failed")

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            library().srg_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            msg = library().srg_last_error(self.h)
            raise LbmError(rc, msg.decode() if msg else "")

    @staticmethod
    def _fp(a):
        return a.ctypes.data_as(C.POINTER(C.c_float))

    def set_params(self, flat):
        flat = _f32(flat)
        assert flat.size == SRG_PARAMS
        self._check(library().srg_set_params(self.h, self._fp(flat)))

    def get_params(self):
        out = np.zeros(SRG_PARAMS, np.float32)
        self._check(library().srg_get_params(self.h, self._fp(out)))
        return out

    def set_train(self, X, label, traj):
        X = _f32(X, (-1, SRG_IN))
        lab = np.ascontiguousarray(label, dtype=np.int32)
        tr = _f32(traj, (-1, 48))
        self._keep = (X, lab, tr)
        self._check(library().srg_set_train(self.h, self._fp(X),
                                            lab.ctypes.data_as(C.POINTER(C.c_int32)),
                                            self._fp(tr), X.shape[0]))

    def train(self, epochs: int, batch: int = 256, lr: float = 1e-3, w_traj: float = 1.0,
              seed: int = 0):
        out = np.zeros(max(1, epochs), np.float32)
        self._check(library().srg_train(self.h, int(epochs), int(batch), float(lr), float(w_traj),
                                        int(seed), self._fp(out)))
        return out[:epochs]

    def gradients(self, X, label, traj, w_traj: float = 1.0):
        X = _f32(X, (-1, SRG_IN))
        lab = np.ascontiguousarray(label, dtype=np.int32)
        tr = _f32(traj, (-1, 48))
        g = np.zeros(SRG_PARAMS, np.float32)
        loss = C.c_float(0.0)
        self._check(library().srg_gradients(self.h, self._fp(X),
                                            lab.ctypes.data_as(C.POINTER(C.c_int32)),
                                            self._fp(tr), X.shape[0], float(w_traj), self._fp(g),
                                            C.byref(loss)))
        return g, loss.value

    def predict(self, X):
        """Host arrays in and out: y (n x 51)."""
        X = _f32(X, (-1, SRG_IN))
        y = np.zeros((X.shape[0], SRG_OUT), np.float32)
        self._check(library().srg_predict(self.h, X.ctypes.data, X.shape[0], y.ctypes.data, 0, 0))
        return y

    def predict_device(self, X, y):
        """Device tensors (float32, contiguous): X (n x 6) -> y (n x 51), asynchronous."""
        self._check(library().srg_predict(self.h, C.c_void_p(X.data_ptr()), X.shape[0],
                                          C.c_void_p(y.data_ptr()), 1, 1))

    def sync(self):
        self._check(library().srg_sync(self.h))


def he_init(seed: int, sizes=(6, 256, 256, 256, 256, 51)):
    """He-normal weights and zero biases from numpy Generator(PCG64(seed))."""
    g = np.random.Generator(np.random.PCG64(seed))
    ps = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        ps.append(g.normal(0.0, np.sqrt(2.0 / a), size=(a, b)))
        ps.append(np.zeros(b))
    return ps


def flatten(params):
    """Canonical flat order of a list [W1, b1, ..., W5, b5] (W as in x out)."""
    return np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in params]).astype(np.float32)


def unflatten(flat, sizes=(6, 256, 256, 256, 256, 51)):
    ps, k = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        ps.append(np.asarray(flat[k:k + a * b]).reshape(a, b))
        k += a * b
        ps.append(np.asarray(flat[k:k + b]))
        k += b
    return ps
