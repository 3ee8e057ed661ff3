"""ctypes binding of the surrogate network (include/lbsg.h): argument marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np

from . import lbch
from .lbch import _check, _stream_handle, lib

MAX_LEVELS = 6


class Arch(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("chans", ctypes.c_int32 * MAX_LEVELS), ("in_ch", ctypes.c_int32),
                ("out_scale", ctypes.c_float)]


def make_arch(chans, in_ch, out_scale=1.0) -> Arch:
    a = Arch()
    a.levels = len(chans)
    for i, c in enumerate(chans):
        a.chans[i] = c
    a.in_ch = in_ch
    a.out_scale = out_scale
    return a


_SIGS = {
    "lbsg_create": (ctypes.c_int, [ctypes.POINTER(Arch), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "lbsg_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "lbsg_param_count": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "lbsg_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int64]),
    "lbsg_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int64]),
    "lbsg_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_void_p]),
    "lbsg_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbsg_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                       ctypes.POINTER(ctypes.c_double)]),
    "lbsg_gather": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_float), ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbsg_gather_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_float), ctypes.c_int32, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "lbsg_predict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
}
_bound = False


def _bind():
    global _bound
    if not _bound:
        h = lib()
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return lib()


class Surrogate:
    """The periodic U-Net (lbsg_net). Device tensors are passed as raw pointers (e.g. torch .data_ptr())."""

    def __init__(self, chans, in_ch, max_batch, max_h, max_w, train=True, seed=0, stream=None, out_scale=1.0):
        L = _bind()
        self.arch = make_arch(chans, in_ch, out_scale)
        self.chans, self.in_ch = tuple(chans), in_ch
        self._h = ctypes.c_void_p()
        _check(L.lbsg_create(ctypes.byref(self.arch), max_batch, max_h, max_w, 1 if train else 0, seed,
                             _stream_handle(stream), ctypes.byref(self._h)), "lbsg_create")
        n = ctypes.c_int64()
        _check(L.lbsg_param_count(self._h, ctypes.byref(n)), "lbsg_param_count")
        self.nparam = n.value

    def close(self):
        if self._h:
            _bind().lbsg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.empty(self.nparam, dtype=np.float32)
        _check(_bind().lbsg_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), self.nparam),
               "lbsg_get_params")
        return out

    def set_params(self, flat: np.ndarray):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check(_bind().lbsg_set_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
               "lbsg_set_params")

    def forward(self, x_ptr: int, batch: int, h: int, w: int, out_ptr: int):
        _check(_bind().lbsg_forward(self._h, ctypes.c_void_p(x_ptr), batch, h, w, ctypes.c_void_p(out_ptr)),
               "lbsg_forward")

    def backward(self, dphi_ptr: int, grads_ptr: int):
        _check(_bind().lbsg_backward(self._h, ctypes.c_void_p(dphi_ptr), ctypes.c_void_p(grads_ptr)), "lbsg_backward")

    def train_step(self, x_ptr, target_ptr, batch, h, w, margin, lr, want_loss=True):
        loss = ctypes.c_double()
        _check(_bind().lbsg_train_step(self._h, ctypes.c_void_p(x_ptr), ctypes.c_void_p(target_ptr), batch, h, w,
                                       margin, lr, ctypes.byref(loss) if want_loss else None), "lbsg_train_step")
        return loss.value if want_loss else None

    def predict(self, phi_ptr: int, cond, h: int, w: int, out_ptr: int):
        c = (ctypes.c_float * max(1, len(cond)))(*cond)
        _check(_bind().lbsg_predict(self._h, ctypes.c_void_p(phi_ptr), c, len(cond), h, w, ctypes.c_void_p(out_ptr)),
               "lbsg_predict")


def layer_names(levels):
    names = []
    for l in range(levels):
        names += [f"enc{l}a", f"enc{l}b"]
    for l in range(levels - 2, -1, -1):
        names += [f"dec{l}a", f"dec{l}b"]
    return names + ["head"]


def gather(field_ptr: int, h: int, w: int, yx: np.ndarray, crop: int, cond: np.ndarray | None,
           x_ptr: int | None, y_ptr: int | None, stream=None, noalloc: bool = False):
    """Crops of a periodic device field into training inputs / targets (lbsg_gather, or
    lbsg_gather_noalloc when noalloc: no device allocation, at most
    LBSG_GATHER_NOALLOC_MAX_CROPS crops)."""
    yx = np.ascontiguousarray(yx, dtype=np.int32).reshape(-1, 2)
    k = yx.shape[0]
    if cond is None or cond.size == 0:
        c, nc = None, 0
    else:
        cond = np.ascontiguousarray(cond, dtype=np.float32).reshape(k, -1)
        c, nc = cond.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), cond.shape[1]
    name = "lbsg_gather_noalloc" if noalloc else "lbsg_gather"
    _check(getattr(_bind(), name)(ctypes.c_void_p(field_ptr), h, w, yx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  k, crop, c, nc, ctypes.c_void_p(x_ptr) if x_ptr else None,
                                  ctypes.c_void_p(y_ptr) if y_ptr else None, _stream_handle(stream)), name)
