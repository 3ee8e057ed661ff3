"""Thin ctypes binding of liblbch (include/lbch.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels.  PyTorch is
imported first so that the process holds one HIP runtime (the library links
against the same soname); torch is used only to hand device pointers and
streams to the library.  If the library is missing this module raises: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # one HIP runtime per process: torch's, loaded before the library
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbch.so")

OK, E_INVALID, E_UNSUPPORTED, E_OOM, E_DEVICE, E_NONFINITE, E_STATE = 0, -1, -2, -3, -4, -5, -6
D2Q9, D3Q15 = 0, 1
FP64, FP32 = 0, 1
BC_PERIODIC = 0
REG_NONE, REG_LINEAR, REG_WILLMORE = 0, 1, 2
Q_DERIVED, Q_LITERAL = 0, 1
COLLISION_MRT, COLLISION_SRT, COLLISION_TRT = 0, 1, 2
ABI_VERSION = 2


class LbchError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func} -> {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("lattice", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("boundary", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("mobility", ctypes.c_double),
        ("s", ctypes.c_double * 9),
        ("kappa", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("aniso_m", ctypes.c_int32),
        ("regularization", ctypes.c_int32),
        ("aniso_theta0", ctypes.c_double),
        ("eps_reg", ctypes.c_double),
        ("q_form", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("grad_floor", ctypes.c_double),
    ]


_SIGNATURES = {
    "lbch_abi_version": (ctypes.c_int32, []),
    "lbch_last_error": (ctypes.c_char_p, []),
    "lbch_params_default": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "lbch_params_from_sigma_width": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_double, ctypes.c_double]),
    "lbch_params_validate": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "lbch_relaxation_rates": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_double)]),
    "lbch_params_set_collision": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_double]),
    "lbch_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "lbch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "lbch_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64]),
    "lbch_init_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64]),
    "lbch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "lbch_step_extrapolated": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "lbch_get_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "lbch_synchronize": (ctypes.c_int, [ctypes.c_void_p]),
    "lbch_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "lbch_free_energy": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "lbch_phi_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "lbch_state_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "lbch_save_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "lbch_load_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "lbch_set_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "lbch_get_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "lbch_set_row_loader": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "lbch_set_time_blocking": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "lbch_get_time_blocking": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "lbch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "lbch_batch_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "lbch_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "lbch_batch_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.c_int64]),
    "lbch_batch_init_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                              ctypes.c_int64]),
    "lbch_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "lbch_batch_get_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "lbch_batch_synchronize": (ctypes.c_int, [ctypes.c_void_p]),
    "lbch_batch_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]),
    "lbch_batch_free_energy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double)]),
    "lbch_batch_phi_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32]),
    "lbch_batch_set_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "lbch_batch_get_tiling": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int32)] * 4),
    "lbch_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "lbch_batch_nodes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "lbch_batch_set_time_blocking": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "lbch_batch_get_time_blocking": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "lbch_diag_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Loads liblbch.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2501_03759_amd.build; "
                               "there is no CPU fallback")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(status: int, func: str):
    if status != OK:
        raise LbchError(status, func, lib().lbch_last_error().decode())


def _dp(x):
    return ctypes.cast(x, ctypes.POINTER(ctypes.c_double)) if x is not None else None


def default_params(**overrides) -> Params:
    """Eq 39 defaults, then keyword overrides (s may be a 9-sequence)."""
    p = Params()
    _check(lib().lbch_params_default(ctypes.byref(p)), "lbch_params_default")
    sigma_width = overrides.pop("sigma_width", None)
    if sigma_width is not None:
        _check(lib().lbch_params_from_sigma_width(ctypes.byref(p), *sigma_width), "lbch_params_from_sigma_width")
    for k, v in overrides.items():
        if k == "s":
            for i, sv in enumerate(v):
                p.s[i] = sv
        else:
            setattr(p, k, v)
    return p


def validate(p: Params) -> int:
    return lib().lbch_params_validate(ctypes.byref(p))


def set_collision(p: Params, model: int, magic: float = 0.25) -> Params:
    """Sets the free rates of p for MRT, SRT or TRT (lbch_params_set_collision); returns p."""
    _check(lib().lbch_params_set_collision(ctypes.byref(p), model, magic), "lbch_params_set_collision")
    return p


def relaxation_rates(p: Params) -> np.ndarray:
    out = (ctypes.c_double * 9)()
    _check(lib().lbch_relaxation_rates(ctypes.byref(p), out), "lbch_relaxation_rates")
    return np.array(out[:])


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        return ctypes.c_void_p(None)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)      # torch.cuda.Stream


class Sim:
    """One periodic grid (lbch_sim)."""

    def __init__(self, params: Params, stream=None):
        self.params = params
        self._h = ctypes.c_void_p()
        _check(lib().lbch_create(ctypes.byref(params), _stream_handle(stream), ctypes.byref(self._h)), "lbch_create")
        self.nx, self.ny, self.nz = params.nx, params.ny, params.nz
        self.shape = (params.nz, params.ny, params.nx) if params.lattice == D3Q15 else (params.ny, params.nx)

    def close(self):
        if self._h:
            lib().lbch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def init(self, phi0: np.ndarray):
        a = np.ascontiguousarray(phi0, dtype=np.float64)
        _check(lib().lbch_init(self._h, _dp(a.ctypes.data), a.size), "lbch_init")

    def init_device(self, ptr: int, dtype: int, n: int):
        _check(lib().lbch_init_device(self._h, ctypes.c_void_p(ptr), dtype, n), "lbch_init_device")

    def step(self, n: int = 1):
        _check(lib().lbch_step(self._h, int(n)), "lbch_step")

    def step_extrapolated(self, ext: float):
        """Two steps storing f_{n+2} + ext (f_{n+2} - f_n) (lbch_step_extrapolated)."""
        _check(lib().lbch_step_extrapolated(self._h, float(ext)), "lbch_step_extrapolated")

    @property
    def nstep(self) -> int:
        v = ctypes.c_int64()
        _check(lib().lbch_get_step(self._h, ctypes.byref(v)), "lbch_get_step")
        return v.value

    def synchronize(self):
        _check(lib().lbch_synchronize(self._h), "lbch_synchronize")

    def moments(self, want_phi: bool = True, check: bool = True):
        phi = np.empty(self.shape, dtype=np.float64) if want_phi else None
        mass, lo, hi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = lib().lbch_moments(self._h, _dp(phi.ctypes.data) if want_phi else None, ctypes.byref(mass),
                                ctypes.byref(lo), ctypes.byref(hi))
        if check:
            _check(st, "lbch_moments")
        return phi, mass.value, lo.value, hi.value

    def phi(self) -> np.ndarray:
        return self.moments(True)[0]

    def free_energy(self):
        e = ctypes.c_double()
        terms = (ctypes.c_double * 4)()
        _check(lib().lbch_free_energy(self._h, ctypes.byref(e), terms), "lbch_free_energy")
        return e.value, list(terms)

    def phi_device(self, ptr: int, dtype: int):
        _check(lib().lbch_phi_device(self._h, ctypes.c_void_p(ptr), dtype), "lbch_phi_device")

    def state_bytes(self) -> int:
        v = ctypes.c_int64()
        _check(lib().lbch_state_bytes(self._h, ctypes.byref(v)), "lbch_state_bytes")
        return v.value

    def save_state(self) -> bytes:
        buf = ctypes.create_string_buffer(self.state_bytes())
        _check(lib().lbch_save_state(self._h, buf, 0), "lbch_save_state")
        return buf.raw

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().lbch_load_state(self._h, buf, 0), "lbch_load_state")

    def set_tiling(self, block_threads: int, rows_per_block: int):
        _check(lib().lbch_set_tiling(self._h, block_threads, rows_per_block), "lbch_set_tiling")

    def autotune(self, steps_per_trial: int = 5):
        """Picks the fastest launch shape for this grid; returns (block_threads, rows, ms_per_step)."""
        a, r, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().lbch_autotune(self._h, steps_per_trial, ctypes.byref(a), ctypes.byref(r), ctypes.byref(ms)),
               "lbch_autotune")
        return a.value, r.value, ms.value

    def set_row_loader(self, mode: int):
        _check(lib().lbch_set_row_loader(self._h, mode), "lbch_set_row_loader")

    def set_time_blocking(self, depth: int):
        """Time steps per kernel launch (1 or 2); resets the tiling to that depth's default."""
        _check(lib().lbch_set_time_blocking(self._h, depth), "lbch_set_time_blocking")

    def time_blocking(self) -> int:
        d = ctypes.c_int32()
        _check(lib().lbch_get_time_blocking(self._h, ctypes.byref(d)), "lbch_get_time_blocking")
        return d.value

    def tiling(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lbch_get_tiling(self._h, ctypes.byref(a), ctypes.byref(b)), "lbch_get_tiling")
        return a.value, b.value


def diag_copy(src_ptr: int, dst_ptr: int, nbytes: int, stream=None):
    """Plain streaming copy (measurement helper of include/lbch_diag.h)."""
    _check(lib().lbch_diag_copy(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), nbytes,
                                _stream_handle(stream)), "lbch_diag_copy")


class Batch:
    """An ensemble of independent periodic grids advanced together (lbch_batch)."""

    def __init__(self, members, stream=None):
        arr = (Params * len(members))(*members)
        self._h = ctypes.c_void_p()
        _check(lib().lbch_batch_create(arr, len(members), _stream_handle(stream), ctypes.byref(self._h)),
               "lbch_batch_create")
        self.shapes = [(m.ny, m.nx) for m in members]

    def close(self):
        if self._h:
            lib().lbch_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __len__(self):
        return len(self.shapes)

    def init(self, member: int, phi0: np.ndarray):
        a = np.ascontiguousarray(phi0, dtype=np.float64)
        _check(lib().lbch_batch_init(self._h, member, _dp(a.ctypes.data), a.size), "lbch_batch_init")

    def init_device(self, member: int, ptr: int, dtype: int, n: int):
        _check(lib().lbch_batch_init_device(self._h, member, ctypes.c_void_p(ptr), dtype, n), "lbch_batch_init_device")

    def step(self, n: int = 1):
        _check(lib().lbch_batch_step(self._h, int(n)), "lbch_batch_step")

    @property
    def nstep(self) -> int:
        v = ctypes.c_int64()
        _check(lib().lbch_batch_get_step(self._h, ctypes.byref(v)), "lbch_batch_get_step")
        return v.value

    def synchronize(self):
        _check(lib().lbch_batch_synchronize(self._h), "lbch_batch_synchronize")

    def moments(self, member: int, want_phi: bool = True):
        ny, nx = self.shapes[member]
        phi = np.empty((ny, nx), dtype=np.float64) if want_phi else None
        mass, lo, hi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().lbch_batch_moments(self._h, member, _dp(phi.ctypes.data) if want_phi else None,
                                        ctypes.byref(mass), ctypes.byref(lo), ctypes.byref(hi)), "lbch_batch_moments")
        return phi, mass.value, lo.value, hi.value

    def phi(self, member: int) -> np.ndarray:
        return self.moments(member)[0]

    def free_energy(self, member: int):
        e = ctypes.c_double()
        terms = (ctypes.c_double * 4)()
        _check(lib().lbch_batch_free_energy(self._h, member, ctypes.byref(e), terms), "lbch_batch_free_energy")
        return e.value, list(terms)

    def phi_device(self, member: int, ptr: int, dtype: int):
        _check(lib().lbch_batch_phi_device(self._h, member, ctypes.c_void_p(ptr), dtype), "lbch_batch_phi_device")

    def set_tiling(self, block_threads: int, rows_per_block: int = 0, persistent_blocks: int = 0):
        _check(lib().lbch_batch_set_tiling(self._h, block_threads, rows_per_block, persistent_blocks),
               "lbch_batch_set_tiling")

    def tiling(self):
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().lbch_batch_get_tiling(self._h, *[ctypes.byref(x) for x in v]), "lbch_batch_get_tiling")
        return tuple(x.value for x in v)

    def autotune(self, steps_per_trial: int = 3):
        a, r, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().lbch_batch_autotune(self._h, steps_per_trial, ctypes.byref(a), ctypes.byref(r),
                                         ctypes.byref(ms)), "lbch_batch_autotune")
        return a.value, r.value, ms.value

    def set_time_blocking(self, depth: int):
        _check(lib().lbch_batch_set_time_blocking(self._h, depth), "lbch_batch_set_time_blocking")

    def time_blocking(self) -> int:
        d = ctypes.c_int32()
        _check(lib().lbch_batch_get_time_blocking(self._h, ctypes.byref(d)), "lbch_batch_get_time_blocking")
        return d.value

    @property
    def nodes(self) -> int:
        v = ctypes.c_int64()
        _check(lib().lbch_batch_nodes(self._h, ctypes.byref(v)), "lbch_batch_nodes")
        return v.value


class HybridOpts(ctypes.Structure):
    _fields_ = [("jump", ctypes.c_int32), ("correct_steps", ctypes.c_int32), ("tol_energy", ctypes.c_double),
                ("windows", ctypes.c_int32), ("window_interior", ctypes.c_int32), ("window_margin", ctypes.c_int32),
                ("tol_window", ctypes.c_double), ("check_every", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("ncond", ctypes.c_int32), ("cond", ctypes.c_float * 8), ("dry_run", ctypes.c_int32),
                ("extrapolate", ctypes.c_int32), ("inner_steps", ctypes.c_int32), ("inner_jump", ctypes.c_int32)]


class HybridStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int64), ("accepted", ctypes.c_int64), ("rejected_energy", ctypes.c_int64),
                ("rejected_window", ctypes.c_int64), ("plain_steps", ctypes.c_int64),
                ("max_window_err", ctypes.c_double), ("last_energy", ctypes.c_double),
                ("ms_surrogate", ctypes.c_double), ("ms_correct", ctypes.c_double), ("ms_checks", ctypes.c_double),
                ("ms_plain", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def hybrid_opts(**kw) -> HybridOpts:
    L = lib()
    L.lbch_hybrid_default_opts.restype = ctypes.c_int
    L.lbch_hybrid_default_opts.argtypes = [ctypes.POINTER(HybridOpts)]
    o = HybridOpts()
    _check(L.lbch_hybrid_default_opts(ctypes.byref(o)), "lbch_hybrid_default_opts")
    cond = kw.pop("cond", None)
    if cond is not None:
        o.ncond = len(cond)
        for i, v in enumerate(cond):
            o.cond[i] = v
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def hybrid_advance(sim: Sim, net, opts: HybridOpts, nsteps: int) -> HybridStats:
    """Surrogate-jump / lattice Boltzmann correction schedule (include/lbch_hybrid.h)."""
    L = lib()
    L.lbch_hybrid_advance.restype = ctypes.c_int
    L.lbch_hybrid_advance.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(HybridOpts), ctypes.c_int64,
                                      ctypes.POINTER(HybridStats)]
    st = HybridStats()
    _check(L.lbch_hybrid_advance(sim.handle, net._h if net is not None else None, ctypes.byref(opts), nsteps,
                                 ctypes.byref(st)), "lbch_hybrid_advance")
    return st


def extrapolate(base_ptr: int, phi_t_ptr: int, phi_t1_ptr: int, k: float, n: int, out_ptr: int, stream=None):
    """out = base + k (phi_t1 - phi_t) on FP32 device arrays (lbch_extrapolate)."""
    L = lib()
    L.lbch_extrapolate.restype = ctypes.c_int
    L.lbch_extrapolate.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_void_p]
    _check(L.lbch_extrapolate(ctypes.c_void_p(base_ptr), ctypes.c_void_p(phi_t_ptr), ctypes.c_void_p(phi_t1_ptr), k, n,
                              ctypes.c_void_p(out_ptr), _stream_handle(stream)), "lbch_extrapolate")

