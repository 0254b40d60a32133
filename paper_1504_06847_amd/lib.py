"""ctypes view of libmuffin.so (the C ABI declared in include/muffin.h).

Argument marshalling only: every step of the reconstruction runs in the
library's HIP kernels.  Loading fails loudly when the library is not built;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, byref, c_char_p, c_double, c_int, c_size_t,
                    c_void_p)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmuffin.so")

MUFFIN_OK = 0
MUFFIN_NOT_CONVERGED = 1
MUFFIN_EINVAL = -1
MUFFIN_EUNSUPPORTED = -2
MUFFIN_EWORKSPACE = -3
MUFFIN_EDEVICE = -4
MUFFIN_ENONFINITE = -5
MUFFIN_F32 = 0
MUFFIN_F64 = 1
MUFFIN_DIRAC = 0
MUFFIN_DCT2_ORTHO = 0
MUFFIN_CHEBYSHEV = 1
MUFFIN_SPECTRAL_DIRAC = 2
MUFFIN_MAX_SPECTRAL = 4
MUFFIN_MODE_MSE = 0
MUFFIN_MODE_VJP = 1
MUFFIN_MAX_BANDS = 256
MUFFIN_MAX_BATCH = 256
MUFFIN_NOALLOC_SCRATCH_MIB = 64

ERROR_NAMES = {
    MUFFIN_EINVAL: "MUFFIN_EINVAL", MUFFIN_EUNSUPPORTED: "MUFFIN_EUNSUPPORTED",
    MUFFIN_EWORKSPACE: "MUFFIN_EWORKSPACE", MUFFIN_EDEVICE: "MUFFIN_EDEVICE",
    MUFFIN_ENONFINITE: "MUFFIN_ENONFINITE",
}


class MuffinShape(Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("L", c_int), ("dtype", c_int)]


class MuffinParams(Structure):
    _fields_ = [("mu_eps", c_double), ("mu_s", c_double), ("mu_nu", c_double),
                ("rho_P", c_double), ("rho_T", c_double), ("rho_V", c_double),
                ("rho_S", c_double), ("n_s", c_int), ("spatial", c_int * 9),
                ("n_nu", c_int), ("spectral", c_int * 4), ("check_every", c_int),
                ("eps_abs", c_double), ("eps_rel", c_double)]


class MuffinReport(Structure):
    _fields_ = [("iters", c_int), ("converged", c_int), ("r_pri", c_double),
                ("r_dual", c_double), ("eps_pri", c_double), ("eps_dual", c_double),
                ("objective", c_double), ("E", c_double)]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# (name, restype, argtypes) for every entry point of include/muffin.h
SIGNATURES = [
    ("muffin_default_params", None, [POINTER(MuffinParams)]),
    ("muffin_workspace_bytes", c_size_t, [POINTER(MuffinShape), POINTER(MuffinParams)]),
    ("muffin_validate", c_int, [POINTER(MuffinShape), POINTER(MuffinParams)]),
    ("muffin_wavelet_filter", c_int, [c_int, POINTER(c_double)]),
    ("muffin_spectral_basis", c_int, [c_int, c_int, POINTER(c_double)]),
    ("muffin_setup", c_int, [POINTER(c_void_p), POINTER(MuffinShape), POINTER(MuffinParams),
                             c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("muffin_iterate", c_int, [c_void_p, c_int]),
    ("muffin_solve", c_int, [c_void_p, c_int, POINTER(MuffinReport)]),
    ("muffin_solve_adaptive", c_int, [c_void_p, c_int, c_double, c_double, POINTER(MuffinReport)]),
    ("muffin_get_params", c_int, [c_void_p, POINTER(MuffinParams)]),
    ("muffin_step_report", c_int, [c_void_p, POINTER(MuffinReport)]),
    ("muffin_get_x", c_int, [c_void_p, c_void_p]),
    ("muffin_get_p", c_int, [c_void_p, c_void_p]),
    ("muffin_grad", c_int, [c_void_p, c_int, c_int, c_void_p, c_int, POINTER(c_double),
                            POINTER(c_double)]),
    ("muffin_grad_params", c_int, [c_void_p, c_int, c_int, c_void_p, c_int, POINTER(c_double),
                                   POINTER(c_double)]),
    ("muffin_grad_dirty", c_int, [c_void_p, c_int, c_int, c_void_p, c_int, POINTER(c_double), c_void_p]),
    ("muffin_grad_record", c_int, [c_void_p, c_int, c_int, c_int]),
    ("muffin_grad_replay", c_int, [c_void_p, c_void_p, c_int, POINTER(c_double), POINTER(c_double), c_void_p]),
    ("muffin_grad_workspace_bytes", c_size_t, [c_void_p, c_int, c_int, c_int]),
    ("muffin_set_grad_workspace", c_int, [c_void_p, c_void_p, c_size_t]),
    ("muffin_grad_noalloc", c_int, [c_void_p, c_int, c_int, c_void_p, c_int, POINTER(c_double),
                                    POINTER(c_double)]),
    ("muffin_state_bytes", c_size_t, [c_void_p]),
    ("muffin_get_state", c_int, [c_void_p, c_void_p]),
    ("muffin_set_state", c_int, [c_void_p, c_void_p]),
    ("muffin_set_params", c_int, [c_void_p, POINTER(MuffinParams)]),
    ("muffin_reset", c_int, [c_void_p]),
    ("muffin_iterations", c_int, [c_void_p]),
    ("muffin_set_graph", c_int, [c_void_p, c_int]),
    ("muffin_autotune", c_int, [c_void_p, c_int, POINTER(c_int)]),
    ("muffin_set_schedule", c_int, [c_void_p, POINTER(c_int)]),
    ("muffin_get_schedule", c_int, [c_void_p, POINTER(c_int)]),
    ("muffin_fused_available", c_int, [c_void_p]),
    ("muffin_batch_workspace_bytes", c_size_t, [c_int, POINTER(MuffinShape), POINTER(MuffinParams)]),
    ("muffin_setup_batch", c_int, [POINTER(c_void_p), c_int, POINTER(MuffinShape), POINTER(MuffinParams),
                                   POINTER(c_void_p), POINTER(c_void_p), c_void_p, c_size_t, c_void_p]),
    ("muffin_batch_cube", c_void_p, [c_void_p, c_int]),
    ("muffin_batch_autotune", c_int, [c_void_p, c_int]),
    ("muffin_batch_launches", c_int, [c_void_p]),
    ("muffin_vis_workspace_bytes", c_size_t, [POINTER(MuffinShape), POINTER(MuffinParams)]),
    ("muffin_setup_vis", c_int, [POINTER(c_void_p), POINTER(MuffinShape), POINTER(MuffinParams), POINTER(c_int),
                                 POINTER(c_double), POINTER(c_double), c_int, c_void_p, c_size_t, c_void_p]),
    ("muffin_vis_cg_iters", c_int, [c_void_p]),
    ("muffin_profile", c_int, [c_void_p, c_int, POINTER(c_double), POINTER(c_char_p), c_int]),
    ("muffin_destroy", c_int, [c_void_p]),
    ("muffin_last_error", c_char_p, []),
]

_LIB = None


class MuffinError(RuntimeError):
    def __init__(self, code, where, message):
        self.code = code
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {message}")


def load(path: str | None = None):
    """Load libmuffin.so (built by ``python -m paper_1504_06847_amd.build``)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libmuffin.so is not built ({p}); run "
                           "`python -m paper_1504_06847_amd.build` first")
    lib = ctypes.CDLL(p)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _LIB = lib
    return lib


def last_error(lib=None) -> str:
    lib = lib or load()
    m = lib.muffin_last_error()
    return m.decode() if m else ""


def check(rc: int, where: str, lib=None) -> int:
    if rc < 0:
        raise MuffinError(rc, where, last_error(lib))
    return rc


def make_params(lib=None, **kw) -> MuffinParams:
    lib = lib or load()
    p = MuffinParams()
    lib.muffin_default_params(byref(p))
    for k, v in kw.items():
        if k == "spatial":
            for i, s in enumerate(v):
                p.spatial[i] = s
        elif k == "spectral":
            v = tuple(v) if isinstance(v, (tuple, list)) else (int(v),)
            p.n_nu = len(v)
            for i, s in enumerate(v):
                p.spectral[i] = s
        elif not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        else:
            setattr(p, k, v)
    return p
