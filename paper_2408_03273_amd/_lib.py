"""ctypes binding of libmpewald.so (the HIP library); argument marshalling only."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# MPEWALD_LIB names another build of the library (e.g. one with a sanitized host pass)
LIB_PATH = os.environ.get("MPEWALD_LIB") or os.path.join(_HERE, "libmpewald.so")

EWALD_OK = 0
EWALD_ERR_ARG = -1
EWALD_ERR_CUTOFF = -2
EWALD_ERR_CAPACITY = -3
EWALD_ERR_HIP = -4
EWALD_ERR_OOM = -5

EWALD_FP64 = 0
EWALD_FP32_REAL = 1
EWALD_FP32_RECIP = 2

EWALD_QMQM = 1
EWALD_PLAIN = 2
EWALD_CELL_LIST = 4
EWALD_PROFILE = 8
EWALD_PROFILE_HOT = 16
EWALD_NO_BACKGROUND = 32
EWALD_DETERMINISTIC = 64

EWALD_FWD = 0
EWALD_FWD_BWD = 1

STATUS_NAMES = {0: "EWALD_OK", -1: "EWALD_ERR_ARG", -2: "EWALD_ERR_CUTOFF", -3: "EWALD_ERR_CAPACITY",
                -4: "EWALD_ERR_HIP", -5: "EWALD_ERR_OOM"}

# every symbol the public header declares
EXPORTED = ("ewald_setup", "ewald_destroy", "ewald_set_box", "ewald_ctx_bytes", "ewald_forward", "ewald_backward",
            "ewald_moments_update", "ewald_suggest_params", "ewald_region_forward", "ewald_region_backward",
            "ewald_octupole_error", "ewald_batch", "ewald_autotune", "ewald_profile_report", "ewald_plan_describe", "ewald_last_error",
            "ewald_version", "ewald_fp64_probe", "ewald_octupole_error_noalloc")


class EwaldParams(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double * 3), ("alpha", ctypes.c_double), ("rcut", ctypes.c_double),
                ("kmax", ctypes.c_int * 3), ("precision", ctypes.c_int), ("flags", ctypes.c_int),
                ("max_qm", ctypes.c_int), ("max_mm", ctypes.c_int), ("max_frames", ctypes.c_int)]


class EwaldFrame(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double * 3), ("n_qm", ctypes.c_int), ("n_mm", ctypes.c_int),
                ("qm_offset", ctypes.c_int), ("mm_offset", ctypes.c_int)]


class EwaldError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    lib.ewald_setup.argtypes = [ctypes.POINTER(EwaldParams), ctypes.POINTER(vp)]
    lib.ewald_destroy.argtypes = [vp]
    lib.ewald_set_box.argtypes = [vp, ctypes.c_double * 3]
    lib.ewald_ctx_bytes.argtypes = [vp, ip, ip]
    lib.ewald_ctx_bytes.restype = ctypes.c_size_t
    lib.ewald_forward.argtypes = [vp, ip, vp, vp, vp, vp, ip, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.ewald_backward.argtypes = [vp, vp, ip, vp, vp, vp, vp, ip, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.ewald_suggest_params.argtypes = [ctypes.c_double * 3, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int * 3]
    lib.ewald_moments_update.argtypes = [vp, vp, ip, vp, vp, vp, vp, ip, vp, vp, vp, vp, vp]
    lib.ewald_batch.argtypes = [vp, ip, ctypes.POINTER(EwaldFrame), vp, vp, vp, vp, vp, vp, ip, vp, vp, vp, vp, vp,
                                vp, vp, vp, vp, vp, vp]
    dd = ctypes.c_double
    lib.ewald_region_forward.argtypes = [vp, ip, vp, vp, vp, vp, ip, vp, vp, vp, dd, dd, vp, vp, vp, vp, vp]
    lib.ewald_region_backward.argtypes = [vp, ip, vp, vp, vp, vp, ip, vp, vp, vp, dd, dd, vp, vp, vp, vp, vp, vp, vp,
                                          vp, vp, vp, vp]
    lib.ewald_octupole_error.argtypes = [vp, ip, vp, vp, ip, vp, vp, ip, dd, dd, dd, dd, vp, vp, vp]
    lib.ewald_octupole_error_noalloc.argtypes = [dp, ip, vp, vp, ip, vp, vp, ip, dd, dd, dd, dd,
                                                 vp, vp, vp]
    lib.ewald_autotune.argtypes = [vp, ip, ctypes.c_char_p]
    lib.ewald_profile_report.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.ewald_plan_describe.argtypes = [vp]
    lib.ewald_plan_describe.restype = ctypes.c_char_p
    lib.ewald_last_error.argtypes = []
    lib.ewald_last_error.restype = ctypes.c_char_p
    lib.ewald_version.argtypes = []
    lib.ewald_version.restype = ctypes.c_char_p
    lib.ewald_fp64_probe.argtypes = [ip, ip, ip, vp, dp, vp]
    lib.ewald_fp64_probe.restype = ip
    for name in ("ewald_setup", "ewald_destroy", "ewald_set_box", "ewald_forward", "ewald_backward",
                 "ewald_moments_update", "ewald_suggest_params", "ewald_region_forward", "ewald_region_backward",
                 "ewald_octupole_error", "ewald_octupole_error_noalloc", "ewald_batch", "ewald_autotune",
                 "ewald_profile_report"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != EWALD_OK:
        msg = load().ewald_last_error().decode(errors="replace")
        raise EwaldError(status, msg)
