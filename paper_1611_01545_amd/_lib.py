"""ctypes declarations of libpm's C ABI (include/pm.h).

Loads the in-tree libpm.so built by build.py. torch is imported first so that the
library binds to the HIP runtime torch already loaded (same SONAME), giving one
runtime, one device context and shared device pointers. There is no fallback: if the
library is missing, importing this module raises.
"""

from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must be loaded before libpm, see module docstring)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpm.so")

PM_FLOAT = 0
PM_COMPRESSED = 1

STATUS = {
    0: "PM_OK",
    1: "PM_ERR_ARG",
    2: "PM_ERR_SHAPE",
    3: "PM_ERR_NOMEM",
    4: "PM_ERR_DEVICE",
    5: "PM_ERR_CAPACITY",
    6: "PM_ERR_CORRUPT",
    7: "PM_ERR_RANGE",
}


class PmConfig(ctypes.Structure):
    _fields_ = [
        ("n_mesh", ctypes.c_int64),
        ("n_cell", ctypes.c_int64),
        ("brick", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("box", ctypes.c_double),
        ("G", ctypes.c_double),
        ("soft_cells", ctypes.c_double),
        ("kernel", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("r_split", ctypes.c_double),
    ]


class PmSizes(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "context_bytes", "step_mesh_bytes", "step_scratch_bytes", "vjp_scratch_bytes",
        "float_deposit_scratch_bytes", "compressed_species_bytes", "float_species_bytes")]


class PmSpecies(ctypes.Structure):
    _fields_ = [
        ("layout", ctypes.c_int32),
        ("widths", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("mass", ctypes.c_double),
        ("x", ctypes.c_void_p),
        ("v", ctypes.c_void_p),
        ("count", ctypes.c_void_p),
        ("pos", ctypes.c_void_p),
        ("vel", ctypes.c_void_p),
        ("esc", ctypes.c_void_p),
        ("cap_esc", ctypes.c_int64),
        ("hdr", ctypes.c_void_p),
    ]


# (name, argtypes) of every exported entry point declared in include/pm.h
P = ctypes.c_void_p
I64 = ctypes.c_int64
PS = ctypes.POINTER(PmSpecies)
EXPORTS = [
    ("pm_status_str", [ctypes.c_int]),
    ("pm_create", [ctypes.POINTER(PmConfig), P, ctypes.POINTER(P)]),
    ("pm_query_sizes", [ctypes.POINTER(PmConfig), I64, ctypes.c_int, ctypes.POINTER(PmSizes)]),
    ("pm_scratch_bytes", [P, ctypes.POINTER(I64)]),
    ("pm_destroy", [P]),
    ("pm_sync", [P]),
    ("pm_last_error_detail", [P, ctypes.POINTER(I64)]),
    ("pm_encode", [P, PS, PS, P]),
    ("pm_decode", [P, PS, PS]),
    ("pm_deposit", [P, PS, ctypes.c_int, P]),
    ("pm_force", [P, P, P, P]),
    ("pm_kick_drift", [P, PS, PS, ctypes.c_int, P, P, ctypes.c_double, ctypes.c_double]),
    ("pm_kick_drift_perm", [P, PS, PS, ctypes.c_int, P, P, ctypes.c_double,
                            ctypes.c_double, P]),
    ("pm_step", [P, PS, PS, ctypes.c_int, ctypes.c_double]),
    ("pm_step_vjp", [P, PS, ctypes.c_int, ctypes.c_double, P, P, P, P]),
    ("pm_loss_density_vjp", [P, PS, ctypes.c_int, P, P, P]),
    ("pm_pp_accel", [P, PS, ctypes.c_int, ctypes.c_double, P, P]),
    ("pm_step_pp", [P, PS, PS, ctypes.c_int, ctypes.c_double, ctypes.c_double, P]),
    ("pm_interp_accel", [P, PS, ctypes.c_int, P, P, ctypes.c_int]),
    ("pm_step_p3m", [P, P, PS, PS, ctypes.c_int, ctypes.c_double, ctypes.c_double, P]),
    ("pm_reduce", [P, PS, ctypes.c_int, P, P, P]),
    ("pm_reduce_noalloc", [P, PS, ctypes.c_int, P, P, P]),
    ("pm_pack", [P, PS, ctypes.c_int32, P, I64, P]),
    ("pm_pack_size", [P, PS, ctypes.POINTER(I64)]),
    ("pm_unpack", [P, P, I64, PS, ctypes.POINTER(ctypes.c_double),
                   ctypes.POINTER(ctypes.c_int32)]),
    ("pm_profile", [P, ctypes.c_int]),
    ("pm_profile_read", [P, P, P, ctypes.c_int]),
    ("pm_kernel_table", [P, P, I64]),
]


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"libpm.so not found at {path}: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` or "
            "`python paper_1611_01545_amd/build.py`")
    lib = ctypes.CDLL(path)
    for name, args in EXPORTS:
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "pm_status_str" else ctypes.c_int
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


class PMError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)}")


def check(code: int, where: str):
    if code != 0:
        raise PMError(code, where)
