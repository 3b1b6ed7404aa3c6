"""ctypes binding of libmiugks.so (argument marshalling only).

Every function of include/miugks.h is exposed under the same name.  The
library is loaded from this package directory; importing this module on a
machine where it is missing raises ImportError (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmiugks.so")

OK, EINVAL, ENOMEM, EDEVICE, EDIVERGED, ENOTCONVERGED, ESTATE = range(7)
FACE_INTERIOR, FACE_WALL, FACE_FARFIELD, FACE_OUTFLOW, FACE_SYMMETRY = range(5)
FP64, FP32F = 0, 1
QUAD_TRAPEZOID, QUAD_SIMPSON38, QUAD_GAUSS_HERMITE = range(3)
CYCLE_F = -1
LOAD_PRESSURE, LOAD_SHEAR, LOAD_HEAT = range(3)

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_ip = ctypes.POINTER(ctypes.c_int)


class MeshDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("n_levels", ctypes.c_int),
                ("x", _dp), ("y", _dp), ("face_type_x", _u8p), ("face_type_y", _u8p),
                ("wall_x", _dp), ("wall_y", _dp), ("solid", _u8p)]


class VGridDesc(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_int), ("nv", ctypes.c_int), ("u", _dp), ("v", _dp),
                ("wu", _dp), ("wv", _dp)]


class GasDesc(ctypes.Structure):
    _fields_ = [("K_int", ctypes.c_int), ("Pr", ctypes.c_double), ("omega", ctypes.c_double),
                ("Kn", ctypes.c_double), ("rho_inf", ctypes.c_double), ("U_inf", ctypes.c_double),
                ("V_inf", ctypes.c_double), ("T_inf", ctypes.c_double)]


class SolverDesc(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("nu_coarse", ctypes.c_int), ("cfl", ctypes.c_double),
                ("dtn_growth", ctypes.c_double), ("mass_renorm", ctypes.c_int), ("fas_levels", ctypes.c_int),
                ("nu_coarse_cs", ctypes.c_int), ("cycle_gamma", ctypes.c_int),
                ("cycle_gamma_cs", ctypes.c_int), ("dtn_max", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_SIGS = {
    "miugks_set_allocator": (ctypes.c_int, [ALLOC_FN, FREE_FN, ctypes.c_void_p]),
    "miugks_quadrature": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]),
    "miugks_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(MeshDesc),
                                     ctypes.POINTER(VGridDesc), ctypes.POINTER(GasDesc),
                                     ctypes.POINTER(SolverDesc), ctypes.c_void_p]),
    "miugks_destroy": (None, [ctypes.c_void_p]),
    "miugks_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "miugks_init_macro": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp, _dp]),
    "miugks_iterate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _ip, _dp]),
    "miugks_fmg": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _ip]),
    "miugks_explicit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _dp]),
    "miugks_get_macro": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp]),
    "miugks_get_f": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "miugks_get_f_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "miugks_set_f": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "miugks_wall_list": (ctypes.c_int, [ctypes.c_void_p, _ip, _ip, _ip]),
    "miugks_wall_loads": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp, _dp, _ip]),
    "miugks_objective": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _ip, ctypes.c_int, _dp]),
    "miugks_set_wall_T": (ctypes.c_int, [ctypes.c_void_p, _ip, _dp, ctypes.c_int]),
    "miugks_residual_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                               ctypes.c_int]),
    "miugks_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _ip, ctypes.c_int, _ip, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_int, _dp, _ip, _dp]),
    "miugks_adjoint_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _ip, ctypes.c_int, _ip, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _ip, _dp]),
    "miugks_residual": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp]),
    "miugks_get_div": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "miugks_predict": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp]),
    "miugks_micro_residual": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_void_p, _dp, ctypes.c_int,
                                             ctypes.c_int]),
    "miugks_correct": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _dp, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.c_int]),
    "miugks_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "miugks_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p), _ip, _dp,
                                     _dp]),
    "miugks_sizes": (ctypes.c_int, [ctypes.c_void_p, _ip, _ip, _ip, _ip]),
}

EXPORTS = tuple(_SIGS)


def _load():
    # Bind to the HIP runtime torch already carries, so that one process holds
    # a single runtime (a second copy would not see the device, and device
    # pointers are shared with torch tensors).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__; __graft_entry__.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class MiugksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"miugks error {code}: {msg}")
        self.code = code


def dptr(a: np.ndarray):
    return a.ctypes.data_as(_dp) if a is not None else None


def iptr(a: np.ndarray):
    return a.ctypes.data_as(_ip) if a is not None else None


def u8ptr(a: np.ndarray):
    return a.ctypes.data_as(_u8p) if a is not None else None


def quadrature(kind: int, n: int, lo: float = 0.0, hi: float = 0.0):
    """Nodes and weights of the library's 1-D rule."""
    x = np.zeros(n)
    w = np.zeros(n)
    rc = lib.miugks_quadrature(kind, n, lo, hi, dptr(x), dptr(w))
    if rc:
        raise MiugksError(rc, f"quadrature kind={kind} n={n}")
    return x, w
