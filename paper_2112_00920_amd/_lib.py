"""ctypes declarations of the C ABI in include/tdks.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdks.so")

TDKS_OK = 0
E_ARG, E_OOM, E_HIP, E_STATE, E_NUMERIC, E_UNSUPPORTED = -1, -2, -3, -4, -5, -6
FP64, FP32_MIXED = 0, 1
HXC_SCF, HXC_FROZEN, HXC_NONE = 0, 1, 2
PROP_TAYLOR, PROP_PC = 0, 1
HOST, DEVICE = 0, 1
PER_INSTANCE, PER_GROUP = 0, 1

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int_p = ctypes.POINTER(ctypes.c_int)

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Species(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double), ("w", ctypes.c_double), ("rc", ctypes.c_double),
                ("Rc", ctypes.c_double), ("Es", ctypes.c_double), ("Ep", ctypes.c_double)]


class InstanceDesc(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_double * 9),
        ("grid", ctypes.c_int * 3),
        ("n_atoms", ctypes.c_int),
        ("atom_frac", c_double_p),
        ("atom_species", c_int_p),
        ("n_species", ctypes.c_int),
        ("species", ctypes.POINTER(Species)),
        ("n_k", ctypes.c_int),
        ("k_frac", c_double_p),
        ("k_weight", c_double_p),
        ("n_bands", ctypes.c_int),
        ("occ", c_double_p),
        ("group", ctypes.c_int),
        ("v_hxc_frozen", c_double_p),
    ]


class TilingRule(ctypes.Structure):
    _fields_ = [
        ("grid", ctypes.c_int * 3),
        ("nonorth", ctypes.c_int),
        ("n_bands", ctypes.c_int),
        ("block_size", ctypes.c_int),
        ("waves_per_simd", ctypes.c_int),
        ("bands_per_group", ctypes.c_int),
        ("k_per_group", ctypes.c_int),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("dt", ctypes.c_double),
        ("taylor_order", ctypes.c_int),
        ("hxc_mode", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("alloc", ALLOC_FN),
        ("free", FREE_FN),
        ("alloc_user", ctypes.c_void_p),
        ("bands_per_group", ctypes.c_int),
        ("k_per_group", ctypes.c_int),
        ("block_size", ctypes.c_int),
        ("graph_steps", ctypes.c_int),
        ("waves_per_simd", ctypes.c_int),
        ("propagator", ctypes.c_int),
        ("norm_stride", ctypes.c_int),
        ("record_stride", ctypes.c_int),
        ("tiling_rules", ctypes.POINTER(TilingRule)),
        ("n_tiling_rules", ctypes.c_int),
    ]


SYMBOLS = {
    "tdks_default_options": (None, [ctypes.POINTER(Options)]),
    "tdks_create": (ctypes.c_int, [ctypes.POINTER(InstanceDesc), ctypes.c_int, ctypes.POINTER(Options),
                                   ctypes.POINTER(ctypes.c_void_p)]),
    "tdks_destroy": (None, [ctypes.c_void_p]),
    "tdks_last_error": (ctypes.c_char_p, []),
    "tdks_load_orbitals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]),
    "tdks_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, c_double_p]),
    "tdks_steps_done": (ctypes.c_int, [ctypes.c_void_p]),
    "tdks_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_ulonglong)]),
    "tdks_step_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "tdks_ground_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_void_p]),
    "tdks_current": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, c_double_p, ctypes.c_size_t,
                                    ctypes.POINTER(ctypes.c_size_t)]),
    "tdks_current_pre": (ctypes.c_int, [ctypes.c_void_p, c_double_p]),
    "tdks_current_at": (ctypes.c_int, [ctypes.c_void_p, c_double_p, c_double_p]),
    "tdks_density": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, c_double_p]),
    "tdks_vhxc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, c_double_p]),
    "tdks_vloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, c_double_p]),
    "tdks_get_orbitals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]),
    "tdks_norms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, c_double_p]),
    "tdks_apply_h": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                    c_double_p, ctypes.c_int]),
    "tdks_tiling": (ctypes.c_int, [ctypes.c_void_p, c_int_p, c_int_p, c_int_p, c_int_p, c_int_p, c_int_p]),
    "tdks_time_kernels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, c_double_p, c_double_p]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads libtdks.so; raises ImportError (never falls back) when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libtdks.so not found at {path}; build it with "
                          "`python -m paper_2112_00920_amd.build`")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7); importing
    # torch first makes this library bind to that one, so that a process holds one HIP
    # runtime whose device memory and streams both sides share
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    for name, (res, args) in SYMBOLS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class TdksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tdks error {code}: {msg}")
        self.code = code


def check(rc: int):
    if rc != TDKS_OK:
        raise TdksError(rc, load().tdks_last_error().decode(errors="replace"))
