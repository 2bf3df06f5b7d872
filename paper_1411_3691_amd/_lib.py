"""ctypes binding of libmhc.so (argument marshalling only).

torch is imported before the library is opened: torch's HIP runtime and
libmhc's then resolve to the same ``libamdhip64.so.7`` in the process, so
device pointers and streams created by torch are valid in libmhc.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime that libmhc shares)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmhc.so")

MHC_OK = 0
STATUS_NAMES = {
    0: "MHC_OK", -1: "MHC_E_ARG", -2: "MHC_E_TERM", -3: "MHC_E_SHAPE",
    -4: "MHC_E_DEVICE", -5: "MHC_E_OOM", -6: "MHC_E_STATE",
    -7: "MHC_E_UNSUPPORTED",
}
GREEDY_R1 = 1
GREEDY_R2 = 2
PLAIN_LU = 0
UPDATE_TREE = 1
UPDATE_TREE2 = 2
PLAIN_LU_UNPIVOTED = 3
UPDATE_TREE_UNPIVOTED = 4
PLAIN_LU_THRESHOLD = 5
UPDATE_TREE_THRESHOLD = 6
UPDATE_TREE_AGG = 7
TREE_NO_SHARING = 0x100
TREE_PRUNE = 0x200
TREE_SET_EDGES = 0x400
SCHED_AUTO = 0
SCHED_LANE = 1
SCHED_GROUP = 2


class Schedule(ctypes.Structure):
    """mhc_schedule: kernel family, persistent workgroups per CU, items per
    tile (0 = the library's choice)."""
    _fields_ = [("kernel", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("items_per_tile", ctypes.c_int32)]


# Every function the C header declares, with its ctypes signature.
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PD = ctypes.c_void_p
SIGNATURES = {
    "mhc_last_error": (ctypes.c_char_p, []),
    "mhc_version": (_I32, []),
    "mhc_terms_create": (_I32, [_I32, _I32, _PI32, _PI32, _I32, ctypes.POINTER(_P)]),
    "mhc_terms_destroy": (None, [_P]),
    "mhc_terms_shape": (_I32, [_P, _PI32, _PI32, _PI32]),
    "mhc_tree_build": (_I32, [_P, _I32, ctypes.POINTER(_P)]),
    "mhc_tree_export": (_I32, [_P, _PI32, _PI32, _PI32, _PI32, _PI32]),
    "mhc_tree_stats": (_I32, [_P, _PI32, _PI32, _PI32]),
    "mhc_tree_groups": (_I32, [_P, _PI32, _PI32, _PI32, _PI32, _PI32]),
    "mhc_tree_children": (_I32, [_P, _PI32, _PI32]),
    "mhc_tree_destroy": (None, [_P]),
    "mhc_plan_create": (_I32, [_P, _P, _P, ctypes.POINTER(_P)]),
    "mhc_plan_destroy": (None, [_P]),
    "mhc_contract": (_I32, [_P, _I32, _I32, _P, _PD, _PD, _P, _PD, _P, _P, _I64, _P]),
    "mhc_contract_noalloc": (_I32, [_P, _I32, _I32, _P, _PD, _PD, _P, _PD, _P]),
    "mhc_contract_backward": (_I32, [_P, _I32, _I32, _P, _PD, _PD, _P, _P, _PD, _PD, _P]),
    "mhc_plan_status": (_I32, [_P, _PI64, _PI64]),
    "mhc_plan_attach_sink_tree": (_I32, [_P, _P, _P]),
    "mhc_batch_create": (_I32, [ctypes.POINTER(_P), _PI32, _I32, _I32, ctypes.POINTER(Schedule),
                                ctypes.POINTER(_P)]),
    "mhc_batch_run": (_I32, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                             ctypes.POINTER(_P), ctypes.POINTER(_P), _P]),
    "mhc_batch_info": (_I32, [_P, _PI32, _PI32, _PI64]),
    "mhc_batch_destroy": (None, [_P]),
    "mhc_probe_fma64": (_I32, [_PD, _I32, _I32, _P]),
    "mhc_probe_mfma64": (_I32, [_PD, _I32, _I32, _I32, _P]),
}


class MhcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1411_3691_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != MHC_OK:
        raise MhcError(status, lib().mhc_last_error().decode())
