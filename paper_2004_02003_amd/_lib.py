"""ctypes loader of ``libbto.so`` (argument marshalling only).

Every computation of the path runs in the HIP kernels of the library; when the
library is missing this module raises instead of falling back to anything.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# BTO_LIB_PATH may point at another build of the same library (e.g. an
# instrumented one); there is no fallback when the file is missing.
LIB_PATH = os.environ.get("BTO_LIB_PATH") or os.path.join(HERE, "libbto.so")

BTO_OK, BTO_EINVAL, BTO_ENOMEM, BTO_EHIP, BTO_ESTATE, BTO_ERANGE = 0, -1, -2, -3, -4, -5
BTO_F32, BTO_F16, BTO_BF16 = 0, 1, 2
BTO_TIME_LINEAR, BTO_TIME_FROZEN = 0, 1
BTO_RECORD_EXIT = 2
BTO_RECORD_CKPT = 1 << 4
BTO_SAMPLE_FP64 = 1 << 5
BTO_VALID, BTO_TERMINATED, BTO_INVALID = 0, 1, 2
BTO_ADJ_DROPPED, BTO_ADJ_DROPPED_PARTIAL = 3, 4

EXPORTED = [
    "bto_create", "bto_destroy", "bto_last_error", "bto_seed", "bto_seed_explicit",
    "bto_advect_interval", "bto_flowmap_out", "bto_stats", "bto_adjoint_interval", "bto_ftle",
    "bto_set_tuning", "bto_get_tuning", "bto_exit_points", "bto_place_block", "bto_reconstruct_lattice",
    "bto_flowmap_error", "bto_flowmap_error_static", "bto_adjoint_segment", "bto_touched_points",
]

_ERRNAMES = {BTO_EINVAL: "BTO_EINVAL", BTO_ENOMEM: "BTO_ENOMEM", BTO_EHIP: "BTO_EHIP",
             BTO_ESTATE: "BTO_ESTATE", BTO_ERANGE: "BTO_ERANGE"}


class BTOError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Block(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("origin", ctypes.c_double * 3),
                ("spacing", ctypes.c_double * 3)]


class Tuning(ctypes.Structure):
    _fields_ = [("steps_per_launch", ctypes.c_int32), ("rebin_every", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("lanes_per_particle", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("tiles", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("n_seeds", ctypes.c_int64), ("n_live", ctypes.c_int64),
                ("particle_steps", ctypes.c_int64), ("steps_done", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2004_02003_amd/build.py "
                          "(there is no fallback path)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.bto_create.argtypes = [ctypes.POINTER(Block), i64, i32, ctypes.POINTER(vp)]
    L.bto_destroy.argtypes = [vp]
    L.bto_last_error.argtypes = [vp]
    L.bto_last_error.restype = ctypes.c_char_p
    L.bto_seed.argtypes = [vp, i32, vp, ctypes.POINTER(i64), vp]
    L.bto_seed_explicit.argtypes = [vp, vp, i64, vp]
    L.bto_advect_interval.argtypes = [vp, vp, vp, i32, i32, i32, vp]
    L.bto_flowmap_out.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(i64), vp]
    L.bto_exit_points.argtypes = [vp, vp, vp]
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.bto_place_block.argtypes = [i32p, i32p, i32p, ctypes.POINTER(ctypes.c_double), vp, vp, vp, vp, vp]
    L.bto_reconstruct_lattice.argtypes = [i32p, vp, vp, vp, vp]
    L.bto_flowmap_error.argtypes = [ctypes.c_int64, vp, vp, vp, vp, ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_double), vp]
    L.bto_flowmap_error_static.argtypes = L.bto_flowmap_error.argtypes
    L.bto_stats.argtypes = [vp, ctypes.POINTER(Stats), vp]
    L.bto_adjoint_interval.argtypes = [vp, vp, vp, i32, i32, i32, vp, i32, vp, vp, vp, i32, vp]
    L.bto_adjoint_segment.argtypes = [vp, i32, vp, vp, i32, i32, vp, i32, vp, vp, vp, vp]
    L.bto_ftle.argtypes = [vp, vp, i64, ctypes.c_double, vp, vp]
    L.bto_touched_points.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp]
    L.bto_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.bto_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    for fn in EXPORTED:
        if fn != "bto_last_error":
            getattr(L, fn).restype = ctypes.c_int
    _lib = L
    return L
