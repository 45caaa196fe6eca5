"""ctypes front end of the turbulence evaluator in ``turb.c`` (input generator)."""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "turb.c")
_LIB = os.path.join(_HERE, "libbto_inputs.so")
_DEV_SRC = os.path.join(_HERE, "turb_dev.hip")
_DEV_LIB = os.path.join(_HERE, "libbto_inputs_dev.so")
_DT_CODE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}


def build(force: bool = True) -> str:
    """Compile turb.c (host) and turb_dev.hip (gfx950) next to them."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    if force or not os.path.exists(_DEV_LIB):
        arch = os.environ.get("BTO_OFFLOAD_ARCH", "gfx950")
        cmd = ["hipcc", f"--offload-arch={arch}", "-O3", "-ffp-contract=off", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-o", _DEV_LIB + ".tmp", _DEV_SRC]
        subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
        os.replace(_DEV_LIB + ".tmp", _DEV_LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.turb_grid.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        L.turb_point.argtypes = [ctypes.c_void_p] + [ctypes.c_int32] * 4 + [ctypes.c_void_p]
        L.turb_store_round.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32]
        _lib = L
    return _lib


class _Tables(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("M", ctypes.c_int32), ("C", ctypes.c_int32)] + \
        [(nm, ctypes.c_void_p) for nm in ("exr", "exi", "eyr", "eyi", "ezr", "ezi", "pr", "pi", "amp")] + \
        [("dtype", ctypes.c_int32)]


class TurbEvaluator:
    """Holds the per-axis and per-cycle tables of one turbulence series."""

    def __init__(self, n, modes, times):
        nx, ny, nz = n
        self.n = (nx, ny, nz)
        self.modes = modes
        k = modes.kvec
        ax = [np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64),
              np.arange(nz, dtype=np.float64)]
        arrs = {}
        for d, nm in enumerate("xyz"):
            ang = k[:, d][:, None] * ax[d][None, :]
            arrs["e%sr" % nm] = np.ascontiguousarray(np.cos(ang))
            arrs["e%si" % nm] = np.ascontiguousarray(np.sin(ang))
        psi = modes.omega[None, :] * np.asarray(times)[:, None] + modes.phase[None, :]
        arrs["pr"] = np.ascontiguousarray(np.cos(psi))
        arrs["pi"] = np.ascontiguousarray(np.sin(psi))
        arrs["amp"] = np.ascontiguousarray(modes.amp, dtype=np.float64)
        self.arrs = arrs
        self.M = int(k.shape[0])
        self.C = int(len(times))
        self._tabs = {}

    def tables(self, dtype: str = "f64") -> _Tables:
        """The C table struct (kept alive by this object) for storage ``dtype``."""
        if dtype not in self._tabs:
            t = _Tables()
            t.nx, t.ny, t.nz = self.n
            t.M, t.C = self.M, self.C
            for nm, a in self.arrs.items():
                setattr(t, nm, a.ctypes.data)
            t.dtype = _DT_CODE[dtype]
            self._tabs[dtype] = t
        return self._tabs[dtype]

    def grid_f64(self, c: int) -> np.ndarray:
        nx, ny, nz = self.n
        out = np.empty((nz, ny, nx, 3), dtype=np.float64)
        lib().turb_grid(ctypes.byref(self.tables()), int(c), out.ctypes.data)
        return out

    def point(self, c: int, i: int, j: int, k: int) -> np.ndarray:
        out = np.empty(3, dtype=np.float64)
        lib().turb_point(ctypes.byref(self.tables()), int(c), int(i), int(j), int(k),
                         out.ctypes.data)
        return out

    def fetch_fn(self):
        """Address of the C fetch callback ``turb_fetch(user, c, i, j, k, out)``."""
        return ctypes.cast(lib().turb_fetch, ctypes.c_void_p).value

    def fetch_user(self, dtype: str) -> int:
        return ctypes.addressof(self.tables(dtype))


_dev_lib = None


def dev_lib():
    global _dev_lib
    if _dev_lib is None:
        if not os.path.exists(_DEV_LIB):
            raise ImportError(f"{_DEV_LIB} missing: run bto_inputs._turb.build()")
        L = ctypes.CDLL(_DEV_LIB)
        L.turb_grid_dev.argtypes = [ctypes.c_int32] * 4 + [ctypes.c_void_p] * 9 + \
            [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        L.turb_grid_dev.restype = ctypes.c_int
        _dev_lib = L
    return _dev_lib


class DeviceTurbulence:
    """The same series generated on the GPU (tables uploaded once); grids are
    bit-identical to the host evaluator's."""

    def __init__(self, ev: TurbEvaluator, device="cuda"):
        import torch

        self.ev = ev
        self.t = {k: torch.as_tensor(v, device=device) for k, v in ev.arrs.items()}

    def fill(self, c: int, dtype: str, out, stream=None):
        """Write cycle ``c``'s grid into the device tensor ``out``
        (float32 / float16 / bfloat16 / float64, shape (nz, ny, nx, 3))."""
        import torch

        code = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}[dtype]
        nx, ny, nz = self.ev.n
        st = (stream or torch.cuda.current_stream()).cuda_stream
        t = self.t
        rc = dev_lib().turb_grid_dev(nx, ny, nz, self.ev.M, t["exr"].data_ptr(), t["exi"].data_ptr(),
                                     t["eyr"].data_ptr(), t["eyi"].data_ptr(), t["ezr"].data_ptr(),
                                     t["ezi"].data_ptr(), t["pr"].data_ptr(), t["pi"].data_ptr(),
                                     t["amp"].data_ptr(), int(c), code, out.data_ptr(), st)
        if rc != 0:
            raise RuntimeError(f"turb_grid_dev failed ({rc})")
        return out


def store_round(x: np.ndarray, dtype: str) -> np.ndarray:
    y = np.array(x, dtype=np.float64, copy=True)
    lib().turb_store_round(y.ctypes.data, y.size, _DT_CODE[dtype])
    return y
