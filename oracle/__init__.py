"""FP64 CPU oracle of the per-block BTO path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the product library never imports it.  The arithmetic lives in
``bto_oracle.c`` (plain C, FP64, OpenMP over particles); this module builds it
with gcc and marshals numpy arrays through ctypes.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against exact rational arithmetic, closed forms, invariants and central finite
differences (see the test module docstrings for what pins which part).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bto_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

VALID, TERMINATED, INVALID = 0, 1, 2
LINEAR, FROZEN = 0, 1
_DT_CODE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}

FETCH_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_int32, ctypes.POINTER(ctypes.c_double))


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("n_steps", ctypes.c_int32),
                ("times", ctypes.c_void_p), ("mode", ctypes.c_int32),
                ("first_cycle", ctypes.c_int32), ("fetch", ctypes.c_void_p),
                ("user", ctypes.c_void_p)]


class _Dense(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("dtype", ctypes.c_int32),
                ("grids", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        L.orc_flowmap.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int32]
        L.orc_flowmap.restype = ctypes.c_int
        L.orc_adjoint.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, ctypes.c_int32]
        L.orc_adjoint.restype = ctypes.c_int
        L.orc_sample.argtypes = [vp, ctypes.c_int32, ctypes.c_double, vp, vp, vp]
        L.orc_lattice_count.argtypes = [vp, ctypes.c_int32, vp, vp]
        L.orc_lattice_count.restype = ctypes.c_int64
        L.orc_seed_lattice.argtypes = [vp, ctypes.c_int32, vp, vp]
        _lib = L
    return _lib


def _dtype_of(a: np.ndarray, dtype: Optional[str]) -> str:
    if dtype is not None:
        return dtype
    if a.dtype == np.float64:
        return "f64"
    if a.dtype == np.float32:
        return "f32"
    if a.dtype == np.float16:
        return "f16"
    raise ValueError("pass dtype='bf16' for uint16 bfloat16 grids")


class Field:
    """Grid values for the oracle: dense arrays (one per cycle) or a C fetch
    callback (``fn``, ``user``) that returns one grid point's stored value."""

    def __init__(self, n, grids: Optional[Sequence[np.ndarray]] = None, dtype: Optional[str] = None,
                 fn: Optional[int] = None, user: Optional[int] = None, keep=None,
                 py_fetch=None):
        self.n = tuple(int(v) for v in n)
        self._keep = [keep]
        if grids is not None:
            arrs = [np.ascontiguousarray(g) for g in grids]
            dt = _dtype_of(arrs[0], dtype)
            for g in arrs:
                assert g.shape == (self.n[2], self.n[1], self.n[0], 3), g.shape
            ptrs = (ctypes.c_void_p * len(arrs))(*[g.ctypes.data for g in arrs])
            d = _Dense()
            d.n[:] = self.n
            d.dtype = _DT_CODE[dt]
            d.grids = ctypes.cast(ptrs, ctypes.c_void_p).value
            self._keep += [arrs, ptrs, d]
            self.fn = ctypes.cast(lib().orc_dense_fetch, ctypes.c_void_p).value
            self.user = ctypes.addressof(d)
        elif py_fetch is not None:
            def _cb(user, c, i, j, k, out, _f=py_fetch):
                v = _f(c, i, j, k)
                out[0], out[1], out[2] = float(v[0]), float(v[1]), float(v[2])
            cb = FETCH_FN(_cb)
            self._keep.append(cb)
            self.fn = ctypes.cast(cb, ctypes.c_void_p).value
            self.user = None
        else:
            self.fn, self.user = fn, user

    @classmethod
    def lazy_turbulence(cls, series, dtype: str):
        ev = series.lazy
        return cls(series.n, fn=ev.fetch_fn(), user=ev.fetch_user(dtype), keep=ev)


def _problem(field: Field, times, n_steps, mode, first_cycle):
    times = np.ascontiguousarray(np.asarray(times, dtype=np.float64)[first_cycle:first_cycle + n_steps + 1])
    pr = _Problem()
    pr.n[:] = field.n
    pr.n_steps = int(n_steps)
    pr.times = times.ctypes.data
    pr.mode = int(mode)
    pr.first_cycle = int(first_cycle)
    pr.fetch = field.fn
    pr.user = field.user
    return pr, times


def seed_lattice(n, stride: int, off=None) -> np.ndarray:
    """Seeds off + stride*m per axis (default off = (stride-1)/2), id x-fastest."""
    n3 = (ctypes.c_int32 * 3)(*n)
    off = [(stride - 1) / 2.0] * 3 if off is None else list(off)
    o3 = (ctypes.c_double * 3)(*off)
    m3 = (ctypes.c_int32 * 3)()
    P = lib().orc_lattice_count(n3, int(stride), o3, m3)
    out = np.empty((P, 3), dtype=np.float64)
    lib().orc_seed_lattice(n3, int(stride), o3, out.ctypes.data)
    return out


def flowmap(field: Field, times, seeds: np.ndarray, n_steps: int, mode: int = LINEAR,
            first_cycle: int = 0, jac: bool = False, nthreads: int = 0):
    """Run the interval for every seed; returns a dict of numpy arrays:
    end (P,3), flag (P,), exit (P,), margin (P,), sig (P,), face (P,3) and
    face_cond (P,) (exit point on the box surface for particles terminated in
    a step, NaN otherwise, and its error-growth factor), [jac (P,3,3)]."""
    seeds = np.ascontiguousarray(seeds, dtype=np.float64).reshape(-1, 3)
    P = seeds.shape[0]
    pr, tkeep = _problem(field, times, n_steps, mode, first_cycle)
    out = dict(end=np.empty((P, 3)), flag=np.empty(P, np.uint8), exit=np.empty(P, np.int32),
               margin=np.empty(P), sig=np.empty(P, np.uint64), face=np.empty((P, 3)), face_cond=np.empty(P))
    J = np.empty((P, 3, 3)) if jac else None
    rc = lib().orc_flowmap(ctypes.byref(pr), P, seeds.ctypes.data, out["end"].ctypes.data,
                           out["flag"].ctypes.data, out["exit"].ctypes.data, out["margin"].ctypes.data,
                           out["sig"].ctypes.data, J.ctypes.data if jac else None, out["face"].ctypes.data,
                           out["face_cond"].ctypes.data, int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the problem (bad sizes or non-increasing times)")
    if jac:
        out["jac"] = J
    return out


def adjoint(field: Field, times, seeds: np.ndarray, n_steps: int, cot: np.ndarray,
            mode: int = LINEAR, first_cycle: int = 0, grid_grad: bool = False, nthreads: int = 0):
    """dL/dx0 (P,3) for L = sum over VALID particles of cot_p . x_p(T); with
    ``grid_grad`` also dL/dV as a list of N+1 FP64 grids."""
    seeds = np.ascontiguousarray(seeds, dtype=np.float64).reshape(-1, 3)
    cot = np.ascontiguousarray(cot, dtype=np.float64).reshape(-1, 3)
    P = seeds.shape[0]
    pr, tkeep = _problem(field, times, n_steps, mode, first_cycle)
    g = np.empty((P, 3))
    gg = None
    ptrs = None
    if grid_grad:
        nx, ny, nz = field.n
        gg = [np.zeros((nz, ny, nx, 3)) for _ in range(n_steps + 1)]
        ptrs = (ctypes.c_void_p * len(gg))(*[a.ctypes.data for a in gg])
    rc = lib().orc_adjoint(ctypes.byref(pr), P, seeds.ctypes.data, cot.ctypes.data, g.ctypes.data,
                           ptrs, int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return (g, gg) if grid_grad else g


def fetch(field: Field, c: int, ijk) -> np.ndarray:
    """The stored values of grid points ``ijk`` (M x 3 integer indices) of
    cycle ``c`` as the oracle reads them (through the field's fetch callback,
    before any interpolation)."""
    fn = FETCH_FN(field.fn)
    ijk = np.asarray(ijk, dtype=np.int64).reshape(-1, 3)
    out = np.empty((len(ijk), 3))
    buf = (ctypes.c_double * 3)()
    for q, (i, j, k) in enumerate(ijk):
        fn(field.user, int(c), int(i), int(j), int(k), buf)
        out[q] = buf[:]
    return out


def sample(field: Field, times, n: int, theta: float, p, mode: int = LINEAR):
    """Velocity S(p, n, theta) and its spatial gradient (3x3) at one point."""
    pr, tkeep = _problem(field, times, max(n + 1, 1), mode, 0)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    v = np.empty(3)
    G = np.empty(9)
    lib().orc_sample(ctypes.byref(pr), int(n), float(theta), pp.ctypes.data, v.ctypes.data, G.ctypes.data)
    return v, G.reshape(3, 3)


def ftle(jac: np.ndarray, T: float) -> np.ndarray:
    """sigma = ln sqrt(lambda_max(J^T J)) / |T| per particle (Haller's definition)."""
    C = np.einsum("pki,pkj->pij", jac, jac)
    lam = np.linalg.eigvalsh(C)[:, -1]
    return np.log(np.sqrt(lam)) / abs(T)
