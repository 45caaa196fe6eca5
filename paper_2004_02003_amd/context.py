"""Python face of the C-ABI: one ``Context`` per block.

Argument marshalling only.  torch tensors provide device memory and the
current HIP stream; every step of the path (seeding, RK4 advection, boundary
termination, compaction, flow-map writing) runs in the library's kernels.
"""

from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import BTOError

_TORCH_DT = {torch.float32: _lib.BTO_F32, torch.float16: _lib.BTO_F16, torch.bfloat16: _lib.BTO_BF16}
_MODES = {"linear": _lib.BTO_TIME_LINEAR, "frozen": _lib.BTO_TIME_FROZEN}


def _flags(mode: str, record_exit: bool = False, record_ckpt: bool = False, fp64: bool = False) -> int:
    return (_MODES[mode] | (_lib.BTO_RECORD_EXIT if record_exit else 0)
            | (_lib.BTO_RECORD_CKPT if record_ckpt else 0) | (_lib.BTO_SAMPLE_FP64 if fp64 else 0))


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def grid_to_device(grid: np.ndarray, dtype: str, device="cuda") -> torch.Tensor:
    """Upload a stored grid (float32, float16, or bfloat16 bits as uint16)."""
    g = np.ascontiguousarray(grid)
    if dtype == "bf16":
        t = torch.from_numpy(g.view(np.int16)).view(torch.bfloat16)
    else:
        t = torch.from_numpy(g)
    return t.to(device, non_blocking=False)


class Context:
    """One block of the decomposition: n = (nx, ny, nz) grid points."""

    def __init__(self, n, max_particles: int, origin=(0.0, 0.0, 0.0), spacing=(1.0, 1.0, 1.0),
                 device: int = 0):
        self.L = _lib.load()
        blk = _lib.Block()
        blk.n[:] = [int(v) for v in n]
        blk.origin[:] = [float(v) for v in origin]
        blk.spacing[:] = [float(v) for v in spacing]
        self.n = tuple(int(v) for v in n)
        self.device = int(device)
        self.max_particles = int(max_particles)
        h = ctypes.c_void_p()
        rc = self.L.bto_create(ctypes.byref(blk), int(max_particles), self.device, ctypes.byref(h))
        if rc != 0:
            raise BTOError(rc, "bto_create failed (bad block, capacity or device, or out of memory)")
        self._h = h
        self.n_seeds = 0

    # -- helpers -----------------------------------------------------------
    def _check(self, rc: int):
        if rc != 0:
            msg = self.L.bto_last_error(self._h).decode(errors="replace")
            raise BTOError(rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            self.L.bto_destroy(self._h)
            self._h = None

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
    def handle(self) -> int:
        return self._h.value

    def tuning(self) -> dict:
        t = _lib.Tuning()
        self._check(self.L.bto_get_tuning(self._h, ctypes.byref(t)))
        return dict(steps_per_launch=t.steps_per_launch, rebin_every=t.rebin_every,
                    blocks_per_cu=t.blocks_per_cu, lanes_per_particle=t.lanes_per_particle,
                    ckpt_every=t.ckpt_every, tiles=t.tiles)

    def set_tuning(self, steps_per_launch=None, rebin_every=None, blocks_per_cu=None,
                   lanes_per_particle=None, ckpt_every=None, tiles=None):
        """Launch shape of the advection (events unchanged; positions agree
        to FP32 rounding), the spacing of recorded checkpoints, and the tile
        layout (tile-staged steps; latched at the next seeding)."""
        cur = self.tuning()
        t = _lib.Tuning()
        t.steps_per_launch = cur["steps_per_launch"] if steps_per_launch is None else int(steps_per_launch)
        t.rebin_every = cur["rebin_every"] if rebin_every is None else int(rebin_every)
        t.blocks_per_cu = cur["blocks_per_cu"] if blocks_per_cu is None else int(blocks_per_cu)
        t.lanes_per_particle = (cur["lanes_per_particle"] if lanes_per_particle is None
                                else int(lanes_per_particle))
        t.ckpt_every = cur["ckpt_every"] if ckpt_every is None else int(ckpt_every)
        t.tiles = cur["tiles"] if tiles is None else int(tiles)
        self._check(self.L.bto_set_tuning(self._h, ctypes.byref(t)))

    # -- the path ----------------------------------------------------------
    def seed(self, stride: int, offset=None, stream=None) -> int:
        off = None if offset is None else (ctypes.c_double * 3)(*[float(v) for v in offset])
        P = ctypes.c_int64()
        self._check(self.L.bto_seed(self._h, int(stride), off, ctypes.byref(P), _stream_ptr(stream)))
        self.n_seeds = int(P.value)
        self._new_interval()
        return self.n_seeds

    def _new_interval(self):
        # host-side bookkeeping of the interval (which one, steps advanced so far)
        self.interval_serial = getattr(self, "interval_serial", 0) + 1
        self.steps_advected = 0

    def seed_explicit(self, xyz: torch.Tensor, stream=None) -> int:
        if xyz.dtype != torch.float64 or xyz.dim() != 2 or xyz.shape[1] != 3 or not xyz.is_contiguous():
            raise ValueError("seeds must be a contiguous (n, 3) float64 device tensor")
        self._check(self.L.bto_seed_explicit(self._h, xyz.data_ptr(), int(xyz.shape[0]), _stream_ptr(stream)))
        self.n_seeds = int(xyz.shape[0])
        self._new_interval()
        return self.n_seeds

    def advect(self, grids: Sequence[torch.Tensor], times, mode: str = "linear", record_exit: bool = False,
               stream=None, record_ckpt: bool = False, fp64: bool = False):
        """n = len(grids) - 1 RK4 steps through the given consecutive cycles;
        ``record_exit`` keeps the exit point of every particle terminated here
        (``exit_points``); ``record_ckpt`` records checkpoints every
        ``tuning()["ckpt_every"]`` steps for ``adjoint(..., recorded=True)``;
        ``fp64`` samples the field in extended precision (BTO_SAMPLE_FP64: FP64
        sums and stage velocities over FP32-weighted corner differences)."""
        if len(grids) < 2:
            raise ValueError("need at least two grids (one step)")
        dt = grids[0].dtype
        if dt not in _TORCH_DT:
            raise ValueError(f"unsupported grid dtype {dt}")
        shape = (self.n[2], self.n[1], self.n[0], 3)
        for g in grids:
            if g.dtype != dt or tuple(g.shape) != shape or not g.is_contiguous() or not g.is_cuda:
                raise ValueError(f"every grid must be a contiguous {dt} device tensor of shape {shape}")
        times = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
        if times.shape != (len(grids),):
            raise ValueError("one time per grid")
        ptrs = (ctypes.c_void_p * len(grids))(*[g.data_ptr() for g in grids])
        self._check(self.L.bto_advect_interval(self._h, ptrs, times.ctypes.data, len(grids) - 1,
                                               _TORCH_DT[dt], _flags(mode, record_exit, record_ckpt, fp64),
                                               _stream_ptr(stream)))
        self.steps_advected = getattr(self, "steps_advected", 0) + len(grids) - 1

    def advect_ptrs(self, ptrs, times, dtype: int, mode: str = "linear", record_exit: bool = False, stream=None,
                    record_ckpt: bool = False, fp64: bool = False):
        """Same as ``advect`` with raw device pointers (no per-call tensor checks)."""
        arr = (ctypes.c_void_p * len(ptrs))(*ptrs)
        t = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
        self._check(self.L.bto_advect_interval(self._h, arr, t.ctypes.data, len(ptrs) - 1, int(dtype),
                                               _flags(mode, record_exit, record_ckpt, fp64), _stream_ptr(stream)))
        self.steps_advected = getattr(self, "steps_advected", 0) + len(ptrs) - 1

    def flowmap(self, with_seeds: bool = True, count_valid: bool = False, out=None, stream=None):
        """Seed-ordered flow map: dict with end (P,3) f64, flag (P,) u8,
        exit (P,) i32, optionally seed (P,3) f64 and n_valid."""
        P = self.n_seeds
        dev = torch.device("cuda", self.device)
        if out is None:
            out = dict(end=torch.empty((P, 3), dtype=torch.float64, device=dev),
                       flag=torch.empty(P, dtype=torch.uint8, device=dev),
                       exit=torch.empty(P, dtype=torch.int32, device=dev))
            if with_seeds:
                out["seed"] = torch.empty((P, 3), dtype=torch.float64, device=dev)
        nv = ctypes.c_int64(-1)
        self._check(self.L.bto_flowmap_out(
            self._h, out["seed"].data_ptr() if "seed" in out else None, out["end"].data_ptr(),
            out["flag"].data_ptr(), out["exit"].data_ptr(),
            ctypes.byref(nv) if count_valid else None, _stream_ptr(stream)))
        if count_valid:
            out["n_valid"] = int(nv.value)
        return out

    def exit_points(self, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """(P, 3) float64: where each terminated trajectory left the block
        (world coordinates, on the block surface); NaN for other seeds."""
        if out is None:
            out = torch.empty((self.n_seeds, 3), dtype=torch.float64, device=torch.device("cuda", self.device))
        if out.dtype != torch.float64 or tuple(out.shape) != (self.n_seeds, 3) or not out.is_contiguous():
            raise ValueError("out must be a contiguous (P, 3) float64 device tensor")
        self._check(self.L.bto_exit_points(self._h, out.data_ptr(), _stream_ptr(stream)))
        return out

    def adjoint(self, grids: Sequence[torch.Tensor], times, cot: torch.Tensor, grad_grids=None,
                ckpt_every: int = 10, mode: str = "linear", status: Optional[torch.Tensor] = None,
                stream=None, recorded: bool = False) -> torch.Tensor:
        """Gradients d(cot . x_end)/d x_0 for the current seeds (n_cot = cot.shape[1]
        cotangent vectors per seed; 3 unit cotangents give the Jacobian rows).
        ``recorded``: take the forward trajectory from the checkpoints that the
        interval's advection recorded (``advect(..., record_ckpt=True)``, same
        grids, times and mode) instead of recomputing it.
        ``grad_grids`` (optional list of float32 tensors shaped like the grids)
        receive d L / d V added in place."""
        P = self.n_seeds
        dt = grids[0].dtype
        if cot.dim() == 2:
            cot = cot.view(P, 1, 3)
        if cot.dtype != torch.float32 or tuple(cot.shape[::2]) != (P, 3) or not cot.is_contiguous():
            raise ValueError("cot must be a contiguous float32 tensor (P, n_cot, 3)")
        ncot = int(cot.shape[1])
        shape = (self.n[2], self.n[1], self.n[0], 3)
        for g in grids:
            if g.dtype != dt or tuple(g.shape) != shape or not g.is_contiguous():
                raise ValueError("grids must share dtype and shape")
        times = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
        out = torch.empty((P, ncot, 3), dtype=torch.float32, device=cot.device)
        ptrs = (ctypes.c_void_p * len(grids))(*[g.data_ptr() for g in grids])
        gptr = None
        if grad_grids is not None:
            for g in grad_grids:
                if g.dtype != torch.float32 or tuple(g.shape) != shape or not g.is_contiguous():
                    raise ValueError("grad grids must be contiguous float32 tensors shaped like the grids")
            gptr = (ctypes.c_void_p * len(grad_grids))(*[g.data_ptr() for g in grad_grids])
        self._check(self.L.bto_adjoint_interval(
            self._h, ptrs, times.ctypes.data, len(grids) - 1, _TORCH_DT[dt], _flags(mode, record_ckpt=recorded),
            cot.data_ptr(), ncot,
            out.data_ptr(), gptr, status.data_ptr() if status is not None else None, int(ckpt_every),
            _stream_ptr(stream)))
        return out

    def adjoint_segment(self, segment: int, grids: Sequence[torch.Tensor], times, cot: Optional[torch.Tensor] = None,
                        n_cot: int = 1, grad_seed: Optional[torch.Tensor] = None, grad_grids=None,
                        status: Optional[torch.Tensor] = None, mode: str = "linear", stream=None) -> None:
        """One checkpoint segment of the adjoint of a recorded interval
        (segments swept from the last down to 0): ``grids``/``times`` are the
        segment's cycles, ``cot`` (P, n_cot, 3) is read by the first call,
        ``grad_seed`` (P, n_cot, 3) is written by the call for segment 0."""
        P = self.n_seeds
        dt = grids[0].dtype
        shape = (self.n[2], self.n[1], self.n[0], 3)
        for g in grids:
            if g.dtype != dt or tuple(g.shape) != shape or not g.is_contiguous():
                raise ValueError("grids must share dtype and shape")
        for t, nm in ((cot, "cot"), (grad_seed, "grad_seed")):
            if t is not None and (t.dtype != torch.float32 or t.numel() != P * n_cot * 3 or not t.is_contiguous()):
                raise ValueError(f"{nm} must be a contiguous float32 tensor of P x n_cot x 3")
        times = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
        ptrs = (ctypes.c_void_p * len(grids))(*[g.data_ptr() for g in grids])
        gptr = None
        if grad_grids is not None:
            for g in grad_grids:
                if g.dtype != torch.float32 or tuple(g.shape) != shape or not g.is_contiguous():
                    raise ValueError("grad grids must be contiguous float32 tensors shaped like the grids")
            gptr = (ctypes.c_void_p * len(grad_grids))(*[g.data_ptr() for g in grad_grids])
        self._check(self.L.bto_adjoint_segment(
            self._h, int(segment), ptrs, times.ctypes.data, _TORCH_DT[dt], _flags(mode),
            cot.data_ptr() if cot is not None else None, int(n_cot),
            grad_seed.data_ptr() if grad_seed is not None else None, gptr,
            status.data_ptr() if status is not None else None, _stream_ptr(stream)))

    def touched_points(self, grids: Sequence[torch.Tensor], times, mode: str = "linear", fp64: bool = False,
                       stream=None) -> np.ndarray:
        """Distinct grid points each step of the interval samples, per level,
        for the seeds of the last seeding: (N, 3) uint64 rows of (points of
        level n, points of level n + 1, particles entering step n)."""
        dt = grids[0].dtype
        shape = (self.n[2], self.n[1], self.n[0], 3)
        for g in grids:
            if g.dtype != dt or tuple(g.shape) != shape or not g.is_contiguous():
                raise ValueError("grids must share dtype and shape")
        times = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
        N = len(grids) - 1
        if len(times) != N + 1:
            raise ValueError("one time per grid")
        ptrs = (ctypes.c_void_p * len(grids))(*[g.data_ptr() for g in grids])
        out = torch.empty(3 * N, dtype=torch.int64, device=grids[0].device)
        self._check(self.L.bto_touched_points(self._h, ptrs, times.ctypes.data, N, _TORCH_DT[dt],
                                              _flags(mode, fp64=fp64), out.data_ptr(), _stream_ptr(stream)))
        return out.cpu().numpy().astype(np.uint64).reshape(N, 3)

    def ftle(self, jac: torch.Tensor, T: float, stream=None) -> torch.Tensor:
        """FTLE per seed from (P, 3, 3) float32 Jacobians."""
        jac = jac.contiguous()
        if jac.dtype != torch.float32 or jac.shape[1:] != (3, 3):
            raise ValueError("jac must be float32 (P, 3, 3)")
        out = torch.empty(jac.shape[0], dtype=torch.float32, device=jac.device)
        self._check(self.L.bto_ftle(self._h, jac.data_ptr(), int(jac.shape[0]), float(T), out.data_ptr(),
                                    _stream_ptr(stream)))
        return out

    def stats(self, stream=None) -> dict:
        st = _lib.Stats()
        self._check(self.L.bto_stats(self._h, ctypes.byref(st), _stream_ptr(stream)))
        return dict(n_seeds=st.n_seeds, n_live=st.n_live, particle_steps=st.particle_steps,
                    steps_done=st.steps_done)
