"""In situ driver: consecutive non-overlapping intervals over a stream of cycles.

The simulation hands over one velocity grid per cycle (Section 2.2: in situ
only the current time step is available).  The driver advances the live
particles by one RK4 step per cycle through the library, and every `interval`
cycles (a write cycle, Section 2.3) writes the flow map of the finished
interval and reseeds the lattice for the next one.  Timing follows the paper's
metric (Section 4.2): the average time per cycle of advection and particle
management, with the write cycles (flow-map output and reseeding) excluded.

Argument marshalling and sequencing only; all computation runs in the
library's kernels.
"""

from __future__ import annotations

from typing import Callable, List, Optional

import torch

from .context import _TORCH_DT, Context


class InSituDriver:
    """Feed ``cycle(grid, t)`` once per simulation cycle.

    ``on_flowmap(index, flowmap, t0, t1)`` receives each finished interval's
    seed-ordered flow map (device tensors, reused by the next interval unless
    copied).  With ``copy=True`` every grid is copied into a device ring owned
    by the driver, so the simulation may overwrite its own buffer right after
    the call; otherwise the caller must keep each grid unchanged until the next
    cycle has been enqueued.

    ``overlap=True`` (needs ``copy=True``) runs the driver on two streams of
    its own: the copy of each incoming grid on an ingest stream into a
    three-slot ring, the advection on a compute stream.  Events order them:
    the ingest copy waits for the simulation's stream to reach the call and
    for the last step that read the slot it overwrites; the step waits for
    the copy of its new grid; the simulation's stream waits only for the copy
    (so it may overwrite its buffer), never for the advection, which therefore
    overlaps the simulation's next cycle and the next copy.
    """

    def __init__(self, ctx: Context, interval: int, stride: int, mode: str = "linear", copy: bool = False,
                 on_flowmap: Optional[Callable] = None, timing: bool = True, overlap: bool = False):
        if interval < 1:
            raise ValueError("interval must be >= 1")
        if overlap and not copy:
            raise ValueError("overlap needs copy=True (the driver must own the grids it reads later)")
        self.ctx = ctx
        self.interval = int(interval)
        self.stride = int(stride)
        self.mode = mode
        self.copy = copy
        self.overlap = overlap
        self.on_flowmap = on_flowmap
        self.timing = timing
        self._prev = None
        self._prev_t = None
        self._prev_slot = None
        self._ring: List[torch.Tensor] = []
        self._slot = 0
        self.steps_in_interval = 0
        self.intervals_done = 0
        self._t0 = None
        self._events = []          # (start, end) per advection cycle
        self._out = None
        if overlap:
            self._compute = torch.cuda.Stream()   # default priority
            self._ingest = torch.cuda.Stream()
            self._read_done: List[Optional[torch.cuda.Event]] = [None, None, None]
        else:
            self._compute = None

    def _own(self, grid: torch.Tensor):
        if not self.copy:
            return grid, None
        nslot = 3 if self.overlap else 2
        if not self._ring:
            self._ring = [torch.empty_like(grid) for _ in range(nslot)]
        k = self._slot
        self._slot = (k + 1) % nslot
        dst = self._ring[k]
        if not self.overlap:
            dst.copy_(grid)
            return dst, k
        sim = torch.cuda.current_stream()
        self._ingest.wait_stream(sim)                 # the grid is complete once the simulation gets here
        if self._read_done[k] is not None:
            self._ingest.wait_event(self._read_done[k])  # the step that last read this slot is done
        with torch.cuda.stream(self._ingest):
            dst.copy_(grid)
        copied = torch.cuda.Event()
        copied.record(self._ingest)
        sim.wait_event(copied)                        # the simulation may overwrite its buffer after this
        self._compute.wait_event(copied)              # the next step reads the copy
        grid.record_stream(self._ingest)
        return dst, k

    def _start_interval(self, t):
        self.ctx.seed(self.stride, stream=self._compute)
        self.steps_in_interval = 0
        self._t0 = t

    def _check_grid(self, g: torch.Tensor):
        # each grid is checked once, when it arrives; the step then passes raw pointers
        shape = (self.ctx.n[2], self.ctx.n[1], self.ctx.n[0], 3)
        if g.dtype not in _TORCH_DT or tuple(g.shape) != shape or not g.is_contiguous() or not g.is_cuda:
            raise ValueError(f"every grid must be a contiguous float32/float16/bfloat16 device tensor of shape {shape}")
        if self._prev is not None and g.dtype != self._prev.dtype:
            raise ValueError("all grids of a run must share one dtype")

    def cycle(self, grid: torch.Tensor, t: float):
        """Consume the grid of the next cycle at time ``t``."""
        self._check_grid(grid)
        g, k = self._own(grid)
        if self._prev is None:
            self._start_interval(t)
        else:
            cs = self._compute or torch.cuda.current_stream()
            ptrs = (self._prev.data_ptr(), g.data_ptr())
            times = (self._prev_t, float(t))
            if self.timing:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(cs)
            self.ctx.advect_ptrs(ptrs, times, _TORCH_DT[g.dtype], mode=self.mode, stream=cs)
            if self.timing:
                e1.record(cs)
                self._events.append((e0, e1))
            if self.overlap:
                done = torch.cuda.Event()
                done.record(cs)
                self._read_done[self._prev_slot] = done
                self._read_done[k] = done
            self.steps_in_interval += 1
            if self.steps_in_interval == self.interval:
                # write cycle: flow map of the finished interval, then reseed
                self._out = self.ctx.flowmap(out=self._out, stream=self._compute)
                if self.on_flowmap is not None:
                    if self._compute is not None:
                        torch.cuda.current_stream().wait_stream(self._compute)
                    self.on_flowmap(self.intervals_done, self._out, self._t0, t)
                self.intervals_done += 1
                self._start_interval(t)
        self._prev, self._prev_t, self._prev_slot = g, t, k

    def synchronize(self):
        """Make the caller's current stream wait for everything the driver enqueued."""
        if self._compute is not None:
            torch.cuda.current_stream().wait_stream(self._compute)

    def mean_cycle_ms(self) -> float:
        """Average time per non-write cycle (advection + particle management)."""
        if not self._events:
            return 0.0
        torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in self._events) / len(self._events)
