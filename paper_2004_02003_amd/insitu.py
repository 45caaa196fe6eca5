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

from .context import Context


class InSituDriver:
    """Feed ``cycle(grid, t)`` once per simulation cycle.

    ``on_flowmap(index, flowmap, t0, t1)`` receives each finished interval's
    seed-ordered flow map (device tensors, reused by the next interval unless
    copied).  With ``copy=True`` every grid is copied into a two-slot device
    ring owned by the driver, so the simulation may overwrite its own buffer
    right after the call; otherwise the caller must keep each grid unchanged
    until the next cycle has been enqueued.
    """

    def __init__(self, ctx: Context, interval: int, stride: int, mode: str = "linear", copy: bool = False,
                 on_flowmap: Optional[Callable] = None, timing: bool = True):
        if interval < 1:
            raise ValueError("interval must be >= 1")
        self.ctx = ctx
        self.interval = int(interval)
        self.stride = int(stride)
        self.mode = mode
        self.copy = copy
        self.on_flowmap = on_flowmap
        self.timing = timing
        self._prev = None
        self._prev_t = None
        self._ring: List[torch.Tensor] = []
        self._slot = 0
        self.steps_in_interval = 0
        self.intervals_done = 0
        self._t0 = None
        self._events = []          # (start, end) per advection cycle
        self._out = None

    def _own(self, grid: torch.Tensor) -> torch.Tensor:
        if not self.copy:
            return grid
        if not self._ring:
            self._ring = [torch.empty_like(grid), torch.empty_like(grid)]
        dst = self._ring[self._slot]
        self._slot ^= 1
        dst.copy_(grid)
        return dst

    def _start_interval(self, t):
        self.ctx.seed(self.stride)
        self.steps_in_interval = 0
        self._t0 = t

    def cycle(self, grid: torch.Tensor, t: float):
        """Consume the grid of the next cycle at time ``t``."""
        g = self._own(grid)
        if self._prev is None:
            self._start_interval(t)
        else:
            if self.timing:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
            self.ctx.advect([self._prev, g], [self._prev_t, t], mode=self.mode)
            if self.timing:
                e1.record()
                self._events.append((e0, e1))
            self.steps_in_interval += 1
            if self.steps_in_interval == self.interval:
                # write cycle: flow map of the finished interval, then reseed
                self._out = self.ctx.flowmap(out=self._out)
                if self.on_flowmap is not None:
                    self.on_flowmap(self.intervals_done, self._out, self._t0, t)
                self.intervals_done += 1
                self._start_interval(t)
        self._prev, self._prev_t = g, t

    def mean_cycle_ms(self) -> float:
        """Average time per non-write cycle (advection + particle management)."""
        if not self._events:
            return 0.0
        torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in self._events) / len(self._events)
