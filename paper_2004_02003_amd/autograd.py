"""Differentiable flow map: ``torch.autograd.Function`` over the C-ABI.

Forward: seed the given positions, advance them through the grids (one RK4
step per cycle, boundary termination, checkpoints recorded every
``ckpt_every`` steps) and return the end positions with their flags.
Backward: the library's discrete adjoint from those checkpoints (gradients
with respect to the seed positions and, when the grids require grad, the
grids); if the context has been reseeded or advanced since the forward, the
adjoint reseeds and recomputes the forward itself.  Seeds that leave the
block contribute nothing to the gradients.
"""

from __future__ import annotations

import numpy as np
import torch

from .context import Context


class BTOAdvectFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, bctx: Context, seeds: torch.Tensor, times, mode: str, ckpt_every: int, *grids):
        s = seeds.detach().to(torch.float64).contiguous()
        bctx.seed_explicit(s)
        k_prev = bctx.tuning()["ckpt_every"]
        bctx.set_tuning(ckpt_every=int(ckpt_every))
        try:
            bctx.advect(list(grids), times, mode=mode, record_ckpt=True)
        finally:
            bctx.set_tuning(ckpt_every=k_prev)
        fctx.serial = (bctx.interval_serial, bctx.steps_advected)
        fm = bctx.flowmap(with_seeds=False)
        fctx.bctx = bctx
        fctx.times = np.asarray(times, dtype=np.float64)
        fctx.mode = mode
        fctx.ckpt_every = int(ckpt_every)
        fctx.seed_dtype = seeds.dtype
        fctx.save_for_backward(s, *grids)
        fctx.mark_non_differentiable(fm["flag"], fm["exit"])
        return fm["end"].to(seeds.dtype), fm["flag"], fm["exit"]

    @staticmethod
    def backward(fctx, g_end, g_flag, g_exit):
        s, *grids = fctx.saved_tensors
        bctx = fctx.bctx
        recorded = (bctx.interval_serial, bctx.steps_advected) == fctx.serial
        if not recorded:
            bctx.seed_explicit(s)
        want_grids = any(fctx.needs_input_grad[5:])
        gg = [torch.zeros(g.shape, dtype=torch.float32, device=g.device) for g in grids] if want_grids else None
        cot = g_end.to(torch.float32).contiguous()
        gs = bctx.adjoint(grids, fctx.times, cot, grad_grids=gg, ckpt_every=fctx.ckpt_every, mode=fctx.mode,
                          recorded=recorded)
        g_seed = gs.view(-1, 3).to(fctx.seed_dtype) if fctx.needs_input_grad[1] else None
        g_grids = [g.to(v.dtype) for g, v in zip(gg, grids)] if want_grids else [None] * len(grids)
        return (None, g_seed, None, None, None, *g_grids)


def advect_autograd(bctx: Context, seeds: torch.Tensor, grids, times, mode: str = "linear", ckpt_every: int = 10):
    """End positions (differentiable), flags and exit steps of ``seeds``."""
    return BTOAdvectFn.apply(bctx, seeds, times, mode, ckpt_every, *grids)


def jacobian_ftle(bctx: Context, seeds: torch.Tensor, grids, times, mode: str = "linear", ckpt_every: int = 10):
    """Flow-map Jacobians dx_end/dx_0 (P, 3, 3) and FTLE (P,) for ``seeds``
    (rows of terminated seeds are zero and their FTLE is meaningless)."""
    P = seeds.shape[0]
    bctx.seed_explicit(seeds.to(torch.float64).contiguous())
    cot = torch.eye(3, dtype=torch.float32, device=seeds.device).expand(P, 3, 3).contiguous()
    status = torch.empty(P, dtype=torch.uint8, device=seeds.device)
    J = bctx.adjoint(grids, times, cot, ckpt_every=ckpt_every, mode=mode, status=status)
    T = float(times[-1] - times[0])
    sigma = bctx.ftle(J, T)
    return J, sigma, status


def ftle(bctx: Context, jac: torch.Tensor, T: float) -> torch.Tensor:
    return bctx.ftle(jac, T)
