"""Post hoc side of BTO flow maps on the seed lattice.

* ``place_block``, ``reconstruct_lattice``, ``flowmap_error``: marshalling for
  the library's lattice placement, Eq. (1) rebuild of terminated entries
  (Section 3.2) and Eq. (5)/(6) accuracy metric (Section 4).
* ``run_blocks``: the BTO side of the paper's accuracy experiments on one GPU.
  The domain is cut into equal blocks (each block holds its cells and the grid
  points on its faces, as a rank's block of the simulation grid would); every
  block seeds its own lattice and advects it with termination at its own
  boundary, independently of the others (no communication: Section 3.1), and
  the per-block flow maps are placed into one domain lattice.
* ``run_domain``: the communicating reference -- the same seeds advected
  through the whole domain as one block, so particles cross block boundaries
  freely and only leave at the domain boundary.

Argument marshalling and orchestration only; every arithmetic step runs in the
library's kernels.  Staging a block's sub-grid from a domain-sized grid is a
strided device copy (a rank would own its block directly).
"""

from __future__ import annotations

import ctypes
from typing import Sequence, Tuple

import numpy as np
import torch

from . import _lib
from .context import BTOError, Context

MISSING, KNOWN, REBUILT = 0, 1, 2


def _i3(v) -> ctypes.Array:
    return (ctypes.c_int32 * 3)(*[int(x) for x in v])


def _stream(stream) -> int:
    return (stream or torch.cuda.current_stream()).cuda_stream


def _check(rc: int, what: str):
    if rc != 0:
        raise BTOError(rc, f"{what} failed (bad arguments or a HIP error)")


def place_block(src_end: torch.Tensor, src_flag: torch.Tensor, mb, dst_end: torch.Tensor,
                dst_flag: torch.Tensor, M, off, shift=(0.0, 0.0, 0.0), stream=None):
    """Copy a block's seed-ordered flow map (lattice mb) into the lattice M at
    offset off, adding ``shift`` to the positions."""
    L = _lib.load()
    sh = (ctypes.c_double * 3)(*[float(v) for v in shift])
    _check(L.bto_place_block(_i3(mb), _i3(M), _i3(off), sh, src_end.data_ptr(), src_flag.data_ptr(),
                             dst_end.data_ptr(), dst_flag.data_ptr(), _stream(stream)), "bto_place_block")


def reconstruct_lattice(end: torch.Tensor, flag: torch.Tensor, m, stream=None) -> torch.Tensor:
    """Rebuild non-valid entries of ``end`` (P, 3) float64 in place by Eq. (1);
    returns the (P,) uint8 state: 0 missing (NaN), 1 valid, 2 rebuilt."""
    P = int(np.prod(m))
    if end.dtype != torch.float64 or tuple(end.shape) != (P, 3) or not end.is_contiguous():
        raise ValueError("end must be a contiguous (P, 3) float64 device tensor")
    if flag.dtype != torch.uint8 or flag.numel() != P:
        raise ValueError("flag must be (P,) uint8")
    state = torch.empty(P, dtype=torch.uint8, device=end.device)
    L = _lib.load()
    _check(L.bto_reconstruct_lattice(_i3(m), end.data_ptr(), flag.data_ptr(), state.data_ptr(), _stream(stream)),
           "bto_reconstruct_lattice")
    return state


def flowmap_error(b_end: torch.Tensor, b_state: torch.Tensor, m_end: torch.Tensor, m_flag: torch.Tensor,
                  cell: float = 1.0, stream=None) -> dict:
    """Eq. (5)/(6) of b against the communicating flow map m."""
    out = (ctypes.c_double * 5)()
    L = _lib.load()
    _check(L.bto_flowmap_error(int(b_end.shape[0]), b_end.data_ptr(), b_state.data_ptr(), m_end.data_ptr(),
                               m_flag.data_ptr(), float(cell), out, _stream(stream)), "bto_flowmap_error")
    return dict(mean_l2=out[0], max_l2=out[1], n=int(out[2]), uncovered=int(out[3]), accuracy_pct=out[4])


def lattice_count(cells: int, stride: int) -> int:
    """Lattice points per axis of a block of `cells` cells (cells + 1 points)
    at the default offset (stride - 1) / 2."""
    off = (stride - 1) / 2.0
    return int(np.floor((cells - off) / stride)) + 1


def run_blocks(grids: Sequence[torch.Tensor], times, blocks: Tuple[int, int, int], stride: int,
               mode: str = "linear", spacing: float = 1.0):
    """BTO on a domain cut into blocks[0] x blocks[1] x blocks[2] equal blocks.

    grids: N+1 domain grids (Nz, Ny, Nx, 3) on the device with N_d =
    blocks_d * cells_d + 1 points; every block's cell count must be a multiple
    of ``stride`` (>= 2) so that the block lattices tile the domain lattice.  Returns
    (end (P,3) f64, flag (P,) u8, lattice M) in domain-lattice order (x
    fastest), positions in domain coordinates (origin 0, the given spacing).
    """
    if stride < 2:
        # at stride 1 the lattice has seeds on the faces that neighbouring blocks share,
        # so block lattices overlap instead of tiling the domain lattice
        raise ValueError("run_blocks needs stride >= 2 (stride 1 seeds the shared block faces twice)")
    nz, ny, nx = (int(v) for v in grids[0].shape[:3])
    npts = (nx, ny, nz)
    cells = []
    for d in range(3):
        c, r = divmod(npts[d] - 1, blocks[d])
        if r or c % stride or c < 1:
            raise ValueError("each axis must split into equal blocks whose cells are a multiple of the stride")
        cells.append(c)
    mb = [lattice_count(cells[d], stride) for d in range(3)]
    M = [mb[d] * blocks[d] for d in range(3)]
    P = int(np.prod(M))
    dev = grids[0].device
    end = torch.empty((P, 3), dtype=torch.float64, device=dev)
    flag = torch.empty(P, dtype=torch.uint8, device=dev)
    nb = tuple(c + 1 for c in cells)
    sub = [torch.empty((nb[2], nb[1], nb[0], 3), dtype=grids[0].dtype, device=dev) for _ in grids]
    with Context(nb, int(np.prod(mb)), spacing=[spacing] * 3) as ctx:
        for bz in range(blocks[2]):
            for by in range(blocks[1]):
                for bx in range(blocks[0]):
                    o = (bx * cells[0], by * cells[1], bz * cells[2])
                    for g, s in zip(grids, sub):
                        s.copy_(g[o[2]:o[2] + nb[2], o[1]:o[1] + nb[1], o[0]:o[0] + nb[0]])
                    ctx.seed(stride)
                    ctx.advect(sub, times, mode=mode)
                    fm = ctx.flowmap(with_seeds=False)
                    place_block(fm["end"], fm["flag"], mb, end, flag, M, (bx * mb[0], by * mb[1], bz * mb[2]),
                                shift=[o[d] * spacing for d in range(3)])
    return end, flag, tuple(M)


def run_domain(grids: Sequence[torch.Tensor], times, stride: int, mode: str = "linear", spacing: float = 1.0):
    """The communicating reference: the whole domain as one block."""
    nz, ny, nx = (int(v) for v in grids[0].shape[:3])
    n = (nx, ny, nz)
    M = tuple(lattice_count(n[d] - 1, stride) for d in range(3))
    with Context(n, int(np.prod(M)), spacing=[spacing] * 3) as ctx:
        ctx.seed(stride)
        ctx.advect(grids, times, mode=mode)
        fm = ctx.flowmap(with_seeds=False)
    return fm["end"], fm["flag"], M
