"""The five per-block workloads, by what they are.

Each entry fixes the block, the analytic field, the number of cycles and dt,
the seed-lattice stride, the interval length and the storage precisions.  All
inputs are seeded and synthetic (the paper's Cloverleaf3D, Jet, Nyx and ABC
data files are not available): the ABC block stands for the paper's ABC runs
(one octant of a 256^3 domain), the Fourier-mode turbulence stands for the
turbulent Jet and Nyx data, and the double gyre is a small smoke workload.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Tuple

import numpy as np

from . import fields


@dataclass(frozen=True)
class Workload:
    name: str
    n: Tuple[int, int, int]
    n_cycles: int
    dt: float
    stride: int
    n_steps: int
    dtypes: Tuple[str, ...]
    make_field: Callable[[], fields.FieldSeries]
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def seeds_per_axis(self):
        off = (self.stride - 1) / 2.0
        return tuple(int(math.floor((nd - 1 - off) / self.stride)) + 1 for nd in self.n)

    @property
    def n_seeds(self) -> int:
        a, b, c = self.seeds_per_axis
        return a * b * c


WORKLOADS = {
    # 32^3 double gyre, 16^3 seeds, 50 steps of dt 0.1, FP32 storage.
    "double_gyre_32": Workload(
        "double_gyre_32", (32, 32, 32), 51, 0.1, 2, 50, ("f32",),
        lambda: fields.double_gyre(32, 51, 0.1),
        "A=0.1, eps=0.25, omega=2pi/10, w=0.1 sin(pi z/32)"),
    # 128^3 time-varying ABC + N(0, 0.01^2) noise, 64^3 seeds, 100 steps of dt 0.05.
    "abc_128": Workload(
        "abc_128", (128, 128, 128), 101, 0.05, 2, 100, ("f32",),
        lambda: fields.abc_noise(128, 101, 0.05, seed=1),
        "octant [0,127]^3 of a 256^3 ABC domain; noise seed 1"),
    # 256^3 Fourier turbulence (64 modes), 128^3 seeds, 50 steps of dt 0.02.
    "turb_256": Workload(
        "turb_256", (256, 256, 256), 51, 0.02, 2, 50, ("f32", "f16", "bf16"),
        lambda: fields.turbulence(256, 64, 2, 51, 0.02),
        "mode seed 2, rms displacement 1.5 cells per step"),
    # ABC field as abc_128, 32^3 seeds (stride 4), 100 steps, adjoint with checkpoints every 10.
    "abc_128_adjoint": Workload(
        "abc_128_adjoint", (128, 128, 128), 101, 0.05, 4, 100, ("f32",),
        lambda: fields.abc_noise(128, 101, 0.05, seed=1),
        "loss weights seed 3; checkpoint every 10 steps", dict(ckpt_every=10, weight_seed=3)),
    # 512^3 turbulence (128 modes), FP16 storage, 256^3 seeds, 200 steps of dt 0.01.
    "turb_512": Workload(
        "turb_512", (512, 512, 512), 201, 0.01, 2, 200, ("f16",),
        lambda: fields.turbulence(512, 128, 4, 201, 0.01),
        "mode seed 4; two cycles resident; Jacobian on every 16th seed",
        dict(jacobian_every=16)),
}


def make_workload(name: str) -> Workload:
    return WORKLOADS[name]


def loss_weights(n_seeds: int, seed: int = 3) -> np.ndarray:
    """Seeded N(0, I_3) weights for the scalar loss sum_i w_i . x_i(T)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n_seeds, 3))


def lattice_dims(n, stride: int):
    """Seeds per axis of the lattice off + stride*k (off = (stride-1)/2) that
    stays inside [0, n-1] on each axis."""
    off = (stride - 1) / 2.0
    return tuple(int((int(nd) - 1 - off) // stride) + 1 for nd in n)


def lattice_points(n, stride: int, ids) -> np.ndarray:
    """Cell coordinates of the lattice seeds with the given ids: off + stride*k
    per axis (off = (stride-1)/2), ids x-fastest over lattice_dims(n, stride)."""
    m = lattice_dims(n, stride)
    ids = np.asarray(ids, dtype=np.int64)
    off = (stride - 1) / 2.0
    k = np.stack([ids % m[0], (ids // m[0]) % m[1], ids // (m[0] * m[1])], axis=1)
    return off + stride * k.astype(np.float64)


def row_sample_ids(m, count: int) -> np.ndarray:
    """Ids of ``count`` seeds of an x-fastest lattice of m = (mx, my, mz)
    seeds, spread over the block: the chosen rows (y, z) are every
    (my*mz // count)-th row, and the i-th chosen row gives its seed at x
    index i mod mx, so every x index appears as often as the others (plain
    strides of the id would keep x fixed whenever they divide mx)."""
    mx, rows = int(m[0]), int(m[1]) * int(m[2])
    every = max(1, rows // count)
    r = np.arange(0, rows, every, dtype=np.int64)[:count]
    return r * mx + (np.arange(len(r), dtype=np.int64) % mx)
