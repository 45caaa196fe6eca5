"""Touched grid points per step (bto_touched_points) on the GPU through the
C-ABI, against counts written out by brute force.

In a uniform flow every stage velocity is the flow's velocity, so a seed's
stage points after n steps are x0 + (n + f) h u with f in {0, 1/2, 1}: the
sampled cells are known in closed form, and the distinct corner points per
level are counted here with Python sets (level n: the cells of the first
three stages; level n + 1: those of the last three; frozen time: every stage
reads level n).  The seeds and the flow are chosen so that no stage point
comes within 1e-4 cell of a cell face during the interval, where FP32
sampling could tip a decision.  Cases: a sparse stride-4 lattice (no shared
corners), a dense stride-1 lattice (every corner shared by up to eight
particles), particles leaving the block on the way, and frozen time.  The particles
entering each step must add up to the advection's particle-step count.  On
the differentiation workload (ABC, stride 4) the counts obey the bounds the
sampler fixes: per level, at least one cell's eight corners and at most the
three cells its stages sample per live particle; at the first step, where the
stride-4 seeds lie four cells apart, no corner is shared."""

import sys

import numpy as np
import pytest

from bto_inputs import fields

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2004_02003_amd import _lib

    _lib.load()


def _cell(p, n):
    i = np.floor(p).astype(np.int64)
    return np.minimum(np.maximum(i, 0), np.asarray(n) - 2)


def _corners(cells, n):
    nx, ny, _ = n
    out = set()
    for c in cells:
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    out.add(int(c[0] + dx + nx * (c[1] + dy + ny * (c[2] + dz))))
    return out


def _inside(p, n):
    return np.all((p >= 0.0) & (p <= np.asarray(n, dtype=np.float64) - 1.0), axis=-1)


def _expected(seeds, u, h, N, n, frozen=False):
    """Per step: (level-n points, level-(n+1) points, particles entering)."""
    x = seeds.copy()
    alive = _inside(x, n)
    rows = []
    for _ in range(N):
        y2 = x + 0.5 * h * u
        y4 = x + h * u
        live = alive.copy()
        ok2 = live & _inside(y2, n)          # y3 = y2 in a uniform flow
        ok4 = ok2 & _inside(y4, n)
        c1, c2, c4 = _cell(x[live], n), _cell(y2[ok2], n), _cell(y4[ok4], n)
        if frozen:
            lv0, lv1 = _corners(np.concatenate([c1, c2, c4]), n), set()
        else:
            lv0, lv1 = _corners(np.concatenate([c1, c2]), n), _corners(np.concatenate([c2, c4]), n)
        rows.append((len(lv0), len(lv1), int(live.sum())))
        alive = ok4
        x = np.where(alive[:, None], y4, x)
    return np.array(rows, dtype=np.uint64)


def _min_face_distance(seeds, u, h, N):
    f = np.arange(0, 2 * N + 1) * 0.5
    pts = seeds[None, :, :] + f[:, None, None] * (h * u)[None, None, :]
    return float(np.abs(pts - np.round(pts)).min())


def _run(n, seeds, u, h, N, mode="linear"):
    import torch
    from paper_2004_02003_amd import Context, grid_to_device

    times = np.arange(N + 1) * h
    s = fields.uniform_flow(n, u, times)
    dev = [grid_to_device(g, "f32") for g in s.grids("f32")]
    with Context(n, len(seeds)) as ctx:
        ctx.seed_explicit(torch.as_tensor(seeds, device="cuda"))
        got = ctx.touched_points(dev, times, mode=mode)
        # the context's own advection still runs from the seeding afterwards
        ctx.advect(dev, times, mode=mode)
        st = ctx.stats()
        torch.cuda.synchronize()
    return got, st


@pytest.mark.parametrize("case", ["sparse_stride4", "dense_stride1", "leaving", "frozen"])
def test_touched_points_of_a_uniform_flow_equal_brute_force(case):
    n = (24, 20, 18)
    h = 0.25
    u = np.array([0.31, -0.17, 0.13]) * 4.0
    N = 12
    if case == "sparse_stride4":
        g = [np.arange(1.5, n[d] - 2, 4.0) for d in range(3)]
    elif case == "dense_stride1":
        g = [np.arange(2.5, n[d] - 3, 1.0) for d in range(3)]
    elif case == "leaving":
        u = np.array([0.31, -0.17, 0.13]) * 16.0
        g = [np.arange(1.5, n[d] - 1, 2.0) for d in range(3)]
    else:
        g = [np.arange(1.5, n[d] - 2, 3.0) for d in range(3)]
    z, y, x = np.meshgrid(g[2], g[1], g[0], indexing="ij")
    seeds = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float64)
    assert _min_face_distance(seeds, u, h, N) > 1e-4, "a stage point lies on a cell face"
    _say(f"touched points, uniform flow, {case}: {len(seeds)} seeds")
    exp = _expected(seeds, u, h, N, n, frozen=case == "frozen")
    got, st = _run(n, seeds, u, h, N, mode="frozen" if case == "frozen" else "linear")
    assert np.array_equal(got, exp), f"{case}: got\n{got}\nexpected\n{exp}"
    # the particles entering each step sum to the particle-steps of the advection
    assert int(got[:, 2].sum()) == st["particle_steps"]
    if case == "leaving":
        assert exp[-1, 2] < exp[0, 2]
    if case == "frozen":
        assert np.all(got[:, 1] == 0)


def test_touched_points_of_the_differentiation_workload():
    import torch
    from bto_inputs.workloads import WORKLOADS
    from paper_2004_02003_amd import Context, grid_to_device

    wl = WORKLOADS["abc_128_adjoint"]
    s = wl.make_field()
    dev = [grid_to_device(g, "f32") for g in s.grids("f32")]
    with Context(wl.n, wl.n_seeds) as ctx:
        ctx.seed(wl.stride)
        got = ctx.touched_points(dev, s.times)
        ctx.advect(dev, s.times)
        st = ctx.stats()
        torch.cuda.synchronize()
    _say(f"abc_128_adjoint touched points: first {got[0]}, last {got[-1]}")
    live = got[:, 2].astype(np.int64)
    assert int(live.sum()) == st["particle_steps"]
    for lv in (0, 1):
        pts = got[:, lv].astype(np.int64)
        # at least one cell, at most the three cells a level's stages sample, per live particle
        assert np.all(pts >= 8 * (live > 0)) and np.all(pts <= 24 * live)
    # stride 4: particles 4 cells apart on a slow flow share no corners at first
    assert got[0, 0] >= 8 * got[0, 2]
