"""The tile layout (tile-staged steps) on the GPU through the C-ABI.

With ``tiles=1`` every step stages a tile of cells plus a 2-cell halo of both
grid levels in LDS and samples from there; particles whose stage points leave
the staged box are stepped from the grids by a second launch, and survivors
move to the bucket of the tile they end in.  ``tiles=2`` keeps the tile
layout and order but gathers from the grids.  The arithmetic is the one of the
segment layout, so the flow map must equal, bit for bit, the one of the
segment layout run one step per launch (the same FP32 re-rounding of the
in-cell offset after every step), and agree with the FP64 oracle as every
other configuration does.  The cases cover slow and fast flows (few and many
deferred particles), every storage type and both time modes, ragged blocks,
seeds crowded into a few tiles (bucket overflow into the list), exit points,
streaming calls, a flow map read in the middle of an interval, recorded
checkpoints for the adjoint, blocks at the largest axis length along each axis,
uneven step sizes, intervals without live particles, and the refusal of a storage type with
another tile size inside one interval."""

import sys

import numpy as np
import pytest

import oracle
from bto_inputs import fields

from .parity import compare, oracle_lattice, run_gpu

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


def _dev(grids, dtype):
    from paper_2004_02003_amd import grid_to_device

    return [grid_to_device(g, dtype) for g in grids]


def _same(a, b, label):
    assert np.array_equal(a["flag"], b["flag"]), f"{label}: flags differ"
    assert np.array_equal(a["exit"], b["exit"]), f"{label}: exit steps differ"
    assert np.array_equal(a["end"], b["end"]), f"{label}: end positions differ (max {np.abs(a['end'] - b['end']).max()})"
    assert a["stats"]["particle_steps"] == b["stats"]["particle_steps"], label
    assert a["n_valid"] == b["n_valid"], label


def _pair(n, dev, times, label, **kw):
    """Tile layout (LDS-staged, and gathering in tile order) vs segment layout
    at one step per launch."""
    _say(f"tiles: {label}")
    s = run_gpu(n, dev, times, tuning=dict(steps_per_launch=1), **kw)
    for tiles in (1, 2):
        t = run_gpu(n, dev, times, tuning=dict(tiles=tiles), **kw)
        _same(t, s, f"{label} (tiles={tiles})")
    return t


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
def test_tiles_turbulence_every_storage_type(dt):
    # 1.5 cells per step: many stage points leave their tile's staged box
    n = (72, 61, 50)
    N = 12
    s = fields.turbulence(n, 24, 21, N + 1, 0.02, L=72)
    gr = s.grids(dt)
    g = _pair(n, _dev(gr, dt), s.times, f"turbulence {n} {dt}", stride=2, record_exit=True)
    seeds, o = oracle_lattice(oracle.Field(n, gr, dtype=dt), s.times, n, 2, N, jac=True)
    # FP32 sampling errors stretched by the flow map (first-order bound, J from the oracle)
    vmax = max(float(np.abs(q).max()) for q in s.grids("f32")) * np.sqrt(3.0)
    tol = np.linalg.norm(o["jac"], axis=(1, 2), ord=2) * N * 0.02 * vmax * 2.0 ** -21
    res = compare(g, o, label=f"tiles turbulence {dt}", per_particle_tol=tol, seeds=seeds, n=n)
    assert 0.05 < res["terminated"] < 0.95


@pytest.mark.parametrize("mode", ["linear", "frozen"])
def test_tiles_double_gyre_both_time_modes(mode):
    from bto_inputs.workloads import WORKLOADS

    wl = WORKLOADS["double_gyre_32"]
    s = wl.make_field()
    gr = s.grids("f32")
    g = _pair(wl.n, _dev(gr, "f32"), s.times, f"double gyre {mode}", stride=2, mode=mode)
    seeds, o = oracle_lattice(oracle.Field(wl.n, gr), s.times, wl.n, 2, wl.n_steps,
                              mode=oracle.FROZEN if mode == "frozen" else oracle.LINEAR)
    compare(g, o, label=f"tiles double gyre {mode}", seeds=seeds, n=wl.n)


def test_tiles_ragged_block_stride_3_and_streaming():
    n = (37, 23, 19)
    N = 12
    s = fields.abc_noise(n, N + 1, 0.1, sigma=0.05, seed=12, global_n=48)
    for dt in ("f32", "f16"):
        gr = s.grids(dt)
        dev = _dev(gr, dt)
        g = _pair(n, dev, s.times, f"ragged {dt}", stride=3, chunks=[1] * N, record_exit=True)
        seeds, o = oracle_lattice(oracle.Field(n, gr, dtype=dt), s.times, n, 3, N)
        compare(g, o, label=f"tiles ragged {dt}", seeds=seeds, n=n)


def test_tiles_crowded_seeds_overflow_their_buckets():
    # 6,000 seeds in a 3x3x3-cell region that at most four gathering tiles
    # (32 x 8 x 8 cells) or one staged tile share: the bucket capacity (twice
    # the mean per tile plus 32) is exceeded, the rest waits in the list
    rng = np.random.default_rng(5)
    n = (40, 40, 40)
    N = 10
    s = fields.turbulence(n, 16, 3, N + 1, 0.02, L=40, cfl=0.8)
    seeds = np.concatenate([rng.uniform(14.0, 17.0, size=(6000, 3)), rng.uniform(0.5, 38.5, size=(2000, 3))])
    gr = s.grids("f16")
    g = _pair(n, _dev(gr, "f16"), s.times, "crowded seeds", seeds=seeds)
    o = oracle.flowmap(oracle.Field(n, gr, dtype="f16"), s.times, seeds, N)
    compare(g, o, label="tiles crowded")


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_tiles_at_the_largest_block_axis(axis):
    """A block 1,024 points long along one axis (the 10-bit cell index of the
    packed state) in uniform flow along that axis: both tile layouts equal the
    segment layout, a stride-3 lattice matches the oracle, and seeds over the
    whole long axis, the last cells included, end at x0 + u t or terminate in
    the step that would cross the far face, as the closed form says."""
    n = [12, 10, 9]
    n[axis] = 1024
    n = tuple(n)
    N = 8
    times = np.arange(N + 1) * 0.25
    u = np.zeros(3)
    u[axis] = 3.7
    s = fields.uniform_flow(n, u, times)
    gr = s.grids("f32")
    dev = _dev(gr, "f32")
    _pair(n, dev, times, f"long axis {axis}: lattice", stride=3)
    g = run_gpu(n, dev, times, stride=3, tuning=dict(tiles=2))
    seeds, o = oracle_lattice(oracle.Field(n, gr), times, n, 3, N)
    compare(g, o, label=f"tiles, long axis {axis}", seeds=seeds, n=n)
    xs = np.array([0.3, 500.5, 1000.0, 1015.2, 1016.9, 1019.0, 1021.7, 1022.99])
    seeds = np.tile([[5.5, 4.5, 4.0]], (len(xs), 1))
    seeds[:, axis] = xs
    ge = _pair(n, dev, times, f"long axis {axis}: explicit seeds", seeds=seeds)
    ux = float(np.float32(3.7))
    for i, x0 in enumerate(xs):
        ends = x0 + ux * (times[1:] - times[0])
        inside = ends <= 1023.0
        e = N if inside.all() else int(np.argmin(inside))
        assert ge["exit"][i] == e, (axis, x0, ge["exit"][i], e)
        assert abs(ge["end"][i, axis] - (x0 + ux * (times[e] - times[0]))) < 1e-5


def test_tiles_non_uniform_steps_closed_form():
    """Uneven step sizes (one h per step call) in uniform flow: both tile
    layouts equal the segment layout, match the oracle, end valid particles at
    x0 + u (t_N - t_0), and place exit points where the straight line leaves
    the block."""
    rng = np.random.default_rng(11)
    n = (44, 21, 19)
    N = 24
    times = np.concatenate([[0.5], 0.5 + np.cumsum(rng.uniform(0.2, 0.9, N))])
    u = np.array([1.3, -0.35, 0.4])
    s = fields.uniform_flow(n, u, times)
    gr = s.grids("f32")
    g = _pair(n, _dev(gr, "f32"), times, "uneven steps", stride=2, record_exit=True)
    seeds, o = oracle_lattice(oracle.Field(n, gr), times, n, 2, N)
    res = compare(g, o, label="tiles uneven steps", seeds=seeds, n=n)
    assert 0.0 < res["terminated"] < 1.0
    valid = g["flag"] == oracle.VALID
    np.testing.assert_allclose(g["end"][valid], seeds[valid] + u * (times[-1] - times[0]), atol=1e-5)
    hi = np.array(n, dtype=float) - 1
    t_face = np.where(u > 0, (hi - seeds) / u, np.where(u < 0, -seeds / u, np.inf))
    t_sorted = np.sort(t_face, axis=1)
    term = (g["flag"] == oracle.TERMINATED) & (t_sorted[:, 1] - t_sorted[:, 0] > 1e-6)
    assert term.sum() > 100
    np.testing.assert_allclose(g["face"][term], (seeds + u * t_sorted[:, :1])[term], atol=1e-5)


def test_intervals_without_live_particles():
    """Degenerate intervals in each layout: seeds that all lie outside the
    block (terminated at step 0 where they were placed, no exit point, no
    particle-step counted), and no seeds at all (empty flow map, exit points
    and seed gradients, with the empty tensors' null data pointers)."""
    import torch
    from paper_2004_02003_amd import Context

    n = (40, 20, 18)
    N = 6
    s = fields.abc_noise(n, N + 1, 0.1, sigma=0.0, seed=3, global_n=48)
    gr = s.grids("f16")
    dev = _dev(gr, "f16")
    outside = np.array([[-0.5, 3, 3], [39.01, 5, 5], [5, -2, 5], [5, 5, 17.5], [1e9, 0, 0]], dtype=np.float64)
    for tiles in (0, 1, 2):
        tuning = dict(tiles=tiles) if tiles else dict(steps_per_launch=1)
        _say(f"no live particles, tiles={tiles}")
        g = run_gpu(n, dev, s.times, seeds=outside, tuning=tuning, record_exit=True)
        assert np.all(g["flag"] == 1) and np.all(g["exit"] == 0)
        assert np.array_equal(g["end"], outside)
        assert np.all(np.isnan(g["face"]))
        assert g["stats"]["particle_steps"] == 0 and g["n_valid"] == 0
        with Context(n, 1) as ctx:
            ctx.set_tuning(**tuning)
            assert ctx.seed_explicit(torch.empty((0, 3), dtype=torch.float64, device="cuda")) == 0
            ctx.advect(dev, s.times)
            fm = ctx.flowmap(count_valid=True)
            assert tuple(fm["end"].shape) == (0, 3) and fm["n_valid"] == 0
            assert tuple(ctx.exit_points().shape) == (0, 3)
            gs = ctx.adjoint(dev, s.times, torch.empty((0, 1, 3), dtype=torch.float32, device="cuda"))
            assert gs.shape[0] == 0
            st = ctx.stats()
            torch.cuda.synchronize()
            assert st["particle_steps"] == 0 and st["n_live"] == 0 and st["steps_done"] == N


def test_tiles_flowmap_mid_interval_and_recorded_checkpoints():
    import torch
    from paper_2004_02003_amd import Context

    n = (48, 40, 36)
    N = 20
    s = fields.turbulence(n, 16, 8, N + 1, 0.02, L=48)
    gr = s.grids("f32")
    dev = _dev(gr, "f32")
    seeds, o = oracle_lattice(oracle.Field(n, gr), s.times, n, 3, N, jac=True)
    w = torch.as_tensor(np.random.default_rng(4).standard_normal((len(seeds), 3)), dtype=torch.float32,
                        device="cuda").contiguous()
    out = {}
    for tiles in (0, 1, 2):
        _say(f"tiles={tiles}: flow map mid-interval, recorded checkpoints")
        with Context(n, len(seeds)) as ctx:
            ctx.set_tuning(tiles=tiles, steps_per_launch=1, ckpt_every=5)
            ctx.seed(3)
            ctx.advect(dev[:8], s.times[:8], record_ckpt=True)
            mid = {k: v.cpu().numpy() for k, v in ctx.flowmap().items()}
            ctx.advect(dev[7:], s.times[7:], record_ckpt=True)
            fm = {k: v.cpu().numpy() for k, v in ctx.flowmap().items()}
            g = ctx.adjoint(dev, s.times, w, ckpt_every=5, recorded=True).cpu().numpy()
            torch.cuda.synchronize()
            out[tiles] = (mid, fm, g)
    for tiles in (1, 2):
        for k in ("end", "flag", "exit"):
            assert np.array_equal(out[0][0][k], out[tiles][0][k]), f"mid-interval {k} (tiles={tiles})"
            assert np.array_equal(out[0][1][k], out[tiles][1][k]), f"end of interval {k} (tiles={tiles})"
        assert np.array_equal(out[0][2], out[tiles][2]), f"seed gradients from recorded checkpoints (tiles={tiles})"
    fm = dict(out[1][1])
    vmax = max(float(np.abs(q).max()) for q in gr) * np.sqrt(3.0)
    tol = np.linalg.norm(o["jac"], axis=(1, 2), ord=2) * N * 0.02 * vmax * 2.0 ** -21
    compare(fm, o, label="tiles mid-interval", per_particle_tol=tol, seeds=seeds, n=n)


def test_tiles_refuse_a_storage_type_of_another_tile_size():
    import torch
    from paper_2004_02003_amd import Context, _lib
    from paper_2004_02003_amd.context import BTOError

    n = (30, 30, 30)
    s = fields.uniform_flow(n, np.array([0.3, 0.2, -0.1]), np.arange(4) * 0.5)
    d16 = _dev(s.grids("f16"), "f16")
    d32 = _dev(s.grids("f32"), "f32")
    with Context(n, 4000) as ctx:
        ctx.set_tuning(tiles=1)
        ctx.seed(2)
        ctx.advect(d16[:2], s.times[:2])
        with pytest.raises(BTOError) as e:
            ctx.advect(d32[1:3], s.times[1:3])
        assert e.value.code == _lib.BTO_EINVAL and "tile" in str(e.value)
        ctx.advect(d16[1:], s.times[1:])
        fm = ctx.flowmap(count_valid=True)
        torch.cuda.synchronize()
        assert ctx.stats()["steps_done"] == 3
    o = oracle.flowmap(oracle.Field(n, s.grids("f16"), dtype="f16"), s.times, oracle.seed_lattice(n, 2), 3)
    assert np.array_equal(fm["flag"].cpu().numpy(), o["flag"])
    # gathering tiles have one size for every storage type: mixing is allowed,
    # with the same result as the segment layout run one step per launch
    res = {}
    for tune in (dict(tiles=2), dict(steps_per_launch=1)):
        with Context(n, 4000) as ctx:
            ctx.set_tuning(**tune)
            ctx.seed(2)
            ctx.advect(d16[:2], s.times[:2])
            ctx.advect(d32[1:3], s.times[1:3])
            fm = ctx.flowmap(count_valid=True)
            torch.cuda.synchronize()
            assert ctx.stats()["steps_done"] == 2
            res[tuple(tune)] = {k: v.cpu().numpy() for k, v in fm.items() if k != "n_valid"}
    a, b = res[("tiles",)], res[("steps_per_launch",)]
    assert np.array_equal(a["end"], b["end"]) and np.array_equal(a["flag"], b["flag"])
