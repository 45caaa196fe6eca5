"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Flags and exit steps must match exactly outside a 1e-6-cell face margin; end
positions within 1e-5 cells (FP32 arithmetic on the stored grid; FP64
positions).  Inputs are seeded synthetic fields; every expected value comes
from the oracle run on the very same stored grid values.
"""

import math
import os
import sys

import numpy as np
import pytest

import oracle
from bto_inputs import fields, quant
from bto_inputs.workloads import WORKLOADS

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

    _lib.load()  # fails loudly if the library is missing


def _dev(grids, dtype):
    from paper_2004_02003_amd import grid_to_device

    return [grid_to_device(g, dtype) for g in grids]


def test_seeding_without_steps_returns_the_seeds():
    _say("seed-only 37x23x19 stride 3")
    n = (37, 23, 19)
    import torch
    from paper_2004_02003_amd import Context

    with Context(n, 5000) as ctx:
        P = ctx.seed(3)
        fm = ctx.flowmap(count_valid=True)
        torch.cuda.synchronize()
    seeds = oracle.seed_lattice(n, 3)
    assert P == len(seeds) and fm["n_valid"] == P
    assert np.array_equal(fm["seed"].cpu().numpy(), seeds)
    assert np.array_equal(fm["end"].cpu().numpy(), seeds)
    assert np.all(fm["flag"].cpu().numpy() == 0) and np.all(fm["exit"].cpu().numpy() == 0)


def test_uniform_flow_closed_form_on_gpu():
    _say("uniform flow 20^3 non-uniform steps")
    rng = np.random.default_rng(7)
    n = (20, 20, 20)
    N = 30
    times = np.concatenate([[0.25], 0.25 + np.cumsum(rng.uniform(0.1, 0.5, N))])
    u = np.array([0.7, -0.3, 0.45])
    s = fields.uniform_flow(n, u, times)
    g = run_gpu(n, _dev(s.grids("f32"), "f32"), times, stride=3, record_exit=True)
    o = oracle.flowmap(oracle.Field(n, s.grids("f32")), times, oracle.seed_lattice(n, 3), N)
    res = compare(g, o, label="uniform", seeds=oracle.seed_lattice(n, 3), n=n)
    assert g["stats"]["particle_steps"] == int(np.where(o["flag"] == 0, N, o["exit"] + 1).sum())
    # exit points: where the straight line x0 + u t leaves the box
    seeds = oracle.seed_lattice(n, 3)
    hi = np.array(n, dtype=float) - 1
    t_face = np.where(u > 0, (hi - seeds) / u, np.where(u < 0, -seeds / u, np.inf))
    t_sorted = np.sort(t_face, axis=1)
    term = (g["flag"] == oracle.TERMINATED) & (t_sorted[:, 1] - t_sorted[:, 0] > 1e-6)
    line = seeds + u * t_sorted[:, :1]
    assert term.sum() > 100 and res["exit_points"] > 100
    np.testing.assert_allclose(g["face"][term], line[term], atol=1e-5)
    assert np.all(np.isnan(g["face"][g["flag"] == oracle.VALID]))


def test_solid_body_rotation_on_gpu():
    _say("solid-body rotation 16x16x6")
    n = (16, 16, 6)
    N = 40
    times = np.arange(N + 1) * 0.125
    s = fields.solid_body_rotation(n, 0.5, (7.5, 7.5), 0.05, times)
    rng = np.random.default_rng(2)
    r0 = rng.uniform(0.5, 6.0, 300)
    ph = rng.uniform(0, 2 * math.pi, 300)
    seeds = np.stack([7.5 + r0 * np.cos(ph), 7.5 + r0 * np.sin(ph), np.full(300, 1.5)], axis=1)
    g = run_gpu(n, _dev(s.grids("f32"), "f32"), times, seeds=seeds)
    th = 0.5 * 0.125
    R = 1 + 1j * th + (1j * th) ** 2 / 2 + (1j * th) ** 3 / 6 + (1j * th) ** 4 / 24
    zN = ((seeds[:, 0] - 7.5) + 1j * (seeds[:, 1] - 7.5)) * R ** N
    assert np.all(g["flag"] == 0)
    np.testing.assert_allclose(g["end"][:, 0], 7.5 + zN.real, atol=1e-5)
    np.testing.assert_allclose(g["end"][:, 1], 7.5 + zN.imag, atol=1e-5)


def test_double_gyre_full_parity():
    wl = WORKLOADS["double_gyre_32"]
    _say(f"{wl.name} full")
    s = wl.make_field()
    gr = s.grids("f32")
    g = run_gpu(wl.n, _dev(gr, "f32"), s.times, stride=wl.stride, record_exit=True)
    _, o = oracle_lattice(oracle.Field(wl.n, gr), s.times, wl.n, wl.stride, wl.n_steps)
    res = compare(g, o, label=wl.name)
    assert 0.15 < res["terminated"] < 0.35
    assert g["n_valid"] == int((o["flag"] == 0).sum()) or res["ambiguous"] > 0


def test_double_gyre_frozen_mode_parity():
    wl = WORKLOADS["double_gyre_32"]
    _say(f"{wl.name} frozen")
    s = wl.make_field()
    gr = s.grids("f32")
    g = run_gpu(wl.n, _dev(gr, "f32"), s.times, stride=wl.stride, mode="frozen")
    _, o = oracle_lattice(oracle.Field(wl.n, gr), s.times, wl.n, wl.stride, wl.n_steps, mode=oracle.FROZEN)
    compare(g, o, label="frozen")


def test_streaming_one_call_per_cycle_matches_one_call():
    wl = WORKLOADS["double_gyre_32"]
    _say("double gyre streaming (2 grids per call)")
    s = wl.make_field()
    gr = s.grids("f32")
    dev = _dev(gr, "f32")
    a = run_gpu(wl.n, dev, s.times, stride=2)
    b = run_gpu(wl.n, dev, s.times, stride=2, chunks=[1] * wl.n_steps)
    c = run_gpu(wl.n, dev, s.times, stride=2, chunks=[7, 33, 10])
    _, o = oracle_lattice(oracle.Field(wl.n, gr), s.times, wl.n, 2, wl.n_steps, jac=True)
    # Each launch re-rounds the position to the stored state (<= 2^-33 cells),
    # which can move a later stage point across a cell face, where the FP32
    # sampler rounds differently: two runs differ by at most twice the
    # first-order FP32 sampling bound ||J|| N h max|V| 2^-21 (J from the oracle)
    vmax = float(np.abs(gr).max()) * np.sqrt(3.0)
    h = float(s.times[1] - s.times[0])
    tol = 1e-7 + 2.0 * np.linalg.norm(o["jac"], axis=(1, 2), ord=2) * wl.n_steps * h * vmax * 2.0 ** -21
    for r, lab in ((b, "per-cycle"), (c, "ragged chunks")):
        compare(r, o, label=lab)
        amb = o["margin"] < 1e-6
        assert np.array_equal(r["flag"][~amb], a["flag"][~amb])
        d = np.abs(r["end"] - a["end"]).max(axis=1)
        ok = ~amb & (o["flag"] == 0)
        assert np.all(d[ok] <= tol[ok]), f"{lab}: {d[ok].max():.3e} beyond {tol[ok][np.argmax(d[ok] - tol[ok])]:.3e}"
        _say(f"{lab}: max |one call - streamed| {d[ok].max():.2e}, median bound {np.median(tol[ok]):.2e}")


def test_ragged_block_and_lattice_all_dtypes():
    n = (37, 23, 19)
    N = 12
    s = fields.abc_noise(n, N + 1, 0.1, sigma=0.05, seed=12, global_n=48)
    for dt in ("f32", "f16", "bf16"):
        _say(f"ragged 37x23x19 stride 3 {dt}")
        gr = s.grids(dt)
        g = run_gpu(n, _dev(gr, dt), s.times, stride=3, record_exit=True)
        sd, o = oracle_lattice(oracle.Field(n, gr, dtype=dt), s.times, n, 3, N)
        res = compare(g, o, label=dt, seeds=sd, n=n)
        assert 0.0 < res["terminated"] < 1.0


def test_explicit_seeds_including_outside_and_permutation():
    n = (24, 24, 24)
    N = 16
    s = fields.abc_noise(n, N + 1, 0.05, sigma=0.02, seed=9, global_n=64)
    gr = s.grids("f32")
    rng = np.random.default_rng(5)
    seeds = rng.uniform(-1.0, 24.0, size=(3000, 3))
    seeds[:10] = [[0, 0, 0], [23, 23, 23], [23, 0, 11.5], [-1e-9, 3, 3], [3, 23.0000001, 3],
                  [11.5, 11.5, 11.5], [0.5, 0.5, 0.5], [22.5, 22.5, 22.5], [5, 5, 23], [23, 5, 5]]
    _say("explicit seeds 3000 (with outside)")
    g = run_gpu(n, _dev(gr, "f32"), s.times, seeds=seeds, record_exit=True)
    o = oracle.flowmap(oracle.Field(n, gr), s.times, seeds, N)
    compare(g, o, label="explicit")
    outside = ~np.all((seeds >= 0) & (seeds <= 23), axis=1)
    assert np.all(g["flag"][outside] == 1) and np.all(g["exit"][outside] == 0)
    assert np.array_equal(g["end"][outside], seeds[outside])
    assert np.all(np.isnan(g["face"][outside]))  # no exit point for seeds outside the block
    perm = rng.permutation(len(seeds))
    _say("explicit seeds permuted")
    gp = run_gpu(n, _dev(gr, "f32"), s.times, seeds=seeds[perm], record_exit=True)
    assert np.array_equal(gp["flag"], g["flag"][perm])
    assert np.array_equal(gp["exit"], g["exit"][perm])
    assert np.array_equal(gp["end"], g["end"][perm])
    assert np.array_equal(gp["face"], g["face"][perm], equal_nan=True)
    # the gathering tile layout bins the same seeds by tile: same parity,
    # and its flow map is just as independent of the seed order
    _say("explicit seeds, gathering tiles (and permuted)")
    gt = run_gpu(n, _dev(gr, "f32"), s.times, seeds=seeds, record_exit=True, tuning=dict(tiles=2))
    compare(gt, o, label="explicit, tiles")
    assert np.array_equal(gt["flag"][outside], g["flag"][outside]) and np.array_equal(gt["end"][outside], seeds[outside])
    gtp = run_gpu(n, _dev(gr, "f32"), s.times, seeds=seeds[perm], record_exit=True, tuning=dict(tiles=2))
    for k in ("flag", "exit", "end"):
        assert np.array_equal(gtp[k], gt[k][perm]), k
    assert np.array_equal(gtp["face"], gt["face"][perm], equal_nan=True)


def test_world_coordinates_origin_and_spacing():
    n = (20, 16, 12)
    N = 10
    s = fields.abc_noise(n, N + 1, 0.05, sigma=0.02, seed=10, global_n=40)
    gr = s.grids("f32")
    origin = np.array([-3.0, 10.5, 2.25])
    spacing = np.array([0.5, 2.0, 0.25])
    # a grid in world units per time: cell velocity times spacing
    grw = [(quant.promote(g, "f32") * spacing).astype(np.float32) for g in gr]
    cells = [(quant.promote(g2, "f32") / spacing) for g2 in grw]
    _, o = oracle_lattice(oracle.Field(n, cells), s.times, n, 2, N)
    dev = _dev(grw, "f32")
    one_step = None
    # every layout writes world coordinates: fused segments, one step per
    # launch, and both tile layouts (their own flow-map writer), which equal
    # the one-step segment run bit for bit
    for tuning in (None, dict(steps_per_launch=1), dict(tiles=1), dict(tiles=2)):
        _say(f"origin/spacing 20x16x12 {tuning}")
        g = run_gpu(n, dev, s.times, stride=2, origin=origin, spacing=spacing, record_exit=True, tuning=tuning)
        g_cells = dict(g)
        g_cells["end"] = (g["end"] - origin) / spacing
        g_cells["face"] = (g["face"] - origin) / spacing
        compare(g_cells, o, label=f"world {tuning}")
        np.testing.assert_allclose((g["seed"] - origin) / spacing, oracle.seed_lattice(n, 2), atol=0)
        if tuning == dict(steps_per_launch=1):
            one_step = g
        elif tuning is not None:
            for k in ("flag", "exit", "end"):
                assert np.array_equal(g[k], one_step[k]), (tuning, k)
            assert np.array_equal(g["face"], one_step["face"], equal_nan=True), tuning


def test_nonfinite_velocity_flags_invalid_on_gpu():
    n = (10, 10, 10)
    s = fields.uniform_flow(n, [0.5, 0.0, 0.0], np.arange(6) * 0.2)
    gs = s.grids("f32")
    gs[2][5, 5, 5] = np.nan
    seeds = np.array([[4.0, 5.0, 5.0], [4.0, 2.0, 2.0]])
    dev = _dev(gs, "f32")
    for tuning in (None, dict(tiles=1), dict(tiles=2)):  # every layout
        _say(f"nan field {tuning}")
        g = run_gpu(n, dev, s.times, seeds=seeds, tuning=tuning)
        assert g["flag"].tolist() == [2, 0] and g["exit"][0] == 1, tuning
        assert np.all(np.isfinite(g["end"]))
        np.testing.assert_allclose(g["end"][0], [4.1, 5.0, 5.0], atol=1e-6)
        assert g["stats"]["particle_steps"] == 2 + len(s.times) - 1, tuning  # the INVALID step counts


def test_abc_128_full_size_sampled_parity():
    wl = WORKLOADS["abc_128"]
    _say(f"{wl.name} full size, oracle on every 5th seed")
    s = wl.make_field()
    gr = s.grids("f32")
    g = run_gpu(wl.n, _dev(gr, "f32"), s.times, stride=wl.stride)
    ids = np.arange(0, wl.n_seeds, 5)
    _, o = oracle_lattice(oracle.Field(wl.n, gr), s.times, wl.n, wl.stride, wl.n_steps, ids=ids)
    sub = {k: g[k][ids] for k in ("end", "flag", "exit")}
    res = compare(sub, o, label=wl.name)
    _say(f"{wl.name}: {res}")
    assert 0.08 < res["terminated"] < 0.25
    # whole-population properties: every seed accounted for, counts consistent
    assert g["n_valid"] == int((g["flag"] == 0).sum())
    assert g["stats"]["n_live"] == g["n_valid"]
    assert np.all(g["exit"][g["flag"] == 0] == wl.n_steps)
    steps = np.where(g["flag"] == 0, wl.n_steps, g["exit"] + 1).sum()
    assert g["stats"]["particle_steps"] == steps


def test_insitu_driver_consecutive_intervals_match_oracle():
    """Three non-overlapping intervals of 16 cycles fed one grid per cycle
    (two-slot ring copy); each interval's flow map matches the oracle started
    at that interval's first cycle with fresh seeds."""
    import torch
    from paper_2004_02003_amd import Context, InSituDriver

    wl = WORKLOADS["double_gyre_32"]
    _say("in situ driver, 3 intervals of 16")
    s = wl.make_field()
    gr = s.grids("f32")
    maps = {}

    def keep(idx, fm, t0, t1):
        maps[idx] = ({k: v.cpu().numpy() for k, v in fm.items()}, t0, t1)

    with Context(wl.n, wl.n_seeds) as ctx:
        drv = InSituDriver(ctx, interval=16, stride=2, copy=True, on_flowmap=keep)
        src = torch.empty((32, 32, 32, 3), dtype=torch.float32, device="cuda")
        for c in range(49):
            src.copy_(torch.from_numpy(gr[c]))  # the "simulation" overwrites its buffer every cycle
            drv.cycle(src, float(s.times[c]))
        torch.cuda.synchronize()
        assert drv.intervals_done == 3 and drv.mean_cycle_ms() > 0
    seeds = oracle.seed_lattice(wl.n, 2)
    F = oracle.Field(wl.n, gr)
    for idx in range(3):
        fm, t0, t1 = maps[idx]
        assert t0 == s.times[16 * idx] and t1 == s.times[16 * (idx + 1)]
        o = oracle.flowmap(F, s.times, seeds, 16, first_cycle=16 * idx)
        compare(fm, o, label=f"interval {idx}")



def test_insitu_driver_overlapped_ingest_matches_serial():
    """Copy on an ingest stream into a three-slot ring, advection on the
    driver's compute stream: the same flow maps, bit for bit, as the serial
    two-slot driver, with the simulation overwriting its buffer every cycle."""
    import torch
    from paper_2004_02003_amd import Context, InSituDriver

    wl = WORKLOADS["double_gyre_32"]
    _say("in situ driver, overlapped ingest vs serial")
    s = wl.make_field()
    gr = s.grids("f32")
    host = [torch.from_numpy(g).pin_memory() for g in gr[:49]]
    results = {}
    for overlap in (False, True):
        maps = {}

        def keep(idx, fm, t0, t1, _m=maps):
            _m[idx] = {k: v.cpu().numpy() for k, v in fm.items()}

        with Context(wl.n, wl.n_seeds) as ctx:
            drv = InSituDriver(ctx, interval=16, stride=2, copy=True, overlap=overlap, on_flowmap=keep)
            src = torch.empty((32, 32, 32, 3), dtype=torch.float32, device="cuda")
            for c in range(49):
                src.copy_(host[c], non_blocking=True)  # the "simulation" rewrites its buffer every cycle
                drv.cycle(src, float(s.times[c]))
            drv.synchronize()
            torch.cuda.synchronize()
            assert drv.intervals_done == 3 and drv.mean_cycle_ms() > 0
        results[overlap] = maps
    for idx in range(3):
        for k in ("end", "flag", "exit"):
            assert np.array_equal(results[True][idx][k], results[False][idx][k]), (idx, k)
    with pytest.raises(ValueError):
        InSituDriver(None, interval=4, stride=2, copy=False, overlap=True)

def test_rebin_between_launches_keeps_results():
    """Re-sorting live particles by brick between launches changes only their
    order: the seed-ordered flow map matches the oracle and the run without
    re-sorting."""
    import os

    n = (40, 36, 44)
    N = 30
    s = fields.abc_noise(n, N + 1, 0.05, sigma=0.05, seed=21, global_n=48)
    gr = s.grids("f32")
    dev = _dev(gr, "f32")
    _say("rebin every 4 steps, 40x36x44")
    a = run_gpu(n, dev, s.times, stride=2)
    os.environ["BTO_REBIN_EVERY"] = "4"
    try:
        b = run_gpu(n, dev, s.times, stride=2)
        c = run_gpu(n, dev, s.times, stride=2, chunks=[3, 9, 1, 17], record_exit=True)
    finally:
        del os.environ["BTO_REBIN_EVERY"]
    _, o = oracle_lattice(oracle.Field(n, gr), s.times, n, 2, N)
    for r, lab in ((b, "rebin"), (c, "rebin, ragged calls")):
        res = compare(r, o, label=lab)
        assert 0.05 < res["terminated"] < 0.9
        amb = o["margin"] < 1e-6
        assert np.array_equal(r["flag"][~amb], a["flag"][~amb])
        assert np.abs(r["end"] - a["end"]).max() < 5e-6
        assert r["stats"]["particle_steps"] == a["stats"]["particle_steps"] or amb.any()


def test_two_lanes_per_particle_matches_oracle_and_one_lane():
    """Pairs of lanes per particle (each lane weights one x-corner of every
    cell row, the pair adds its partial sums): same events as the oracle and
    as one lane per particle, positions within FP32 rounding of both.  An odd
    seed count leaves a half-filled last batch; rebinning and ragged calls
    move particles between pairs and launches."""
    n = (40, 36, 44)
    N = 30
    s = fields.abc_noise(n, N + 1, 0.05, sigma=0.05, seed=23, global_n=48)
    gr = s.grids("f32")
    dev = _dev(gr, "f32")
    rng = np.random.default_rng(5)
    seeds = rng.uniform(0.0, 1.0, size=(4001, 3)) * (np.array(n) - 1)
    _say("two lanes per particle, 40x36x44, 4001 seeds")
    a = run_gpu(n, dev, s.times, seeds=seeds)
    b = run_gpu(n, dev, s.times, seeds=seeds, tuning=dict(lanes_per_particle=2))
    c = run_gpu(n, dev, s.times, seeds=seeds, chunks=[3, 9, 1, 17],
                tuning=dict(lanes_per_particle=2, rebin_every=4, steps_per_launch=7), record_exit=True)
    o = oracle.flowmap(oracle.Field(n, gr), s.times, seeds, N)
    amb = o["margin"] < 1e-6
    for r, lab in ((b, "2 lanes"), (c, "2 lanes, rebin, ragged calls")):
        res = compare(r, o, label=lab)
        assert 0.05 < res["terminated"] < 0.9
        assert np.array_equal(r["flag"][~amb], a["flag"][~amb])
        assert np.abs(r["end"] - a["end"]).max() < 5e-6
        assert r["n_valid"] == int((r["flag"] == 0).sum())
        assert r["stats"]["particle_steps"] == a["stats"]["particle_steps"] or amb.any()


def test_exit_points_only_for_calls_that_record_them():
    """Exit points are kept for particles terminated by a call made with
    BTO_RECORD_EXIT; particles terminated by other calls (and every seed
    before any call) read NaN.  Recording changes nothing else."""
    import torch
    from paper_2004_02003_amd import Context

    n = (20, 20, 20)
    N = 30
    rng = np.random.default_rng(7)
    times = np.concatenate([[0.25], 0.25 + np.cumsum(rng.uniform(0.1, 0.5, N))])
    s = fields.uniform_flow(n, np.array([0.7, -0.3, 0.45]), times)
    dev = _dev(s.grids("f32"), "f32")
    o = oracle.flowmap(oracle.Field(n, s.grids("f32")), times, oracle.seed_lattice(n, 3), N)
    _say("exit points: recording calls only")
    plain = run_gpu(n, dev, times, stride=3)
    with Context(n, len(o["flag"])) as ctx:
        ctx.seed(3)
        assert torch.isnan(ctx.exit_points()).all()
        ctx.advect(dev[:11], times[:11], record_exit=True)    # steps 0..9 record
        ctx.advect(dev[10:], times[10:], record_exit=False)  # steps 10..29 do not
        fm = ctx.flowmap()
        face = ctx.exit_points().cpu().numpy()
        g = {k: v.cpu().numpy() for k, v in fm.items()}
    # same events; positions agree to the FP32 repacking at the call boundary
    safe = o["margin"] >= 1e-6
    assert np.array_equal(g["flag"][safe], plain["flag"][safe]) and np.array_equal(g["exit"][safe], plain["exit"][safe])
    assert np.abs(g["end"] - plain["end"]).max() < 5e-6
    early = (g["flag"] == oracle.TERMINATED) & (g["exit"] < 10)
    late = (g["flag"] == oracle.TERMINATED) & (g["exit"] >= 10)
    assert early.sum() > 20 and late.sum() > 20
    assert np.all(np.isnan(face[late])) and np.all(np.isnan(face[g["flag"] == oracle.VALID]))
    ok = early & (o["margin"] >= 1e-6)
    np.testing.assert_allclose(face[ok], o["face"][ok], atol=3e-5)


@pytest.mark.parametrize("n", [(40, 36, 44), (23, 9, 2), (5, 64, 33)])
def test_seed_orders_give_identical_flow_maps(n):
    """Octant-major (default), natural x-fastest (z-slab segments) and brick
    orders only move particles between lanes and segments: every particle's
    arithmetic is the same, so flow maps and counters are bit-identical.  The
    lattices have uneven octants, and (23, 9, 2) empty ones (one z layer)."""
    import os

    N = 12
    s = fields.abc_noise(n, N + 1, 0.05, sigma=0.05, seed=31, global_n=48)
    gr = s.grids("f32")
    dev = _dev(gr, "f32")
    runs = {}
    for name, env in (("octant", {}), ("natural", {"BTO_OCTANT_SEED": "0"}),
                      ("bricks", {"BTO_OCTANT_SEED": "0", "BTO_BRICK": "16,2,2"})):
        _say(f"seed order {name} {n}")
        old = {k: os.environ.get(k) for k in env}
        os.environ.update(env)
        try:
            runs[name] = run_gpu(n, dev, s.times, stride=2, record_exit=True)
        finally:
            for k, v in old.items():
                if v is None:
                    del os.environ[k]
                else:
                    os.environ[k] = v
    _, o = oracle_lattice(oracle.Field(n, gr), s.times, n, 2, N)
    compare(runs["octant"], o, label=f"octant {n}")
    for name in ("natural", "bricks"):
        for k in ("end", "flag", "exit", "seed"):
            assert np.array_equal(runs[name][k], runs["octant"][k]), (name, k)
        assert np.array_equal(runs[name]["face"], runs["octant"]["face"], equal_nan=True)
        assert runs[name]["stats"] == runs["octant"]["stats"]


def test_plain_c_consumer_of_the_c_abi():
    """The C program paper_2004_02003_amd/c_abi_demo.c (no Python, no PyTorch:
    HIP runtime for memory, libbto.so for everything else) checks a uniform
    flow interval with non-uniform steps against the closed form, including
    exit points and an out-of-order call; run here as a child process."""
    import subprocess

    from paper_2004_02003_amd import build as hip_build

    _say("plain C consumer of the C-ABI")
    assert os.path.exists(hip_build.DEMO), "build() compiles the C demo next to libbto.so"
    r = subprocess.run([hip_build.DEMO], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("c-abi demo ok"), r.stdout


def test_error_paths_and_tuning_through_the_c_abi():
    """Validation happens before anything is enqueued: out-of-order calls,
    bad arguments and capacity overflow return the documented codes, the
    message names the problem, and the context stays usable afterwards."""
    import torch
    from paper_2004_02003_amd import BTOError, Context
    from paper_2004_02003_amd import _lib

    _say("error paths")
    n = (12, 10, 8)
    s = fields.uniform_flow(n, [0.2, 0.1, 0.0], np.arange(4) * 0.5)
    dev = _dev(s.grids("f32"), "f32")
    with Context(n, 100) as ctx:
        with pytest.raises(BTOError) as e:
            ctx.advect(dev, s.times)
        assert e.value.code == _lib.BTO_ESTATE
        with pytest.raises(BTOError) as e:
            ctx.touched_points(dev, s.times)
        assert e.value.code == _lib.BTO_ESTATE and "seeding" in str(e.value)
        with pytest.raises(BTOError) as e:
            ctx.seed(1)  # 12*10*8 = 960 seeds > capacity 100
        assert e.value.code == _lib.BTO_ERANGE and "capacity" in str(e.value)
        with pytest.raises(BTOError) as e:
            ctx.seed(0)
        assert e.value.code == _lib.BTO_EINVAL
        P = ctx.seed(3)
        assert P == 4 * 3 * 3  # offsets 1, 4, 7, (10) on axes of 12, 10, 8 points
        with pytest.raises(BTOError) as e:
            ctx.advect(dev, [0.0, 1.0, 1.0, 2.0])
        assert e.value.code == _lib.BTO_EINVAL and "increasing" in str(e.value)
        with pytest.raises(BTOError) as e:
            ctx.advect_ptrs([g.data_ptr() for g in dev], s.times, 7)
        assert e.value.code == _lib.BTO_EINVAL and "dtype" in str(e.value)
        with pytest.raises(BTOError) as e:
            ctx.advect_ptrs([dev[0].data_ptr(), 0], s.times[:2], 0)
        assert e.value.code == _lib.BTO_EINVAL
        with pytest.raises(BTOError) as e:
            ctx.touched_points(dev, [0.0, 1.0, 1.0, 2.0])
        assert e.value.code == _lib.BTO_EINVAL and "increasing" in str(e.value)
        t = ctx.touched_points(dev, s.times)  # a diagnostic walk: the interval is not advanced
        assert t.shape == (3, 3) and int(t[0, 2]) == P and ctx.stats()["steps_done"] == 0
        with pytest.raises(BTOError) as e:
            ctx.set_tuning(steps_per_launch=0)
        assert e.value.code == _lib.BTO_EINVAL
        with pytest.raises(BTOError) as e:
            ctx.set_tuning(lanes_per_particle=3)
        assert e.value.code == _lib.BTO_EINVAL and "lanes_per_particle" in str(e.value)
        with pytest.raises(BTOError) as e:
            ctx.set_tuning(ckpt_every=0)
        assert e.value.code == _lib.BTO_EINVAL and "ckpt_every" in str(e.value)
        with pytest.raises(BTOError) as e:
            ctx.set_tuning(tiles=3)
        assert e.value.code == _lib.BTO_EINVAL and "tiles" in str(e.value)
        ctx.set_tuning(steps_per_launch=2, rebin_every=1, blocks_per_cu=1, lanes_per_particle=2, ckpt_every=7)
        assert ctx.tuning() == dict(steps_per_launch=2, rebin_every=1, blocks_per_cu=1, lanes_per_particle=2,
                                    ckpt_every=7, tiles=0)
        ctx.advect(dev, s.times)  # still usable after the failures
        fm = ctx.flowmap(count_valid=True)
        torch.cuda.synchronize()
        assert fm["n_valid"] + int((fm["flag"] != 0).sum()) == P
        with pytest.raises(BTOError) as e:
            ctx.adjoint(dev, s.times, torch.zeros((P, 2, 3), dtype=torch.float32, device="cuda"))
        assert e.value.code == _lib.BTO_EINVAL
    with pytest.raises(BTOError):
        Context((1, 4, 4), 10)


def test_randomized_small_blocks_against_the_oracle():
    """Seeded random small cases: block sizes down to 2 points per axis, seeds
    anywhere (on faces, outside, near edges), 1 to 9 steps with random
    non-uniform times, every launch shape and the exit-point variant; flags
    and exit steps bit-exact outside the 1e-6 margin, positions within 1e-5."""
    rng = np.random.default_rng(2024)
    for case in range(24):
        n = tuple(int(v) for v in rng.integers(2, 14, 3))
        N = int(rng.integers(1, 10))
        times = np.concatenate([[rng.uniform(-1, 1)], rng.uniform(0.05, 0.3, N)]).cumsum()
        s = fields.abc_noise(n, N + 1, 0.1, sigma=0.05, seed=100 + case, global_n=int(rng.integers(6, 24)))
        dt = ["f32", "f16", "bf16"][case % 3]
        gr = s.grids(dt)
        hi = np.array(n, dtype=float) - 1
        P = int(rng.integers(1, 300))
        seeds = rng.uniform(-0.5, 1.5, (P, 3)) * hi
        k = rng.integers(0, P, P // 4)
        ax = rng.integers(0, 3, len(k))
        seeds[k, ax] = np.where(rng.random(len(k)) < 0.5, 0.0, hi[ax])  # seeds on faces
        tuning = dict(steps_per_launch=int(rng.integers(1, 6)), rebin_every=int(rng.integers(0, 4)),
                      lanes_per_particle=int(rng.integers(1, 3)))
        mode = "frozen" if case % 5 == 4 else "linear"
        chunks = None
        if N >= 3 and case % 2:
            cut = int(rng.integers(1, N))
            chunks = [cut, N - cut]
        _say(f"random case {case}: n={n} N={N} P={P} {dt} {mode} {tuning} chunks={chunks}")
        g = run_gpu(n, _dev(gr, dt), times, seeds=seeds, mode=mode, chunks=chunks, tuning=tuning,
                    record_exit=(case % 2 == 0))
        o = oracle.flowmap(oracle.Field(n, gr, dtype=dt), times, seeds, N,
                           mode=oracle.FROZEN if mode == "frozen" else oracle.LINEAR)
        on_face = np.any((seeds == 0.0) | (seeds == hi), axis=1)
        assert np.all(o["margin"][on_face] == 0.0)
        compare(g, o, label=f"random case {case}", max_excluded=float(on_face.mean()) + 0.01)
        assert g["n_valid"] == int((g["flag"] == 0).sum())


def test_largest_block_axis_closed_form_and_oracle():
    """A block at the largest supported axis length (1,024 points, the 10-bit
    cell index of the packed particle state) in uniform flow along x: seeds
    across the whole axis, including the last cells, end at x0 + u t or
    terminate in the step that would cross the x = 1023 face, as the closed
    form and the oracle say (also with a lattice seeded over the full axis)."""
    n = (1024, 4, 3)
    N = 8
    times = np.arange(N + 1) * 0.25
    u = (3.7, 0.1, 0.0)
    s = fields.uniform_flow(n, u, times)
    gr = s.grids("f32")
    xs = np.array([0.3, 500.5, 1000.0, 1015.2, 1016.9, 1019.0, 1021.7, 1022.99, 1023.0])
    seeds = np.stack([xs, np.full_like(xs, 1.5), np.full_like(xs, 1.0)], axis=1)
    _say("largest block axis 1024")
    dev = _dev(gr, "f32")
    g = run_gpu(n, dev, times, seeds=seeds, record_exit=True)
    o = oracle.flowmap(oracle.Field(n, gr), times, seeds, N)
    # one of the nine seeds starts on the x = 1023 face (margin 0)
    compare(g, o, label="axis 1024", max_excluded=1.0 / len(xs))
    # closed form: x(t) = x0 + u t while inside
    ux = np.float32(3.7)
    for i, x0 in enumerate(xs):
        ends = x0 + float(ux) * (times[1:] - times[0])
        inside = ends <= 1023.0
        e = N if inside.all() else int(np.argmin(inside))
        assert g["exit"][i] == e, (x0, g["exit"][i], e)
        want = x0 + float(ux) * (times[e] - times[0])
        assert abs(g["end"][i, 0] - want) < 1e-5
    gl = run_gpu(n, dev, times, stride=3)
    sl, ol = oracle_lattice(oracle.Field(n, gr), times, n, 3, N)
    compare(gl, ol, label="axis 1024 lattice", seeds=sl, n=n)
