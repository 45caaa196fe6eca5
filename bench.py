"""Benchmark of the per-block BTO path on one MI355X.

One step = one interval of the hot path over the resident input: seed the
lattice, advance every live particle by the interval's RK4 steps (one per
cycle) with boundary termination and compaction, and write the flow map.
Workload: the 128^3 time-varying ABC block with noise (101 cycles, dt 0.05,
64^3 seeds at stride 2, 100-step interval), FP32 grids resident in HBM.

Prints one JSON line: particle-RK4-steps/s of the whole step, the roofline of
the dominant kernel (the fused advection launch, timed with HIP events on the
stream it runs on), and the FP64 oracle timed on the host cores.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-RK4-steps/s on 1 MI355X + %HBM peak; FP32 vs FP16 field at stated err"
HBM_PEAK_GBS = 8000.0
STATE_BYTES = 40          # 16 B state + 4 B id, read once and written once per launch
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "advect_f32_abc128_traffic.json")
KERNEL_SOURCES = ["paper_2004_02003_amd/csrc/bto_device.h", "paper_2004_02003_amd/csrc/advect.hip"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def device_copy_rate(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """GB/s (read + write bytes) of a plain device-to-device copy, median of reps."""
    import torch

    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (float(np.median(ts)) * 1e-3) / 1e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def field_bytes_per_point(dt: str) -> int:
    return 12 if dt == "f32" else 6


def launch_plan(n_steps: int, kmax: int, rb: int):
    """The library's balanced split of one advect call into launches."""
    if 0 < rb < kmax:
        kmax = rb
    nl = (n_steps + kmax - 1) // kmax
    return [n_steps // nl + (1 if l < n_steps % nl else 0) for l in range(nl)]


def algorithmic_bytes(per_launch, dt: str, stride: int):
    """Bytes the fused launches must move: per particle-step one new grid level
    over the points its cell touches (stride^3 points per seed at the lattice
    density, i.e. 8 at stride 2), the first level once per launch, and the
    particle state in and out once per launch."""
    bpt = field_bytes_per_point(dt) * (stride ** 3 if stride <= 2 else 8)
    total = 0
    for live_in, psteps in per_launch:
        total += bpt * (psteps + live_in) + STATE_BYTES * live_in
    return total


# Per-cycle time of the paper's own metric (Section 4.2: mean time per
# non-write cycle of advection + particle management) on the paper's per-rank
# ABC shape: a 64^3 block of a 256^3 domain (64 ranks), one period in 1000
# steps, intervals 25/50/100, reductions 1:1, 1:8, 1:27.  Context only: the
# paper's times (ABC table, Lagrangian-BTO seconds per step) are V100 times
# inside Ascent/VTK-h, a different machine and framework.
PAPER_ABC_TABLE_MS = {(25, 1): 5.9, (50, 1): 6.6, (100, 1): 6.7,
                      (25, 2): 2.6, (50, 2): 3.3, (100, 2): 2.6,
                      (25, 3): 2.4, (50, 3): 2.9, (100, 3): 2.7}
# The paper's in situ saving of BTO over the communicating Lagrangian-MPI
# baseline (Abstract; Section 5 weak scaling and the ABC/Jet/Nyx tables), with
# the hardware it was measured on.  Quoted as context only: the communicating
# baseline is not built here, so no ratio of ours is compared with it.
PAPER_INSITU_SAVING = {
    "claim": "BTO saves 2x-4x of the in situ execution time of Lagrangian-MPI (Abstract); about 3x on average in "
             "the Cloverleaf3D weak scaling (2.0x-4.1x per configuration); per configuration 1.6x-2.8x (ABC), "
             "1.2x-3.9x (Jet) and 1.4x-5.2x (Nyx) in the WF2 tables",
    "hardware": "Summit: per node two IBM Power9 CPUs (22 cores each) and six NVIDIA Tesla V100 GPUs (16 GB HBM2) "
                "over NVLink; VTK-m / VTK-h / Ascent filters",
}


def paper_context(log):
    import math
    import torch
    from bto_inputs import fields
    from paper_2004_02003_amd import Context, InSituDriver, grid_to_device

    n, total = 64, 200
    s = fields.abc_noise(n, total + 1, 2 * math.pi / 1000, sigma=0.0, global_n=256, offset=(64, 64, 64))
    dev = [grid_to_device(g, "f32") for g in s.grids("f32")]
    out = {"paper_insitu_saving_context": PAPER_INSITU_SAVING}
    for interval in (25, 50, 100):
        for stride in (1, 2, 3):
            term = []

            def keep(idx, fm, t0, t1, _term=term):
                _term.append(float((fm["flag"] != 0).float().mean()))

            with Context((n, n, n), n ** 3) as ctx:
                drv = InSituDriver(ctx, interval=interval, stride=stride, on_flowmap=keep)
                for c in range(len(dev)):
                    drv.cycle(dev[c], float(s.times[c]))
                torch.cuda.synchronize()
                ms = drv.mean_cycle_ms()
                particles = ctx.n_seeds
            key = f"abc_64_block_1to{stride ** 3}_interval{interval}"
            out[key] = {"ms_per_cycle": round(ms, 4),
                        "discarded_pct": round(100 * sum(term) / len(term), 2),
                        "paper_v100_ms_per_cycle": PAPER_ABC_TABLE_MS[(interval, stride)],
                        "particles": particles, "intervals": len(term)}
            log(f"paper context {key}: {ms:.4f} ms per cycle")
    return out


# Launch shape per workload (results do not depend on it).  The coherent ABC
# block runs best as seeded; the turbulent blocks mix their particles, so a
# periodic re-sort restores cache locality, and for FP32 grids two lanes per
# particle halve the cache lines a row load touches.
LAUNCH_SHAPE = {
    "turb_256": dict(rebin_every=5, lanes_per_particle=2),
    "turb_512": dict(rebin_every=10, lanes_per_particle=2),
}


def posthoc_accuracy(log):
    """The paper's accuracy experiment (Section 4, ABC table) at node scale on
    one GPU: a 132^3-cell ABC domain cut into 2 x 2 x 2 blocks of 66^3 cells
    (about the paper's per-rank 64^3 blocks, divisible by both strides), seeds
    at 1:8 and 1:27, consecutive intervals of 25, 50 and 100 steps over 100
    cycles.  BTO advects every block on its own; the reference advects the
    whole domain (the communicating result); terminated entries are rebuilt by
    Eq. (1) and scored by Eq. (5)/(6) per interval, then summarised across
    the intervals as the paper does (total average L2, average and greatest
    maximum L2, discarded %).  Times are HIP events for the 1:8, interval-50
    case."""
    import torch
    from bto_inputs import fields
    from paper_2004_02003_amd import grid_to_device, posthoc

    n, cycles = 133, 101
    s = fields.abc_noise(n, cycles, 0.05, sigma=0.01, seed=1, global_n=132)
    dev = [grid_to_device(g, "f32") for g in s.grids("f32")]
    out = {"domain": "ABC 132^3 cells (133^3 points), 2x2x2 blocks of 66^3 cells, dt 0.05, 100 cycles"}
    for stride in (2, 3):
        for interval in (25, 50, 100):
            per = []
            for k in range((cycles - 1) // interval):
                g = dev[k * interval:(k + 1) * interval + 1]
                t = s.times[k * interval:(k + 1) * interval + 1]
                timed = stride == 2 and interval == 50 and k == 0
                if timed:
                    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
                    ev[0].record()
                b_end, b_flag, M = posthoc.run_blocks(g, t, (2, 2, 2), stride)
                if timed:
                    ev[1].record()
                m_end, m_flag, _ = posthoc.run_domain(g, t, stride)
                if timed:
                    ev[2].record()
                state = posthoc.reconstruct_lattice(b_end, b_flag, M)
                if timed:
                    ev[3].record()
                acc = posthoc.flowmap_error(b_end, state, m_end, m_flag, cell=1.0)
                if timed:
                    ev[4].record()
                    torch.cuda.synchronize()
                    out["ms_1to8_interval50"] = {"bto_blocks_incl_staging": round(ev[0].elapsed_time(ev[1]), 3),
                                                 "domain_reference": round(ev[1].elapsed_time(ev[2]), 3),
                                                 "rebuild_kernels": round(ev[2].elapsed_time(ev[3]), 4),
                                                 "metric": round(ev[3].elapsed_time(ev[4]), 4)}
                st = state.cpu().numpy()
                per.append(dict(term=float((b_flag != 0).float().mean()), rebuilt=float((st == 2).mean()),
                                missing=int((st == 0).sum()), **acc))
            L = float(np.mean([r["mean_l2"] for r in per]))
            key = f"1to{stride ** 3}_interval{interval}"
            out[key] = {"intervals": len(per), "seeds": int(np.prod(M)),
                        "discarded_pct": round(100 * float(np.mean([r["term"] for r in per])), 3),
                        "rebuilt_pct": round(100 * float(np.mean([r["rebuilt"] for r in per])), 3),
                        "left_missing": int(np.mean([r["missing"] for r in per])),
                        "total_average_l2": L,
                        "average_max_l2": float(np.mean([r["max_l2"] for r in per])),
                        "greatest_max_l2": float(np.max([r["max_l2"] for r in per])),
                        "accuracy_pct": round((1.0 - L) / 1.0 * 100.0, 4)}
            log(f"post hoc {key}: {out[key]}")
    del dev
    torch.cuda.empty_cache()
    return out


def insitu_overlap(log, n=128, modes=32):
    """The in situ driver fed by a running "simulation": every cycle the device
    turbulence generator computes the next grid into the simulation's own
    buffer (n^3 points, FP32) on the caller's stream, and the driver copies it
    into its ring and advects (n/2)^3 particles one step.  Serial (copy and
    advection on the caller's stream) vs overlapped (ingest and compute streams
    of the driver's own, so the advection of step c runs beside the generation
    of grid c+1).  Wall-clock ms per cycle over 50 cycles, best of 3, and the
    generator alone for scale."""
    import torch
    from bto_inputs import _turb, fields
    from paper_2004_02003_amd import Context, InSituDriver

    ncyc = 51
    s = fields.turbulence(n, modes, 2, ncyc, 0.02)
    gen = _turb.DeviceTurbulence(s.lazy)
    buf = torch.empty((n, n, n, 3), dtype=torch.float32, device="cuda")
    out = {"workload": f"turbulence {n}^3, {modes} modes, f32, {n // 2}^3 seeds, 50 cycles"}

    def wall(fn, reps=3):
        best = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t0) / (ncyc - 1))
        return round(1e3 * best, 4)

    def gen_only():
        for c in range(ncyc):
            gen.fill(c, "f32", buf)
    out["generator_only_ms_per_cycle"] = wall(gen_only)
    for overlap in (False, True):
        with Context((n, n, n), (n // 2) ** 3) as ctx:
            def run():
                drv = InSituDriver(ctx, interval=ncyc - 1, stride=2, copy=True, overlap=overlap, timing=False)
                for c in range(ncyc):
                    gen.fill(c, "f32", buf)
                    drv.cycle(buf, float(s.times[c]))
                drv.synchronize()
            out[("overlapped" if overlap else "serial") + "_ms_per_cycle"] = wall(run)
    log(f"in situ with a running simulation: {out}")
    return out


UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def precision_statement(log, threads):
    """End-position error of the GPU path against the FP64 oracle on the FP64
    field, per storage type, for the turbulence blocks (the 256^3 precision
    workload in f32/f16/bf16, the 512^3 scale workload in f16 through a
    two-slot ring), on a fixed seed subset; with the first-order bound
    ||J|| N h max|V| (u_storage + 2^-21) per seed (J from the oracle's tangent,
    u the storage's unit roundoff, 2^-21 the FP32 sampling arithmetic)."""
    import torch
    import oracle
    from bto_inputs import _turb
    from bto_inputs.workloads import WORKLOADS
    from paper_2004_02003_amd import Context

    out = {}
    for name, every in (("turb_256", 509), ("turb_512", 32771)):  # steps coprime with the lattice rows
        wl = WORKLOADS[name]
        s = wl.make_field()
        gen = _turb.DeviceTurbulence(s.lazy)
        N = wl.n_steps
        ids = np.arange(0, wl.n_seeds, every)
        seeds = oracle.seed_lattice(wl.n, wl.stride)[ids]
        t0 = time.perf_counter()
        o = oracle.flowmap(oracle.Field.lazy_turbulence(s, "f64"), s.times, seeds, N, jac=True, nthreads=threads)
        log(f"precision {name}: FP64 oracle on {len(ids)} seeds in {time.perf_counter() - t0:.1f} s")
        nJ = np.linalg.norm(o["jac"], axis=(1, 2), ord=2)
        shape = (wl.n[2], wl.n[1], wl.n[0], 3)
        res = {}
        for dt in wl.dtypes:
            tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dt]
            vmax = 0.0
            with Context(wl.n, wl.n_seeds) as ctx:
                ctx.set_tuning(**{k: v for k, v in LAUNCH_SHAPE.get(name, {}).items()})
                ctx.seed(wl.stride)
                slots = [torch.empty(shape, dtype=tdt, device="cuda") for _ in range(2)]
                gen.fill(0, dt, slots[0])
                for c in range(N):
                    gen.fill(c + 1, dt, slots[(c + 1) % 2])
                    if c % 10 == 0:
                        vmax = max(vmax, float(slots[(c + 1) % 2].float().abs().max()))
                    ctx.advect([slots[c % 2], slots[(c + 1) % 2]], s.times[c:c + 2])
                fm = ctx.flowmap()
                torch.cuda.synchronize()
                end = fm["end"].cpu().numpy()[ids]
                flag = fm["flag"].cpu().numpy()[ids]
                del slots
            torch.cuda.empty_cache()
            both = (flag == 0) & (o["flag"] == 0)
            err = np.linalg.norm(end[both] - o["end"][both], axis=1)
            bound = nJ[both] * N * wl.dt * vmax * np.sqrt(3.0) * (UNIT_ROUNDOFF[dt] + 2.0 ** -21)
            safe = o["margin"] >= 1e-6
            res[dt] = {"mean": float(err.mean()), "p99": float(np.quantile(err, 0.99)), "max": float(err.max()),
                       "n": int(both.sum()), "within_first_order_bound_pct": round(100.0 * float((err <= bound).mean()), 2),
                       "bound_median": float(np.median(bound)),
                       "flag_disagree": int((flag != o["flag"]).sum()),
                       "flag_disagree_outside_margin": int(((flag != o["flag"]) & safe).sum())}
            log(f"precision {name} {dt}: {res[dt]}")
        out[name] = {"seeds": f"every {every}th of {wl.n_seeds}", "steps": N, "cells": "end-position L2 error, cells",
                     **res}
    return out


def per_cycle(log):
    """One RK4 step per launch (the in situ call form) on three ABC blocks:
    128^3 at stride 2 and 64^3 at strides 2 and 1, 100 cycles each, HIP events
    around the 100 calls (mean per cycle over 4 repetitions).  The 64^3 block
    at stride 1 has as many particles as the 128^3 block at stride 2 but an
    eighth of the field bytes."""
    import math
    import torch
    from bto_inputs import fields
    from bto_inputs.workloads import WORKLOADS
    from paper_2004_02003_amd import Context, grid_to_device

    def run(n, stride, dev, times, reps=4):
        with Context((n, n, n), n ** 3) as ctx:
            ptrs = [g.data_ptr() for g in dev]
            N = len(dev) - 1
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for r in range(reps + 1):
                ctx.seed(stride)
                if r >= 1:
                    ev[r - 1][0].record()
                for q in range(N):
                    ctx.advect_ptrs(ptrs[q:q + 2], times[q:q + 2], 0)
                if r >= 1:
                    ev[r - 1][1].record()
            torch.cuda.synchronize()
            ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
            return {"seeds": ctx.n_seeds, "us_per_cycle": round(1e3 * ms / N, 2),
                    "particle_steps": int(ctx.stats()["particle_steps"])}

    out = {}
    s = WORKLOADS["abc_128"].make_field()
    dev = [grid_to_device(g, "f32") for g in s.grids("f32")]
    out["abc_128_stride2"] = run(128, 2, dev, list(s.times))
    del dev
    s2 = fields.abc_noise(64, 101, 2 * math.pi / 1000, sigma=0.0, global_n=256, offset=(64, 64, 64))
    dev2 = [grid_to_device(g, "f32") for g in s2.grids("f32")]
    out["abc_64_stride2"] = run(64, 2, dev2, list(s2.times))
    out["abc_64_stride1"] = run(64, 1, dev2, list(s2.times))
    for k, v in out.items():
        log(f"per cycle {k}: {v['us_per_cycle']} us")
    del dev2
    torch.cuda.empty_cache()
    return out


def differentiation(log):
    """The differentiation workload: 32^3 seeds (stride 4) on the 128^3 ABC
    field, 100 steps, checkpoints every 10.  Times (HIP events, median of 5)
    of the adjoint for the seeded-weight loss (seed gradients, and seed plus
    grid gradients), and of the flow-map Jacobian with FTLE for every seed.
    Throughput counts forward particle-steps of the interval per second of
    the whole backward call (checkpointed forward + recompute + reverse)."""
    import torch
    from bto_inputs.workloads import WORKLOADS, loss_weights
    from paper_2004_02003_amd import Context, grid_to_device, jacobian_ftle

    wl = WORKLOADS["abc_128_adjoint"]
    s = wl.make_field()
    dev = [grid_to_device(g, "f32") for g in s.grids("f32")]
    k = wl.extra["ckpt_every"]
    out = {"workload": f"{wl.name}: {wl.n_seeds} seeds, {wl.n_steps} steps, checkpoint every {k}"}
    with Context(wl.n, wl.n_seeds) as ctx:
        ctx.seed(wl.stride)
        ctx.advect(dev, s.times)
        psteps = ctx.stats()["particle_steps"]
        w = torch.as_tensor(loss_weights(wl.n_seeds, wl.extra["weight_seed"]), dtype=torch.float32,
                            device="cuda").contiguous()
        gg = [torch.zeros(g.shape, dtype=torch.float32, device="cuda") for g in dev]
        seeds = ctx.flowmap()["seed"].clone()

        def timed(fn, reps=5):
            ts = []
            for _ in range(reps + 1):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            return float(np.median(ts[1:]))

        def seed_grad():
            ctx.seed(wl.stride)
            ctx.adjoint(dev, s.times, w, ckpt_every=k)

        def seed_and_grid_grad():
            ctx.seed(wl.stride)
            ctx.adjoint(dev, s.times, w, grad_grids=gg, ckpt_every=k)

        def jac():
            jacobian_ftle(ctx, seeds, dev, s.times, ckpt_every=k)

        def seed_grad_every_step():
            # a checkpoint at every step (N x P x 24 B) removes the recompute sweep
            ctx.seed(wl.stride)
            ctx.adjoint(dev, s.times, w, ckpt_every=1)

        def forward_then_adjoint():
            # the training-loop form: the forward advection, then the adjoint recomputing it
            ctx.seed(wl.stride)
            ctx.advect(dev, s.times)
            ctx.adjoint(dev, s.times, w, ckpt_every=k)

        def forward_recording_then_adjoint():
            # the same with checkpoints recorded by the forward advection (no recomputed forward)
            ctx.seed(wl.stride)
            ctx.advect(dev, s.times, record_ckpt=True)
            ctx.adjoint(dev, s.times, w, ckpt_every=k, recorded=True)

        ctx.set_tuning(ckpt_every=k)
        for name, fn in (("seed_gradient", seed_grad), ("seed_and_grid_gradient", seed_and_grid_grad),
                         ("jacobian_ftle", jac), ("seed_gradient_checkpoint_every_step", seed_grad_every_step),
                         ("forward_then_seed_gradient", forward_then_adjoint),
                         ("forward_recording_checkpoints_then_seed_gradient", forward_recording_then_adjoint)):
            ms = timed(fn)
            out[name] = {"ms": round(ms, 4), "forward_particle_steps_per_s": round(psteps / (ms * 1e-3), 1)}
            log(f"differentiation {name}: {ms:.3f} ms")
    del dev, gg
    torch.cuda.empty_cache()
    return out


# Legs that --leg runs on their own (all of them but per_cycle are part of the
# default run on the abc_128 workload).
LEGS = {
    "paper_context": paper_context,
    "posthoc_accuracy": posthoc_accuracy,
    "insitu_overlap": lambda log: [insitu_overlap(log, 128, 32), insitu_overlap(log, 256, 64)],
    "differentiation": differentiation,
    "per_cycle": per_cycle,
}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="abc_128")
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--steps-per-launch", type=int, default=None,
                    help="RK4 steps fused into one advection launch (1..128; sets BTO_STEPS_PER_LAUNCH)")
    ap.add_argument("--rebin-every", type=int, default=None,
                    help="re-sort live particles every this many steps (0 = never; default per workload)")
    ap.add_argument("--lanes-per-particle", type=int, default=None, choices=(1, 2),
                    help="FP32 grids: lanes per particle (default per workload)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--leg", action="append", choices=sorted(LEGS),
                    help="run only these legs (repeatable) and print their results as one JSON line")
    args = ap.parse_args(argv)
    if args.steps_per_launch is not None:
        os.environ["BTO_STEPS_PER_LAUNCH"] = str(args.steps_per_launch)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the per-block BTO path has no cross-GPU work "
              "(blocks are independent); run one process per block instead.", file=sys.stderr)
        sys.exit(2)

    if args.leg:
        import torch
        from paper_2004_02003_amd import _lib

        _lib.load()
        assert torch.cuda.is_available(), "bench.py needs a HIP device"
        print(json.dumps({name: LEGS[name](log) for name in args.leg}), flush=True)
        return

    import torch
    import oracle
    from bto_inputs.workloads import WORKLOADS
    from paper_2004_02003_amd import Context, grid_to_device
    from paper_2004_02003_amd import _lib

    _lib.load()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    wl = WORKLOADS[args.workload]
    dt = args.dtype
    log(f"workload {wl.name}: generating {wl.n_cycles} grids {wl.n} ({dt})")
    t0 = time.time()
    series = wl.make_field()
    turb = series.lazy is not None
    if turb:
        # large turbulence blocks: grids generated on the device (bit-identical to the host evaluator)
        from bto_inputs import _turb
        gen = _turb.DeviceTurbulence(series.lazy)
        tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dt]
        shape = (wl.n[2], wl.n[1], wl.n[0], 3)
        dev = [gen.fill(c, dt, torch.empty(shape, dtype=tdt, device="cuda")) for c in range(wl.n_cycles)]
        grids_host = None
        args.no_variants = True
    else:
        grids_host = series.grids(dt) if (not args.no_cpu_baseline or not args.no_variants) else None
        dev = [grid_to_device(g, dt) for g in (grids_host if grids_host is not None else series.grids(dt))]
    torch.cuda.synchronize()
    log(f"grids resident ({sum(g.numel() * g.element_size() for g in dev) / 2**30:.2f} GiB) in {time.time() - t0:.1f}s")
    times = np.asarray(series.times, dtype=np.float64)
    N = wl.n_steps
    ptrs = [g.data_ptr() for g in dev]
    dcode = {"f32": _lib.BTO_F32, "f16": _lib.BTO_F16, "bf16": _lib.BTO_BF16}[dt]

    ctx = Context(wl.n, wl.n_seeds)
    tune = dict(LAUNCH_SHAPE.get(wl.name, {}))
    if args.rebin_every is not None:
        tune["rebin_every"] = args.rebin_every
    if args.lanes_per_particle is not None:
        tune["lanes_per_particle"] = args.lanes_per_particle
    if tune:
        ctx.set_tuning(**tune)
    tuning = ctx.tuning()
    P = ctx.seed(wl.stride)
    out = ctx.flowmap()

    # per-launch live counts and particle-steps (untimed pass, one call per launch)
    plan = launch_plan(N, tuning["steps_per_launch"], tuning["rebin_every"])
    per_launch = []
    q = 0
    ctx.seed(wl.stride)
    prev = ctx.stats()
    for K in plan:
        ctx.advect_ptrs(ptrs[q:q + K + 1], times[q:q + K + 1], dcode)
        st = ctx.stats()
        per_launch.append((prev["n_live"], st["particle_steps"] - prev["particle_steps"]))
        prev = st
        q += K
    psteps_interval = prev["particle_steps"]
    n_valid = prev["n_live"]
    log(f"{P} seeds, {psteps_interval} particle-steps per interval, {n_valid} valid at the end, "
        f"{len(plan)} launches of {plan} steps")

    def one_step(ev=None):
        ctx.seed(wl.stride)
        if ev is not None:
            ev[0].record()
        ctx.advect_ptrs(ptrs, times, dcode)
        if ev is not None:
            ev[1].record()
        ctx.flowmap(out=out)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        one_step(evs[k])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    adv_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    st = ctx.stats()
    assert st["particle_steps"] == psteps_interval, "particle-step count changed between intervals"
    ms_per_step = 1e3 * t_total / args.steps
    value = psteps_interval * args.steps / t_total
    launch_ms = adv_ms / len(plan)
    bytes_interval = algorithmic_bytes(per_launch, dt, wl.stride)
    achieved = bytes_interval / len(plan) / (launch_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("kernel_hash") == kernel_hash() and rec.get("workload") == wl.name and rec.get("dtype") == dt:
            traffic = rec.get("bytes_per_launch")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"advect_kernel<{dt},linear>", "launches_per_step": len(plan),
            "avg_launch_ms": round(launch_ms, 4),
            "algorithmic_bytes_per_launch": int(bytes_interval / len(plan))}
    # context for the peak: what a plain 1 GiB device-to-device copy reaches on this GPU
    copy_gbs = device_copy_rate()
    roof["device_copy_GBs"] = round(copy_gbs, 1)
    if traffic:
        roof["traffic_GBs"] = round(traffic / (launch_ms * 1e-3) / 1e9, 1)
    log(f"{value:.3e} particle-steps/s, {ms_per_step:.3f} ms per interval, advect {adv_ms:.3f} ms, "
        f"{achieved:.0f} GB/s algorithmic")

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "particle-RK4-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dt,
        "data": ("synthetic (seeded analytic ABC flow + Gaussian noise; no dataset)" if not turb else
                 "synthetic (seeded divergence-free Fourier-mode turbulence; no dataset)"),
        "config": {"workload": wl.name, "n": list(wl.n), "cycles": wl.n_cycles, "dt": wl.dt,
                   "stride": wl.stride, "seeds": P, "interval_steps": N, "storage": dt,
                   "particle_steps_per_interval": int(psteps_interval), "valid_at_end": int(n_valid),
                   "tuning": tuning},
        "advect_only": {"value": round(psteps_interval / (adv_ms * 1e-3), 1), "ms": round(adv_ms, 4)},
        "roofline": roof,
    }

    # in situ form: one call per cycle with the two resident grids
    if not args.no_variants:
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        for r in range(4):
            ctx.seed(wl.stride)
            if r >= 1:
                ev[r - 1][0].record()
            for s_ in range(N):
                ctx.advect_ptrs(ptrs[s_:s_ + 2], times[s_:s_ + 2], dcode)
            if r >= 1:
                ev[r - 1][1].record()
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        # the same one-step launches enqueued by the library in one call (no Python per cycle)
        ctx.set_tuning(steps_per_launch=1)
        ev2 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        for r in range(4):
            ctx.seed(wl.stride)
            if r >= 1:
                ev2[r - 1][0].record()
            ctx.advect_ptrs(ptrs, times, dcode)
            if r >= 1:
                ev2[r - 1][1].record()
        torch.cuda.synchronize()
        ctx.set_tuning(**tuning)
        ms2 = float(np.mean([a.elapsed_time(b) for a, b in ev2]))
        result["insitu_per_cycle"] = {"value": round(psteps_interval / (ms * 1e-3), 1), "ms": round(ms, 4),
                                      "launches": N, "note": "one Python call per cycle",
                                      "library_enqueued": {"value": round(psteps_interval / (ms2 * 1e-3), 1),
                                                           "ms": round(ms2, 4)}}

    ctx.close()

    # FP16 / BF16 storage of the same field, with the error against the FP64 oracle
    if not args.no_variants:
        variants = {}
        ids = np.arange(0, P, 97)
        seeds = oracle.seed_lattice(wl.n, wl.stride)[ids]
        log("oracle on the FP64 grids for the error statement")
        g64 = [series.make(c) for c in range(series.n_cycles)]
        o64 = oracle.flowmap(oracle.Field(wl.n, g64), times, seeds, N)
        del g64
        for vdt in ("f32", "f16", "bf16"):
            gh = series.grids(vdt) if vdt != dt else grids_host
            dv = [grid_to_device(g, vdt) for g in gh]
            vptr = [g.data_ptr() for g in dv]
            vcode = {"f32": _lib.BTO_F32, "f16": _lib.BTO_F16, "bf16": _lib.BTO_BF16}[vdt]
            with Context(wl.n, wl.n_seeds) as c2:
                c2.seed(wl.stride)
                c2.advect_ptrs(vptr, times, vcode)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                tt = []
                for r in range(5):
                    c2.seed(wl.stride)
                    e0.record()
                    c2.advect_ptrs(vptr, times, vcode)
                    e1.record()
                    torch.cuda.synchronize()
                    tt.append(e0.elapsed_time(e1))
                fm = c2.flowmap()
                stv = c2.stats()
                torch.cuda.synchronize()
                end = fm["end"].cpu().numpy()[ids]
                flag = fm["flag"].cpu().numpy()[ids]
            both = (flag == 0) & (o64["flag"] == 0)
            err = np.linalg.norm(end[both] - o64["end"][both], axis=1)
            variants[vdt] = {
                "advect_value": round(stv["particle_steps"] / (np.median(tt) * 1e-3), 1),
                "advect_ms": round(float(np.median(tt)), 4),
                "err_vs_fp64_cells": {"mean": float(err.mean()), "p99": float(np.quantile(err, 0.99)),
                                      "max": float(err.max()), "n": int(both.sum()),
                                      "flag_disagree": int((flag != o64["flag"]).sum())}}
            del dv
            torch.cuda.empty_cache()
        result["storage_variants"] = variants

    if not args.no_variants and wl.name == "abc_128":
        result["paper_context"] = paper_context(log)
        result["posthoc_accuracy"] = posthoc_accuracy(log)
        result["insitu_overlap"] = [insitu_overlap(log, 128, 32), insitu_overlap(log, 256, 64)]
        result["differentiation"] = differentiation(log)

    if not args.no_cpu_baseline:
        ids = np.arange(0, P, 1 if not turb else 1024)
        seeds = oracle.seed_lattice(wl.n, wl.stride)[ids]
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        F = oracle.Field(wl.n, grids_host, dtype=dt) if not turb else oracle.Field.lazy_turbulence(series, dt)
        log(f"oracle CPU baseline on {len(ids)} seeds, {threads} threads")
        # repeat the sample until about 10 s of CPU work (at most 30 s)
        tc = 0.0
        reps = 0
        ps = 0
        while tc < 10.0 and reps < 50:
            t1 = time.perf_counter()
            o = oracle.flowmap(F, times, seeds, N, nthreads=threads)
            tc += time.perf_counter() - t1
            ps += int(np.where(o["flag"] == 0, N, o["exit"] + 1).sum())
            reps += 1
            if tc > 30.0:
                break
        cpu_model = "unknown"
        try:
            with open("/proc/cpuinfo") as fh:
                cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), cpu_model)
        except OSError:
            pass
        result["cpu_baseline"] = {"value": round(ps / tc, 1), "unit": "particle-RK4-steps/s", "cores": threads,
                                  "kind": "oracle", "cpu": cpu_model, "nproc": os.cpu_count(),
                                  "sample": f"{'all' if len(ids) == P else f'every {ids[1] - ids[0]}th'} seed(s) of "
                                            f"{wl.name} ({len(ids)} seeds x {N} steps) x {reps} repeats, {ps} "
                                            f"particle-steps in {tc:.1f} s, FP64, OpenMP"}
        # the same oracle on one thread, on every 16th seed of the same sample
        ids1 = ids[::16]
        t1 = time.perf_counter()
        o1 = oracle.flowmap(F, times, seeds[::16], N, nthreads=1)
        t1 = time.perf_counter() - t1
        ps1 = int(np.where(o1["flag"] == 0, N, o1["exit"] + 1).sum())
        result["cpu_baseline_1thread"] = {"value": round(ps1 / t1, 1), "unit": "particle-RK4-steps/s", "cores": 1,
                                          "kind": "oracle",
                                          "sample": f"{len(ids1)} seeds x {N} steps, {ps1} particle-steps in "
                                                    f"{t1:.1f} s, FP64"}
        if not args.no_variants and wl.name == "abc_128":
            result["precision_turbulence"] = precision_statement(log, threads)

    if args.copy_probe:
        x = torch.empty(2 ** 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copy probe: 3 x 1 GiB device copy done")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
