"""Benchmark of the per-block BTO path on one MI355X.

One step = one interval of the hot path in the in situ form the paper times
(one velocity grid arrives per simulation cycle; Section 2.2, Section 4.2):
seed the lattice, then per cycle one RK4 step of every live particle with
boundary termination and compaction over the two resident grids (cycles n and
n+1), then write the flow map.  Headline workload: the 512^3 Fourier-mode
turbulence block, FP16 storage with FP32 arithmetic, 256^3 = 16,777,216 seeds
at stride 2, a 200-step interval over 201 cycles (dt 0.01).  Only two grids
are resident: the device generator writes cycle c+1's grid into the slot the
previous step no longer reads, on the same stream, outside the timed region.

Prints one JSON line: particle-RK4-steps/s of the interval (seed + 200 steps +
flow-map write, median of HIP-event times over the timed intervals; grid
generation excluded and reported on its own), the roofline of the dominant
kernel at the per-unit figure of two grid levels over 8 points plus 40 bytes
of particle state per live particle-step (136 B for 16-bit storage, 232 B for
FP32), and the CPU baseline leg: the FP64 oracle timed on the host cores, and
(with the other legs) the oracle's FP64 references for the stated error of
the GPU path.  The oracle runs in that leg only.
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
# the dominant kernels and the host code that sets their launch order and buffers
KERNEL_SOURCES = ["paper_2004_02003_amd/csrc/bto_device.h", "paper_2004_02003_amd/csrc/bto_internal.h",
                  "paper_2004_02003_amd/csrc/advect.hip", "paper_2004_02003_amd/csrc/tiles.hip",
                  "paper_2004_02003_amd/csrc/api.hip"]


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


def precision_gpu_runs(log):
    """The GPU side of the stated error (the oracle side is in the CPU
    baseline leg, cpu_reference_errors): end positions and flags of sampled
    seeds of the turbulence blocks, per storage type, through a two-slot ring
    with one call per cycle -- the 256^3 precision workload in f32 (FP32 and
    FP64 sampling), f16 and bf16 on every 509th seed (4,121 seeds), and the
    512^3 scale workload in f16 on 65,536 seeds (one per lattice row, spread
    over x) -- with the largest velocity magnitude of the grids read."""
    import torch
    from bto_inputs import _turb
    from bto_inputs.workloads import WORKLOADS, lattice_dims, lattice_points, row_sample_ids
    from paper_2004_02003_amd import Context

    out = {}
    for name, every in (("turb_256", 509), ("turb_512", 256)):  # 509: coprime with the lattice rows
        wl = WORKLOADS[name]
        s = wl.make_field()
        gen = _turb.DeviceTurbulence(s.lazy)
        N = wl.n_steps
        if every == 256:  # one seed per lattice row, its x index cycling (a plain stride of 256 keeps x fixed)
            ids = row_sample_ids(lattice_dims(wl.n, wl.stride), wl.n_seeds // every)
        else:
            ids = np.arange(0, wl.n_seeds, every)
        runs = [(dt, dt, False) for dt in wl.dtypes]
        if "f32" in wl.dtypes:
            runs.insert(1, ("f32_sampled_fp64", "f32", True))
        res = {}
        for key, dt, fp64 in runs:
            vmax = 0.0
            ring = Ring(gen, wl.n, dt)
            with Context(wl.n, wl.n_seeds) as ctx:
                ctx.set_tuning(**insitu_shape(name, dt))
                ctx.seed(wl.stride)
                p_prev = ring.ptr(0)
                for c in range(N):
                    p_next = ring.ptr(c + 1)
                    if c % 10 == 0:
                        vmax = max(vmax, float(ring.slots[(c + 1) % 2].float().abs().max()))
                    ctx.advect_ptrs([p_prev, p_next], s.times[c:c + 2], DCODE[dt], fp64=fp64)
                    p_prev = p_next
                fm = ctx.flowmap()
                torch.cuda.synchronize()
                res[key] = dict(end=fm["end"].cpu().numpy()[ids], flag=fm["flag"].cpu().numpy()[ids], vmax=vmax,
                                dt=dt, fp64=fp64)
            del ring
            torch.cuda.empty_cache()
        log(f"precision {name}: GPU runs of {len(ids)} sampled seeds done")
        pick = "one per lattice row, x index cycling" if every == 256 else f"every {every}th"
        out[name] = dict(wl=wl, series=s, ids=ids, seeds=lattice_points(wl.n, wl.stride, ids), runs=res,
                         label=f"{pick} of {wl.n_seeds} ({len(ids)})")
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


# Sweeps over the interval's grids (forward, recomputed forward, reverse) and
# FP64 state traffic per live particle-step of each adjoint variant.
ADJOINT_MODEL = {
    "seed_gradient": dict(sweeps=3, grid_grad=False, every_step=False),
    "seed_and_grid_gradient": dict(sweeps=3, grid_grad=True, every_step=False),
    "jacobian_ftle": dict(sweeps=3, grid_grad=False, every_step=False),
    "seed_gradient_checkpoint_every_step": dict(sweeps=2, grid_grad=False, every_step=True),
}


def adjoint_alg_bytes(touched, variant: str, k: int, bytes_per_point: int = 12, n_seeds: int = 0,
                      n_cot: int = 1) -> int:
    """Algorithmic bytes of one adjoint call from the exact touched points.

    touched: (N, 3) rows of (points of level n, points of level n + 1,
    particles entering step n).  Each sweep reads the touched points of both
    levels once per step; a grid gradient reads and writes the FP32 gradient
    (12 B) at every touched point of both levels; positions move as FP64
    (24 B): with checkpoints every k steps each checkpoint is written and read
    once and the recomputed step starts are written and read once per step;
    with a checkpoint at every step there is no recompute.  Cotangents in and
    seed gradients out are 12 B per seed and cotangent."""
    m = ADJOINT_MODEL[variant]
    t = np.asarray(touched, dtype=np.float64)
    pts = float(t[:, 0].sum() + t[:, 1].sum())
    live = float(t[:, 2].sum())
    grid = m["sweeps"] * pts * bytes_per_point
    if m["grid_grad"]:
        grid += 2 * pts * 12
    state = 48.0 * live if m["every_step"] else 48.0 * live + 48.0 * live / k
    return int(grid + state + 24 * n_seeds * n_cot)


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
        # exact touched points per step (stride 4: few shared corners)
        ctx.seed(wl.stride)
        touched = ctx.touched_points(dev, s.times)
        live = touched[:, 2].astype(np.float64)
        per = (touched[:, 0] + touched[:, 1]).astype(np.float64)
        out["touched_points"] = {
            "points_per_live_particle_step_both_levels": round(float(per.sum() / live.sum()), 3),
            "level_n_first_last": [int(touched[0, 0]), int(touched[-1, 0])],
            "live_first_last": [int(touched[0, 2]), int(touched[-1, 2])],
            "sweep_bytes": int(per.sum() * 12),
            "how": "bto_touched_points: distinct grid points each step samples per level (bitmap), 12 B per f32 point"}
        log(f"differentiation touched points: {out['touched_points']['points_per_live_particle_step_both_levels']} "
            f"per live particle-step over both levels")

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
            if name in ADJOINT_MODEL:
                alg = adjoint_alg_bytes(touched, name, k, n_seeds=wl.n_seeds, n_cot=3 if name == "jacobian_ftle" else 1)
                gbs = alg / (ms * 1e-3) / 1e9
                out[name]["roofline_effective"] = {
                    "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": alg,
                    "model": ADJOINT_MODEL[name],
                    "note": "effective: a step's two touched levels (sparse, stride 4) sit in the Infinity Cache"}
            log(f"differentiation {name}: {ms:.3f} ms")
    del dev, gg
    torch.cuda.empty_cache()
    return out


# Legs that --leg runs on their own (the default run adds the storage, ABC,
# precision, differentiation and paper-context legs to the headline).
LEGS = {
    "turb_256_storage": lambda log, copy_gbs: turb_storage_legs(log, copy_gbs),
    "abc_128": lambda log, copy_gbs: abc_128_leg(log, copy_gbs),
    "precision_turbulence": lambda log, copy_gbs: precision_leg(log),
    "paper_context": lambda log, copy_gbs: paper_context(log),
    "posthoc_accuracy": lambda log, copy_gbs: posthoc_accuracy(log),
    "insitu_overlap": lambda log, copy_gbs: [insitu_overlap(log, 128, 32), insitu_overlap(log, 256, 64)],
    "differentiation": lambda log, copy_gbs: differentiation(log),
    "per_cycle": lambda log, copy_gbs: per_cycle(log),
}


# --------------------------------------------------------------------------
# The in situ form: one advect call per cycle over the grids of cycles n, n+1
# --------------------------------------------------------------------------
TDT = {"f32": "float32", "f16": "float16", "bf16": "bfloat16"}
DCODE = {"f32": 0, "f16": 1, "bf16": 2}   # bto_dtype


def insitu_bytes_per_pstep(dt: str) -> int:
    """Per-unit figure of the in situ form: each live particle-step reads both
    resident levels over the 8 points its cell touches at the stride-2 lattice
    density, and reads and writes its 20 bytes of state: 2*8*b + 40 bytes."""
    return 2 * 8 * field_bytes_per_point(dt) + STATE_BYTES


class Ring:
    """Two device slots filled cycle by cycle by the turbulence generator: the
    grid of cycle c goes to slot c % 2, which the step of cycle c - 2 was the
    last to read (same stream, so the overwrite waits for it)."""

    def __init__(self, gen, n, dt):
        import torch

        self.gen, self.dt = gen, dt
        shape = (n[2], n[1], n[0], 3)
        self.slots = [torch.empty(shape, dtype=getattr(torch, TDT[dt]), device="cuda") for _ in range(2)]

    def ptr(self, c: int, fill: bool = True) -> int:
        if fill:
            self.gen.fill(c, self.dt, self.slots[c % 2])
        return self.slots[c % 2].data_ptr()


def run_insitu_interval(ctx, stride, N, grid_ptr, times, dcode, out, ev=None, fp64=False):
    """seed, N one-step advect calls, flow-map write.  grid_ptr(c) returns the
    device pointer of cycle c's grid (a ring slot, filled on the stream before
    the step that first reads it).  ev: (seed, steps[N], flowmap) event pairs."""
    if ev is not None:
        ev[0][0].record()
    ctx.seed(stride)
    if ev is not None:
        ev[0][1].record()
    p_prev = grid_ptr(0)
    for c in range(N):
        p_next = grid_ptr(c + 1)
        if ev is not None:
            ev[1][c][0].record()
        ctx.advect_ptrs([p_prev, p_next], times[c:c + 2], dcode, fp64=fp64)
        if ev is not None:
            ev[1][c][1].record()
        p_prev = p_next
    if ev is not None:
        ev[2][0].record()
    ctx.flowmap(out=out)
    if ev is not None:
        ev[2][1].record()


def _event_pairs(n):
    import torch

    return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]


def insitu_measure(ctx, wl, grid_ptr, times, dt, steps, warmup, log, fp64=False):
    """Counting pass (live particles entering every step), warm-up and timed
    intervals of the in situ form.  Returns the measurement record."""
    import torch

    N = wl.n_steps
    dcode = DCODE[dt]
    tuning = ctx.tuning()
    out = None
    # counting pass: live particles entering each step and the particle-steps
    ctx.seed(wl.stride)
    out = ctx.flowmap()
    live_in, psteps_c = [], []
    st = ctx.stats()
    p_prev = grid_ptr(0)
    for c in range(N):
        p_next = grid_ptr(c + 1)
        live_in.append(st["n_live"])
        ctx.advect_ptrs([p_prev, p_next], times[c:c + 2], dcode, fp64=fp64)
        st2 = ctx.stats()
        psteps_c.append(st2["particle_steps"] - st["particle_steps"])
        st = st2
        p_prev = p_next
    psteps = int(st["particle_steps"])
    n_valid = int(st["n_live"])
    assert sum(psteps_c) == psteps
    for _ in range(warmup):
        run_insitu_interval(ctx, wl.stride, N, grid_ptr, times, dcode, out, fp64=fp64)
    torch.cuda.synchronize()
    per = []
    t_wall = []
    for k in range(steps):
        ev = (_event_pairs(1)[0], _event_pairs(N), _event_pairs(1)[0])
        t0 = time.perf_counter()
        run_insitu_interval(ctx, wl.stride, N, grid_ptr, times, dcode, out, ev, fp64=fp64)
        torch.cuda.synchronize()
        t_wall.append(time.perf_counter() - t0)
        step_ms = np.array([a.elapsed_time(b) for a, b in ev[1]])
        per.append(dict(seed=ev[0][0].elapsed_time(ev[0][1]), steps=step_ms,
                        flowmap=ev[2][0].elapsed_time(ev[2][1])))
        assert ctx.stats()["particle_steps"] == psteps, "particle-step count changed between intervals"
    interval_ms = np.array([p["seed"] + p["steps"].sum() + p["flowmap"] for p in per])
    med = int(np.argsort(interval_ms)[len(interval_ms) // 2])
    # launches of the dominant kernel: steps whose call does not also re-sort
    R = tuning["rebin_every"]
    plain = np.array([R == 0 or c == 0 or c % R != 0 for c in range(N)])
    steps_ms = np.stack([p["steps"] for p in per])            # (intervals, N)
    launch_ms = float(np.median(steps_ms[:, plain].mean(axis=1)))
    live_plain = float(np.mean(np.asarray(live_in, dtype=np.float64)[plain]))
    bpp = insitu_bytes_per_pstep(dt)
    alg_launch = bpp * live_plain
    achieved = alg_launch / (launch_ms * 1e-3) / 1e9
    rec = {
        "interval_ms_median": float(interval_ms[med]), "interval_ms_all": [round(float(v), 4) for v in interval_ms],
        "seed_ms": round(per[med]["seed"], 4), "flowmap_ms": round(per[med]["flowmap"], 4),
        "steps_ms": round(float(per[med]["steps"].sum()), 4),
        "wall_s_per_interval_incl_generation": round(float(np.median(t_wall)), 3),
        "particle_steps": psteps, "valid_at_end": n_valid, "live_in": live_in,
        "launch_ms": launch_ms, "launches": int(plain.sum()), "live_per_launch": live_plain,
        "bytes_per_pstep": bpp, "alg_bytes_per_launch": alg_launch, "achieved_GBs": achieved,
        "rebin_step_extra_ms": (round(float(np.median(steps_ms[:, ~plain].mean(axis=1))) - launch_ms, 4)
                                if (~plain).any() else None),
        "tuning": tuning,
    }
    log(f"{wl.name} {dt} in situ: {psteps / (interval_ms[med] * 1e-3):.3e} particle-steps/s, interval "
        f"{interval_ms[med]:.2f} ms (steps {rec['steps_ms']:.2f}), launch {launch_ms * 1e3:.1f} us, "
        f"{achieved:.0f} GB/s at {bpp} B per particle-step")
    return rec


def traffic_record(workload: str, dt: str, form: str):
    """Counter traffic per launch of the dominant kernel (profiles/), while the
    kernel sources still hash to the value recorded with the counters."""
    f = os.path.join(ROOT, "profiles", f"traffic_{workload}_{dt}_{form}.json")
    if not os.path.exists(f):
        return None
    rec = json.load(open(f))
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec


def roofline_of(m, dt, workload, form, kernel, copy_gbs):
    traffic = traffic_record(workload, dt, form)
    roof = {"bound": "hbm", "achieved": round(m["achieved_GBs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(m["achieved_GBs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "kernel": kernel, "bytes_per_particle_step": m["bytes_per_pstep"],
            "particle_steps_per_launch": round(m["live_per_launch"], 1),
            "algorithmic_bytes_per_launch": int(m["alg_bytes_per_launch"]),
            "avg_launch_ms": round(m["launch_ms"], 5), "launches_averaged": m["launches"],
            "device_copy_GBs": round(copy_gbs, 1)}
    if traffic:
        roof["traffic_GBs"] = round(traffic["bytes_per_launch"] / (m["launch_ms"] * 1e-3) / 1e9, 1)
        roof["traffic_source"] = traffic.get("source")
    return roof


def turb_storage_legs(log, copy_gbs, steps=3, warmup=1):
    """The 256^3 precision workload (64-mode turbulence, 128^3 seeds, 50-step
    interval) in FP32, FP16 and BF16 storage: the in situ form (one call per
    cycle, two levels per step) with its roofline at the per-unit figure of
    that form, and the same interval with all 51 grids resident in fused
    launches (the one-level model, a footnote)."""
    import torch
    from bto_inputs import _turb
    from bto_inputs.workloads import WORKLOADS
    from paper_2004_02003_amd import Context

    wl = WORKLOADS["turb_256"]
    s = wl.make_field()
    gen = _turb.DeviceTurbulence(s.lazy)
    times = np.asarray(s.times, dtype=np.float64)
    shape = (wl.n[2], wl.n[1], wl.n[0], 3)
    out = {}
    dev, dev_dt = None, None
    for key, dt, fp64 in (("f32", "f32", False), ("f32_sampled_fp64", "f32", True), ("f16", "f16", False),
                          ("bf16", "bf16", False)):
        if dev_dt != dt:
            dev = None
            torch.cuda.empty_cache()
            dev = [gen.fill(c, dt, torch.empty(shape, dtype=getattr(torch, TDT[dt]), device="cuda"))
                   for c in range(wl.n_cycles)]
            dev_dt = dt
        ptrs = [g.data_ptr() for g in dev]
        with Context(wl.n, wl.n_seeds) as ctx:
            ctx.set_tuning(**insitu_shape(wl.name, dt))
            m = insitu_measure(ctx, wl, lambda c: ptrs[c], times, dt, steps, warmup, log, fp64=fp64)
            rec = {"value": round(m["particle_steps"] / (m["interval_ms_median"] * 1e-3), 1),
                   "interval_ms": round(m["interval_ms_median"], 4), "particle_steps": m["particle_steps"],
                   "valid_at_end": m["valid_at_end"],
                   "roofline": roofline_of(m, dt, wl.name, "insitu_fp64" if fp64 else "insitu",
                                           f"tile_gather_kernel<{dt},linear{',extended-precision sampling' if fp64 else ''}> + "
                                           f"tile_list_kernel (one step per call)", copy_gbs),
                   "tuning": m["tuning"]}
            # fused: all grids resident, several steps per launch (segment layout,
            # latched at the next seeding)
            ctx.set_tuning(**fused_shape(wl.name, dt))
            ts = []
            for r in range(warmup + steps):
                ctx.seed(wl.stride)
                e0, e1 = _event_pairs(1)[0]
                e0.record()
                ctx.advect_ptrs(ptrs, times, DCODE[dt], fp64=fp64)
                e1.record()
                torch.cuda.synchronize()
                if r >= warmup:
                    ts.append(e0.elapsed_time(e1))
            ps = ctx.stats()["particle_steps"]
            rec["fused_all_resident"] = {"value": round(ps / (np.median(ts) * 1e-3), 1),
                                         "advect_ms": round(float(np.median(ts)), 4), "tuning": ctx.tuning(),
                                         "one_level_model_bytes_per_particle_step": 8 * field_bytes_per_point(dt)}
        if fp64:
            rec["sampler"] = "extended precision (BTO_SAMPLE_FP64: FP64 sums and stage velocities, FP32 weights on corner differences)"
        out[key] = rec
        log(f"turb_256 {key}: in situ {rec['value']:.3e}, fused {rec['fused_all_resident']['value']:.3e} "
            f"particle-steps/s")
    dev = None
    torch.cuda.empty_cache()
    return out


# Launch shape per workload and storage (results do not depend on it).
# In situ (one step per call) the turbulent blocks keep their particles in
# the tile layout, sorted by tile (32 x 8 x 8 cells) and run in Hilbert tile order (the
# particles mix at 1.5 cells per step; the tile order keeps the grid lines a
# tile's particles read in L2 for its neighbours).  Fused (all grids
# resident, several steps per launch) they re-sort every few steps, and for
# FP32 grids two lanes per particle halve the cache lines a row load touches.
INSITU_SHAPE = {
    "turb_256": dict(tiles=2),
    "turb_512": dict(tiles=2),
}
FUSED_SHAPE = {
    "turb_256": dict(rebin_every=5, tiles=0),
    "turb_512": dict(rebin_every=10, tiles=0),
}


def insitu_shape(name, dt):
    return dict(INSITU_SHAPE.get(name, {}))


def fused_shape(name, dt):
    d = dict(FUSED_SHAPE.get(name, {}))
    if dt == "f32" and name.startswith("turb"):
        d["lanes_per_particle"] = 2
    return d


def abc_128_leg(log, copy_gbs, steps=5, warmup=1):
    """The 128^3 ABC block (FP32, 64^3 seeds, 100-step interval), whose two
    grid levels fit the Infinity Cache (an effective-bandwidth figure, not an
    HBM one): all grids resident in fused launches (the fast form when cycles
    are resident), and the in situ form, one call per cycle."""
    import torch
    from bto_inputs.workloads import WORKLOADS
    from paper_2004_02003_amd import Context, grid_to_device

    wl = WORKLOADS["abc_128"]
    s = wl.make_field()
    dev = [grid_to_device(g, "f32") for g in s.grids("f32")]
    ptrs = [g.data_ptr() for g in dev]
    times = np.asarray(s.times, dtype=np.float64)
    out = {}
    with Context(wl.n, wl.n_seeds) as ctx:
        tuning = ctx.tuning()
        ts = []
        for r in range(warmup + steps):
            ctx.seed(wl.stride)
            e0, e1 = _event_pairs(1)[0]
            e0.record()
            ctx.advect_ptrs(ptrs, times, DCODE["f32"])
            e1.record()
            torch.cuda.synchronize()
            if r >= warmup:
                ts.append(e0.elapsed_time(e1))
        ps = ctx.stats()["particle_steps"]
        plan = launch_plan(wl.n_steps, tuning["steps_per_launch"], tuning["rebin_every"])
        out["fused_all_resident"] = {"value": round(ps / (np.median(ts) * 1e-3), 1),
                                     "advect_ms": round(float(np.median(ts)), 4), "launches": len(plan),
                                     "particle_steps": int(ps), "tuning": tuning}
        m = insitu_measure(ctx, wl, lambda c: ptrs[c], times, "f32", steps, warmup, log)
        out["insitu"] = {"value": round(m["particle_steps"] / (m["interval_ms_median"] * 1e-3), 1),
                         "interval_ms": round(m["interval_ms_median"], 4),
                         "roofline_effective": roofline_of(m, "f32", wl.name, "insitu", "advect<f32,linear>",
                                                           copy_gbs)}
    log(f"abc_128: fused {out['fused_all_resident']['value']:.3e}, in situ {out['insitu']['value']:.3e}")
    del dev
    torch.cuda.empty_cache()
    return out


def cpu_baseline_of(wl, series, dt, turb, grids_host, log, target_s=10.0):
    """The FP64 oracle, as it stands, on a bounded seed sample of the workload,
    on all host cores and on one; particle-steps counted as on the GPU."""
    import oracle

    P = wl.n_seeds
    from bto_inputs.workloads import lattice_dims, row_sample_ids

    every = 1 if not turb else (4096 if wl.n[0] >= 512 else 1024)
    ids = row_sample_ids(lattice_dims(wl.n, wl.stride), P // every) if every > 1 else np.arange(P)
    seeds = oracle.seed_lattice(wl.n, wl.stride)[ids]
    N = wl.n_steps
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    F = oracle.Field(wl.n, grids_host, dtype=dt) if not turb else oracle.Field.lazy_turbulence(series, dt)
    log(f"oracle CPU baseline on {len(ids)} seeds, {threads} threads")
    tc, reps, ps = 0.0, 0, 0
    while tc < target_s and reps < 50:
        t1 = time.perf_counter()
        o = oracle.flowmap(F, series.times, seeds, N, nthreads=threads)
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
    field_note = ("grid values evaluated on demand from the field's modes and rounded to the storage type"
                  if turb else "dense grids")
    res = {"value": round(ps / tc, 1), "unit": "particle-RK4-steps/s", "cores": threads, "kind": "oracle",
           "cpu": cpu_model, "nproc": os.cpu_count(),
           "sample": f"{'all' if every == 1 else f'one in {every} ({len(ids)}, spread over the lattice rows)'} seed(s) of {wl.name} ({len(ids)} seeds x {N} "
                     f"steps, {dt} storage, {field_note}) x {reps} repeats, {ps} particle-steps in {tc:.1f} s, "
                     f"FP64, OpenMP"}
    ids1 = ids[::16]
    t1 = time.perf_counter()
    o1 = oracle.flowmap(F, series.times, seeds[::16], N, nthreads=1)
    t1 = time.perf_counter() - t1
    ps1 = int(np.where(o1["flag"] == 0, N, o1["exit"] + 1).sum())
    one = {"value": round(ps1 / t1, 1), "unit": "particle-RK4-steps/s", "cores": 1, "kind": "oracle",
           "sample": f"{len(ids1)} seeds x {N} steps, {ps1} particle-steps in {t1:.1f} s, FP64"}
    return res, one


def cpu_reference_errors(gpu, threads, log):
    """The oracle side of the stated error (part of the CPU baseline leg: the
    only bench step that runs the oracle).  For each sampled seed of
    precision_gpu_runs: the FP64 oracle on the FP64 field with its tangent,
    then per storage type the end-position error of the GPU path (mean, p99,
    max over the seeds valid on both sides, the share beyond 1e-5 cells) and
    the first-order bound ||J|| N h max|V| sqrt(3) (u_storage + 2^-21) per seed
    (J from the oracle's tangent, u the storage's unit roundoff, 2^-21 the FP32
    sampling, kept for the extended-precision sampler, whose FP32 sums run over
    corner differences)."""
    import oracle

    out = {}
    for name, g in gpu.items():
        wl, s = g["wl"], g["series"]
        N = wl.n_steps
        t0 = time.perf_counter()
        o = oracle.flowmap(oracle.Field.lazy_turbulence(s, "f64"), s.times, g["seeds"], N, jac=True, nthreads=threads)
        log(f"precision {name}: FP64 oracle on {len(g['ids'])} seeds in {time.perf_counter() - t0:.1f} s")
        nJ = np.linalg.norm(o["jac"], axis=(1, 2), ord=2)
        safe = o["margin"] >= 1e-6
        res = {}
        for key, r in g["runs"].items():
            end, flag = r["end"], r["flag"]
            both = (flag == 0) & (o["flag"] == 0)
            err = np.linalg.norm(end[both] - o["end"][both], axis=1)
            bound = (nJ[both] * N * wl.dt * r["vmax"] * np.sqrt(3.0) *
                     (UNIT_ROUNDOFF[r["dt"]] + 2.0 ** -21))
            res[key] = {"mean": float(err.mean()), "p99": float(np.quantile(err, 0.99)), "max": float(err.max()),
                        "n": int(both.sum()), "beyond_1e-5_pct": round(100.0 * float((err > 1e-5).mean()), 3),
                        "within_first_order_bound_pct": round(100.0 * float((err <= bound).mean()), 2),
                        "bound_median": float(np.median(bound)),
                        "flag_disagree": int((flag != o["flag"]).sum()),
                        "flag_disagree_outside_margin": int(((flag != o["flag"]) & safe).sum())}
            log(f"precision {name} {key}: {res[key]}")
        out[name] = {"seeds": g["label"], "steps": N, "cells": "end-position L2 error, cells", **res}
    return out


def precision_leg(log):
    gpu = precision_gpu_runs(log)
    return cpu_reference_errors(gpu, int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count(), log)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed intervals (median reported)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="turb_512", choices=("turb_512", "turb_256"))
    ap.add_argument("--dtype", default=None, help="storage type (default: f16 for turb_512, f32 for turb_256)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="headline only (no legs)")
    ap.add_argument("--rebin-every", type=int, default=None,
                    help="re-sort live particles every this many steps (0 = never; default per workload)")
    ap.add_argument("--lanes-per-particle", type=int, default=None, choices=(1, 2),
                    help="FP32 grids: lanes per particle (default per workload)")
    ap.add_argument("--tiles", type=int, default=None, choices=(0, 1, 2),
                    help="particle layout: 0 segments, 1 LDS-staged tiles, 2 tiles (default per workload)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--leg", action="append", choices=sorted(LEGS),
                    help="run only these legs (repeatable) and print their results as one JSON line")
    args = ap.parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the per-block BTO path has no cross-GPU work "
              "(blocks are independent); run one process per block instead.", file=sys.stderr)
        sys.exit(2)

    if args.leg:
        import torch
        from paper_2004_02003_amd import _lib

        _lib.load()
        assert torch.cuda.is_available(), "bench.py needs a HIP device"
        copy_gbs = device_copy_rate()
        print(json.dumps({name: LEGS[name](log, copy_gbs) for name in args.leg}), flush=True)
        return

    import torch
    from bto_inputs import _turb
    from bto_inputs.workloads import WORKLOADS
    from paper_2004_02003_amd import Context
    from paper_2004_02003_amd import _lib

    _lib.load()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    wl = WORKLOADS[args.workload]
    dt = args.dtype or ("f16" if wl.name == "turb_512" else "f32")
    series = wl.make_field()
    gen = _turb.DeviceTurbulence(series.lazy)
    times = np.asarray(series.times, dtype=np.float64)
    ring = Ring(gen, wl.n, dt)
    # generation time of one grid (excluded from the timed region)
    e0, e1 = _event_pairs(1)[0]
    ring.ptr(0)
    e0.record()
    ring.ptr(1)
    e1.record()
    torch.cuda.synchronize()
    gen_ms = e0.elapsed_time(e1)
    log(f"workload {wl.name} ({dt}): two-slot ring of {2 * ring.slots[0].numel() * ring.slots[0].element_size() / 2**30:.2f} "
        f"GiB, one grid generated in {gen_ms:.2f} ms")

    ctx = Context(wl.n, wl.n_seeds)
    tune = insitu_shape(wl.name, dt)
    if args.rebin_every is not None:
        tune["rebin_every"] = args.rebin_every
    if args.lanes_per_particle is not None:
        tune["lanes_per_particle"] = args.lanes_per_particle
    if args.tiles is not None:
        tune["tiles"] = args.tiles
    if tune:
        ctx.set_tuning(**tune)
    m = insitu_measure(ctx, wl, ring.ptr, times, dt, args.steps, args.warmup, log)
    ctx.close()
    del ring
    torch.cuda.empty_cache()
    value = m["particle_steps"] / (m["interval_ms_median"] * 1e-3)
    copy_gbs = device_copy_rate()
    kname = (f"tile_gather_kernel<{dt},linear> + tile_list_kernel (one step per call)" if m["tuning"].get("tiles")
             else f"advect_kernel<{dt},linear> (one step per call)")
    roof = roofline_of(m, dt, wl.name, "insitu", kname, copy_gbs)
    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "particle-RK4-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(m["interval_ms_median"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dt,
        "data": "synthetic (seeded divergence-free Fourier-mode turbulence generated on the device; no dataset)",
        "config": {"workload": wl.name, "n": list(wl.n), "cycles": wl.n_cycles, "dt": wl.dt,
                   "stride": wl.stride, "seeds": wl.n_seeds, "interval_steps": wl.n_steps, "storage": dt,
                   "arithmetic": "fp32 sampling, fp64 positions", "resident_grids": 2,
                   "form": "one advect call per cycle (in situ)",
                   "particle_steps_per_interval": m["particle_steps"], "valid_at_end": m["valid_at_end"],
                   "tuning": m["tuning"]},
        "timing": {"interval_ms_all": m["interval_ms_all"], "seed_ms": m["seed_ms"], "steps_ms": m["steps_ms"],
                   "flowmap_ms": m["flowmap_ms"], "rebin_step_extra_ms": m["rebin_step_extra_ms"],
                   "grid_generation_ms_per_cycle": round(gen_ms, 3),
                   "wall_s_per_interval_incl_generation": m["wall_s_per_interval_incl_generation"],
                   "how": "median over the timed intervals of HIP-event times (seed + every step + flow-map "
                          "write) on the stream the kernels run on; grid generation is excluded"},
        "roofline": roof,
    }
    if not args.no_variants:
        result["turb_256_storage"] = turb_storage_legs(log, copy_gbs)
        result["abc_128"] = abc_128_leg(log, copy_gbs)
        precision_gpu = precision_gpu_runs(log)
        result["differentiation"] = differentiation(log)
        result["paper_context"] = paper_context(log)
    if not args.no_cpu_baseline:
        # the CPU baseline leg: the oracle timed on a bounded sample, and (with
        # the legs) the oracle's FP64 references for the stated error
        result["cpu_baseline"], result["cpu_baseline_1thread"] = cpu_baseline_of(wl, series, dt, True, None, log)
        if not args.no_variants:
            result["precision_turbulence"] = cpu_reference_errors(
                precision_gpu, int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count(), log)

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
