"""Host-side logic of bench.py (no GPU): the launch plan mirrors the library's
balanced split, the algorithmic-bytes model is the stated per-unit figure,
the per-workload launch shapes name real workloads, the entry point
refuses more than one GPU before touching a device, and the committed
headline line's roofline follows from its own fields and the counter record
of the current kernel sources."""

import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_launch_plan_matches_the_library_split(bench):
    assert bench.launch_plan(100, 32, 0) == [25, 25, 25, 25]
    assert bench.launch_plan(100, 32, 5) == [5] * 20          # re-sorting caps the launch length
    assert bench.launch_plan(7, 32, 0) == [7]
    assert bench.launch_plan(50, 128, 0) == [50]
    plan = bench.launch_plan(201, 32, 0)
    assert sum(plan) == 201 and max(plan) - min(plan) <= 1 and max(plan) <= 32


def test_insitu_per_unit_figure(bench):
    # two grid levels over the 8 points of a stride-2 particle's cell, plus 20 B
    # of state read and 20 B written, per live particle-step
    assert bench.insitu_bytes_per_pstep("f16") == 136
    assert bench.insitu_bytes_per_pstep("bf16") == 136
    assert bench.insitu_bytes_per_pstep("f32") == 232


def test_launch_shapes_and_tables_are_consistent(bench):
    from bto_inputs.workloads import WORKLOADS

    assert set(bench.INSITU_SHAPE) <= set(WORKLOADS) and set(bench.FUSED_SHAPE) <= set(WORKLOADS)
    for name in WORKLOADS:
        for dt in ("f32", "f16", "bf16"):
            for shape in (bench.insitu_shape(name, dt), bench.fused_shape(name, dt)):
                assert set(shape) <= {"steps_per_launch", "rebin_every", "blocks_per_cu", "lanes_per_particle",
                                      "tiles"}
                assert shape.get("lanes_per_particle", 1) == 1 or dt == "f32"
    assert set(bench.PAPER_ABC_TABLE_MS) == {(i, s) for i in (25, 50, 100) for s in (1, 2, 3)}
    assert set(bench.UNIT_ROUNDOFF) == {"f32", "f16", "bf16"}
    for fn in ("paper_context", "posthoc_accuracy", "insitu_overlap", "precision_gpu_runs", "cpu_reference_errors", "differentiation",
               "per_cycle", "kernel_hash", "main", "insitu_measure", "run_insitu_interval", "turb_storage_legs",
               "abc_128_leg", "cpu_baseline_of", "roofline_of"):
        assert callable(getattr(bench, fn)), fn
    assert set(bench.LEGS) == {"turb_256_storage", "abc_128", "precision_turbulence", "paper_context",
                               "posthoc_accuracy", "insitu_overlap", "differentiation", "per_cycle"}
    assert all(callable(f) for f in bench.LEGS.values())


def test_unknown_leg_is_refused(bench):
    with pytest.raises(SystemExit) as e:
        bench.main(["--leg", "no_such_leg"])
    assert e.value.code == 2


def test_more_than_one_gpu_is_refused(bench):
    with pytest.raises(SystemExit) as e:
        bench.main(["--gpus", "2"])
    assert e.value.code == 2


def test_seed_subsets_spread_over_the_lattice():
    import numpy as np

    import oracle
    from bto_inputs.workloads import lattice_dims, lattice_points, row_sample_ids

    for n, stride in (((37, 23, 19), 3), ((40, 30, 20), 2), ((16, 16, 16), 4)):
        m = lattice_dims(n, stride)
        lat = oracle.seed_lattice(n, stride)
        assert int(np.prod(m)) == len(lat)
        ids = np.arange(len(lat))
        assert np.array_equal(lattice_points(n, stride, ids), lat)
        assert np.array_equal(lattice_points(n, stride, ids[::7]), lat[::7])
    m = (256, 256, 256)
    ids = row_sample_ids(m, 65536)
    assert len(ids) == 65536 and len(np.unique(ids)) == 65536 and ids.max() < 256 ** 3
    x, row = ids % 256, ids // 256
    assert np.array_equal(np.bincount(x), np.full(256, 256))        # every x index equally often
    assert np.array_equal(row, np.arange(65536))                     # one seed per row
    ids = row_sample_ids(m, 4096)
    assert len(ids) == 4096 and np.array_equal(np.bincount(ids % 256), np.full(256, 16))
    assert np.all(np.diff(ids // 256) == 16)


def test_adjoint_byte_model_from_touched_points(bench):
    import numpy as np

    # two steps: 100 + 120 points of level n, 110 + 90 of level n + 1, 10 and 8 particles
    t = np.array([[100, 110, 10], [120, 90, 8]], dtype=np.uint64)
    pts, live = 420, 18
    assert bench.adjoint_alg_bytes(t, "seed_gradient", 2, n_seeds=10) == int(
        3 * pts * 12 + 48 * live + 48 * live / 2 + 24 * 10)
    assert bench.adjoint_alg_bytes(t, "seed_and_grid_gradient", 2, n_seeds=10) == int(
        3 * pts * 12 + 2 * pts * 12 + 48 * live + 48 * live / 2 + 24 * 10)
    assert bench.adjoint_alg_bytes(t, "seed_gradient_checkpoint_every_step", 2, n_seeds=10) == int(
        2 * pts * 12 + 48 * live + 24 * 10)
    assert bench.adjoint_alg_bytes(t, "jacobian_ftle", 2, n_seeds=10, n_cot=3) == int(
        3 * pts * 12 + 48 * live + 48 * live / 2 + 24 * 30)


def test_committed_bench_line_is_self_consistent(bench):
    """The committed line of the headline workload: its roofline fraction is
    the algorithmic bytes per launch (particle-steps per launch x the per-unit
    figure) over the average launch time, against 8 TB/s; its value is the
    interval's particle-steps over the interval time; its traffic is the
    counter record taken on the kernel sources now in the tree."""
    import json

    line = json.load(open(os.path.join(ROOT, "profiles", "bench_turb512_f16.json")))
    assert line["n_gpus"] == 1 and line["config"]["workload"] == "turb_512"
    r = line["roofline"]
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert r["bytes_per_particle_step"] == bench.insitu_bytes_per_pstep("f16")
    alg = r["particle_steps_per_launch"] * r["bytes_per_particle_step"]
    assert abs(alg - r["algorithmic_bytes_per_launch"]) <= 1e-6 * alg + 1
    achieved = r["algorithmic_bytes_per_launch"] / (r["avg_launch_ms"] * 1e-3) / 1e9
    assert abs(achieved - r["achieved"]) <= 1e-3 * achieved
    assert abs(r["frac"] - r["achieved"] / r["peak"]) <= 1e-4
    value = line["config"]["particle_steps_per_interval"] / (line["ms_per_step"] * 1e-3)
    assert abs(value - line["value"]) <= 1e-3 * value
    # the traffic came from the counter record of the same kernel sources
    rec = bench.traffic_record("turb_512", "f16", "insitu")
    assert rec is not None, "counter record missing or taken on other kernel sources"
    assert r["traffic"] == rec["bytes_per_launch"]
    assert os.path.exists(os.path.join(ROOT, "profiles", rec["source"]))
