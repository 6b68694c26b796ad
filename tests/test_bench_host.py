"""Host-side logic of bench.py (no GPU): the one-GPU refusal, steps per
launch of each kind of kernel variant, and the algorithmic bytes per
lattice update the roofline uses (2 q sizeof(population))."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_steps_per_launch():
    assert bench.steps_per_launch("128x4/t2/r32/nt") == 2
    assert bench.steps_per_launch("256x1/npt1") == 1
    assert bench.steps_per_launch("128x4/npt2/r16/nt/rev") == 1
    # the resident D1Q3 kernel: up to RESIDENT_STEPS steps per launch
    assert bench.steps_per_launch("resident2048", 20000) == bench.RESIDENT_STEPS
    assert bench.steps_per_launch("resident2048", 100) == 100


def test_bytes_per_lattice_update():
    assert bench.bytes_per_node(synth.cavity_2d(n=64)) == 72          # D2Q9 FP32
    assert bench.bytes_per_node(synth.planar_2d(n=64)) == 40          # D2Q5 FP32
    assert bench.bytes_per_node(synth.stefan_1d(nx=64)) == 48         # D1Q3 FP64
    assert bench.bytes_per_node(synth.cavity_3d(n=8, q=19)) == 152    # D3Q19 FP32
    assert bench.bytes_per_node(synth.cavity_3d(n=8, q=7)) == 56      # D3Q7 FP32


def test_traffic_of_an_unmeasured_variant_is_null():
    assert bench.measured_traffic("cavity2d_d2q9_f32_8192x8192",
                                  "no/such/variant") is None


def test_default_variants_exist():
    """Every fixed variant the bench times is in the library's table of
    its lattice (the names the profiles in profiles/ are taken under)."""
    lattice = {"cavity": (9, "f32"), "cavity_eebm": (9, "f32"),
               "planar": (5, "f32"), "planar_eebm": (5, "f32"),
               "stefan1d": (3, "f64"), "batched": (5, "f32"),
               "adjoint": (5, "f32"), "cube3d_19": (19, "f32"),
               "cube3d_7": (7, "f32")}
    assert set(lattice) == set(bench.DEFAULT_VARIANTS)
    for key, name in bench.DEFAULT_VARIANTS.items():
        q, s = lattice[key]
        assert bench.variant_id(q, s, name) >= 0, key


def test_cpu_baseline_strips_equal_single_thread():
    """The multi-core oracle leg cuts the lattice into row strips with halo
    rows; their own rows equal the single-thread run bit for bit."""
    r = bench.cpu_baseline(synth.cavity_2d(n=96, ny=80), steps=3, threads=4)
    assert r["strips_equal_single_thread"] is True
    assert r["cores"] == 4 and r["kind"] == "oracle" and r["value"] > 0
    r = bench.cpu_baseline(synth.planar_2d(n=64, ny=50), steps=5, threads=3)
    assert r["strips_equal_single_thread"] is True


def test_batch_kernel_names_by_variant():
    """The trace names the profile summary looks up for a batched launch:
    split two-step variants run the front kernel, the quiet pass and the
    full pass (IREBM) or the plain two-step kernel (EEBM)."""
    import bench
    k = bench.batch_kernels("128x2/t2s/r96/nt")
    assert k == {"front": "batch_front_kernel<5, float, 0>",
                 "quiet": "batch_step2_kernel<5, float, 0, 2, 128, 1>",
                 "full": "batch_step2_kernel<5, float, 0, 2, 128, 2>"}
    assert bench.batch_kernels("128x2/t2s/r96/nt", 2) == {
        "two-step": "batch_step2_kernel<5, float, 2, 2, 128, 0>"}
    assert bench.batch_kernels("128x4/t2/r32/nt") == {
        "two-step": "batch_step2_kernel<5, float, 0, 4, 128, 0>"}
    assert bench.batch_kernels("128x4/npt2/r16/nt") == {
        "one-step": "batch_step_kernel<5, float, 2, 0, true>"}


def test_batch_walls_from_trace_rows():
    """Wall time of a launch: first start to last end of its kernels."""
    import sqlite3
    import bench
    c = sqlite3.connect(":memory:")
    c.execute("create table kernels (name text, start int, end int)")
    rows = [("f", 0, 900), ("q", 10, 1000), ("x", 1005, 1020),
            ("f", 2000, 2500), ("q", 2001, 3000), ("x", 3002, 3010)]
    c.executemany("insert into kernels values (?, ?, ?)", rows)
    w = bench.batch_walls(c, lambda n: n, {"front": "f", "quiet": "q",
                                           "full": "x"})
    assert w == [1.02, 1.01]


def test_cube3d_kernel_names_by_variant():
    """The trace names of a 3D step: a split variant runs the front strip
    with variant 0's kernel, the quiet pass and the full pass (IREBM)."""
    import bench
    assert bench.cube3d_kernels(7, "64x4/npt1/z8/nt/s") == {
        "front": "step3_kernel<7, float, 1, 0, true, 0>",
        "quiet": "step3_kernel<7, float, 1, 0, true, 1>",
        "full": "step3_kernel<7, float, 1, 0, true, 2>"}
    assert bench.cube3d_kernels(7, "64x4/npt1/z8/nt/s", 2) == {
        "step": "step3_kernel<7, float, 1, 2, true, 0>"}
    assert bench.cube3d_kernels(19, "256x1/npt2/z4/nt") == {
        "step": "step3_kernel<19, float, 2, 0, true, 0>"}
