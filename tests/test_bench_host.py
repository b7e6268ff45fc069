"""Host-side checks of bench.py and the synthetic input recipes
(no GPU needed)."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_summary_matches_its_sources_or_is_ignored():
    h = bench.source_hash()
    assert len(h) == 16
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    d = json.load(open(path))
    assert {"source_hash", "fetch_scale", "write_scale", "kernels"} <= set(d)
    t = bench.pmc_traffic("k_apply_mfma", 1.0)
    if d["source_hash"] == h:
        assert t == d["kernels"]["k_apply_mfma"]["hbm_bytes_per_launch"]
    else:
        assert t is None


def test_batched_recipe_shapes():
    shapes = synth.batched_shapes(512)
    assert len(shapes) == 512
    for I, r in shapes:
        assert len(I) == 8 and len(r) == 7
        assert all(64 <= i <= 4096 for i in I)
        assert all(1 <= x <= 31 for x in r)


def test_sum_workload_sizes():
    # the measured workload: N = 16, I = 262144, ranks 20 + 20 -> 40, 47.14 GB of X cores
    nbytes = synth.core_bytes_of_sum([262144] * 16, [40] * 15)
    assert nbytes == 8 * 262144 * (2 * 40 + 14 * 40 * 40)
    assert abs(nbytes / 1e9 - 47.14) < 0.01


def test_generators_are_seeded():
    a = synth.random_tt(1, 0, "A", [8, 9, 10], [3, 4], scaled=True)
    b = synth.random_tt(1, 0, "A", [8, 9, 10], [3, 4], scaled=True)
    c = synth.random_tt(1, 1, "A", [8, 9, 10], [3, 4], scaled=True)
    assert [x.shape for x in a] == [(1, 8, 3), (3, 9, 4), (4, 10, 1)]
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not all(np.array_equal(x, y) for x, y in zip(a, c))


def test_every_leg_and_switch_parses():
    # the switches parse before the GPU-count check, which then exits with 2
    for extra in (["--leg", "norms"], ["--leg", "sum3"], ["--leg", "batched", "--no-per-tensor"],
                  ["--no-norms", "--no-mirror", "--no-sum3", "--no-batched", "--no-large", "--no-cpu-baseline"]):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"] + extra,
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2 and "one GPU" in r.stderr, (extra, r.stderr)
