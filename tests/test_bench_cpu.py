"""Host-side checks of the benchmark driver and of the stored workload inputs."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_stored_workloads_are_the_oracle_output():
    """workload/data/config{0,1}.npz are exactly what the committed generator writes."""
    from oracle import synth
    from workload import WORKLOADS, make_hand_model, seed_sequence
    for idx in (0, 1):
        cfg = WORKLOADS[idx]
        d = np.load(os.path.join(ROOT, "workload", "data", f"config{idx}.npz"))
        model = make_hand_model(seed_sequence(idx, 10_000), cfg.n_hands)
        fr = synth.make_frame(model, cfg, 0)
        assert np.array_equal(d["depth_0"], fr["depth"])
        assert np.array_equal(d["skin_0"], fr["skin"])
        assert np.array_equal(d["h_true"][0], fr["h_true"])
        assert tuple(d["cam"][0]) == fr["cam"]
        assert d["flops_per_eval"] > 0


def test_joint_error_metric():
    sys.path.insert(0, ROOT)
    import bench
    h = np.zeros(52)
    t = np.zeros(52)
    t[:20] = np.deg2rad(2.0)
    assert abs(bench.joint_error_deg(h[:26], t[:26], 1) - 2.0) < 1e-12
    assert abs(bench.joint_error_deg(h, t, 2) - 1.0) < 1e-12


def test_measured_counters_only_for_the_measured_kernel(monkeypatch):
    """The roofline traffic and executed-FLOP figures apply only to the kernel sources they
    were measured on."""
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    rec = {"config": 4, "fetch_kib": 100.0, "write_kib": 10.0, "fetch_scale": 2.0,
           "write_scale": 1.0, "fp32_flop": 3.0e9}
    monkeypatch.setattr(bench, "MEASURED_COUNTERS", {h: rec})
    assert bench.measured_counters(4) == (1024.0 * (200.0 + 10.0), 3.0e9)
    assert bench.measured_counters(3) == (None, None)
    monkeypatch.setattr(bench, "MEASURED_COUNTERS", {"0" * 64: rec})
    assert bench.measured_counters(4) == (None, None)


def test_roofline_achieved_never_exceeds_the_executed_rate():
    """The reported rate is the definition's W x particles / duration, capped by the executed
    FP32 rate; the hit-tile figure and the byte ratio are reported beside it."""
    sys.path.insert(0, ROOT)
    import bench
    work = {"flops_per_eval": 4.0e6, "flops_hit_tiles_per_eval": 1.0e6}
    model = {"n_dof": 52, "prim_type": np.zeros(80, np.int32)}
    frames = [{"depth": np.zeros((480, 640), np.uint16)}]
    r = bench.roofline_figures(work, 0.1, 500.0, model, frames, (None, None))
    assert abs(r["achieved"] - 4.0e6 * 500 / 1e-4 / 1e12) < 1e-9
    assert r["executed"] is None and r["traffic_over_algorithmic"] is None
    r = bench.roofline_figures(work, 0.1, 500.0, model, frames, (3.0e7, 1.0e9))
    assert abs(r["achieved"] - 10.0) < 1e-9 and abs(r["executed"] - 10.0) < 1e-9
    assert r["achieved_definition"] > r["achieved"] > r["achieved_hit_tiles"]
    assert abs(r["traffic_over_algorithmic"] - 3.0e7 / (500 * 212 + 3 * 640 * 480)) < 1e-9


def test_stored_work_counts_reproduce_the_flop_figures():
    """The stored FLOP figures are the per-unit counts applied to the stored coverage."""
    from oracle import flops
    for idx in range(7):
        d = np.load(os.path.join(ROOT, "workload", "data", f"config{idx}.npz"))
        assert d["flops_per_eval"] == flops.flops_from_counts(d["cov_per_eval"],
                                                              d["pixels_per_eval"])
        assert d["flops_hit_tiles_per_eval"] == flops.flops_from_counts(
            d["cov_per_eval"], d["hit_tile_pixels_per_eval"])
        assert 0 < d["hit_tile_pixels_per_eval"] <= d["pixels_per_eval"]


def test_first_staying_index():
    """Evaluations to a target count from the generation after which the error stays below it."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench._first_staying([6.0, 4.0, 6.0, 4.5, 4.0], 5.0) == 3
    assert bench._first_staying([4.0, 4.0], 5.0) == 0
    assert bench._first_staying([4.0, 6.0], 5.0) is None
    assert bench._first_staying([], 5.0) is None
