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


def test_measured_traffic_only_for_the_measured_kernel(monkeypatch):
    """The roofline traffic figure applies only to the kernel sources it was measured on."""
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    rec = {"config": 4, "fetch_kib": 100.0, "write_kib": 10.0, "fetch_scale": 2.0,
           "write_scale": 1.0}
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", {h: rec})
    assert bench.measured_traffic(4) == 1024.0 * (200.0 + 10.0)
    assert bench.measured_traffic(3) is None
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", {"0" * 64: rec})
    assert bench.measured_traffic(4) is None


def test_first_staying_index():
    """Evaluations to a target count from the generation after which the error stays below it."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench._first_staying([6.0, 4.0, 6.0, 4.5, 4.0], 5.0) == 3
    assert bench._first_staying([4.0, 4.0], 5.0) == 0
    assert bench._first_staying([4.0, 6.0], 5.0) is None
    assert bench._first_staying([], 5.0) is None
