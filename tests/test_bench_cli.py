"""CPU checks of the benchmark's command line and host logic: more than one
GPU is refused with a message (the benchmark measures one GPU) before
anything touches a device, and measured HBM traffic is reported only for the
workload the counters were taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_is_reported_only_for_the_counted_workload():
    sys.path.insert(0, ROOT)
    try:
        import bench
    finally:
        sys.path.remove(ROOT)
    here = bench.device_sources_hash() == bench.TRAFFIC_SOURCES
    for regen in (0, 1):
        tb = bench.traffic_bytes("k_rollout4", (8192, 100, "fp32", regen))
        assert (tb is not None) == here
        if here:
            f, w = bench.TRAFFIC_KIB[("k_rollout4", regen)]
            assert abs(tb - (f * bench.FETCH_SCALE + w * bench.WRITE_SCALE) * 1024.0) < 1e-6
    if here:
        # drawing the samples again removes the sample tensor from both kernels
        assert bench.traffic_bytes("k_rollout4", (8192, 100, "fp32", 1)) < 1e6
        assert bench.traffic_bytes("k_final", (8192, 100, "fp32", 1)) < 1e6
    for wl in [(32767, 100, "fp32", 0), (8192, 200, "fp32", 0), (8192, 100, "fp64", 0), None]:
        assert bench.traffic_bytes("k_rollout4", wl) is None
        assert bench.traffic_bytes("k_final", wl) is None
    assert bench.traffic_bytes("k_rollout", (8192, 100, "fp32", 0)) is None
