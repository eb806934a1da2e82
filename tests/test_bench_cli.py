"""Host-side checks of the benchmark script: the one-GPU rule of its command
line, and that its recorded HBM traffic belongs to the instance kernel as the
sources now stand (the figure is dropped when they change)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_tied_to_batch_and_sources():
    b = _bench()
    # fetch counters read half the bytes a plain copy moves, write counters all of them
    assert abs(b.TRAFFIC["fetch_scale"] - 2.0) < 0.01 and b.TRAFFIC["write_scale"] == 1.0
    saved = b.TRAFFIC["sources_sha256"]
    try:
        # reported for the sources it was measured on, at its batch size only
        b.TRAFFIC["sources_sha256"] = b.kernel_sources_sha256()
        t = b.traffic_bytes(b.TRAFFIC["instances"])
        assert t is not None and t > 0
        assert b.traffic_bytes(b.TRAFFIC["instances"] // 2) is None
        # and dropped once they change
        b.TRAFFIC["sources_sha256"] = "0" * 64
        assert b.traffic_bytes(b.TRAFFIC["instances"]) is None
    finally:
        b.TRAFFIC["sources_sha256"] = saved


def test_kernel_sources_exist():
    b = _bench()
    for name in b.KERNEL_SOURCES:
        assert os.path.isfile(os.path.join(ROOT, name)), name
