"""bench.py command line on the host (no GPU): more than one GPU is refused
before anything is imported or launched, and the recorded traffic counters
are only used while the kernel source they were taken on is unchanged."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_records_match_their_sources():
    sys.path.insert(0, ROOT)
    import bench
    for wl in ("mri_256", "msfa_512", "cacti_1024"):
        rec = json.load(open(bench.traffic_file(wl)))
        for name, k in rec["kernels"].items():
            src = os.path.join(ROOT, k["source"])
            assert os.path.exists(src), src
            fresh = hashlib.sha256(open(src, "rb").read()).hexdigest() == k["sha256"]
            got = bench.measured_traffic(name, wl) if name in bench.KERNEL_SOURCES else None
            if name in bench.KERNEL_SOURCES:
                # reported exactly while the source is the one measured, else None
                assert (got == k["hbm_bytes_per_launch"]) if fresh else (got is None)
