"""bench.py's contract on the CPU: one GPU only, and the committed traffic records."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_traffic_records_are_well_formed():
    sys.path.insert(0, ROOT)
    import bench
    for name in ("c2_1080p", "c3_4k_fp16"):
        with open(os.path.join(ROOT, "profiles", f"gather_frame_{name}_traffic.json")) as fh:
            rec = json.load(fh)
        assert rec["workload"] == name
        assert len(rec["device_source_sha256"]) == 64 and len(rec["launch_shape"]) == 4
        total = rec["fetch_kib_per_dispatch"] * 1024 * rec["fetch_factor"] + rec["write_kib_per_dispatch"] * 1024
        assert abs(total - rec["traffic_bytes_per_launch"]) < 1.0
        # reported only for the shape and the device sources the counters were taken with
        assert bench.measured_traffic(name, (1, 1, 1, 1)) is None
