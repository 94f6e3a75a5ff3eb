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


def test_a_failing_leg_is_recorded_not_fatal(capsys):
    """A leg after the headline that raises is recorded as {"error": ...} in its field and
    the run goes on; a leg that succeeds stores its result and prints its progress line."""
    sys.path.insert(0, ROOT)
    import bench

    def boom():
        raise RuntimeError("planted")

    res = {}
    assert bench.run_leg(res, "bad", boom) is None
    assert res["bad"] == {"error": "RuntimeError: planted"}
    assert bench.run_leg(res, "good", lambda a, b=0: {"ms": a + b}, 1.5, b=0.5,
                         say=lambda r: f"good: {r['ms']} ms") == {"ms": 2.0}
    assert res["good"] == {"ms": 2.0}
    err = capsys.readouterr().err
    assert "planted" in err and "good: 2.0 ms" in err
