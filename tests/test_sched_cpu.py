"""CPU test of the request loop's admission logic: builds tests/sched_test.cpp with g++
against the library's host-only header (no HIP) and runs it, with AddressSanitizer and
UndefinedBehaviorSanitizer on the host build."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("sanitize", [False, True], ids=["O2", "asan-ubsan"])
def test_admission_logic(sanitize):
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sched_test")
        cmd = ["g++", "-std=c++17", "-O2", "-Wall", "-Werror",
               "-I", os.path.join(ROOT, "paper_2301_11376_amd", "csrc"),
               os.path.join(ROOT, "tests", "sched_test.cpp"), "-o", exe]
        if sanitize:
            cmd[3:3] = ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert res.returncode == 0, res.stdout + res.stderr
        assert "OK" in res.stdout
        assert "policy simulation ok" in res.stdout
