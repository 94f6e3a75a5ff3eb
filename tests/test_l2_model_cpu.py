"""CPU test of the cache model of the gather's reads (l2_model.cpp): it builds against the
library and the kernels' per-pixel header, runs on the 128x128 workload in the library's
strip order, a slice-major order and the packed normal + radiance layout, and reports
self-consistent figures: L2 misses never above L2 requests, at most 64 lines per load
instruction, the indirect term's normal and radiance reads present, with the packed
layout no more radiance requests reaching the L2 than with separate images (a sample's two
reads then share a line), and with depth in 8 x 4-texel lines the same load instructions."""
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from gbuffer_scene import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def parse(text):
    out = {}
    for kind in ("depth", "normal", "radiance"):
        m = re.search(kind + r"\s+instructions (\d+) lines/instr ([\d.]+) l2_requests/sample ([\d.]+) "
                             r"l2_misses/sample ([\d.]+)", text)
        out[kind] = tuple(float(v) for v in m.groups())
    m = re.search(r"total l2_hit ([\d.]+) l2_misses/sample ([\d.]+) l2_requests/sample ([\d.]+)", text)
    out["total"] = tuple(float(v) for v in m.groups())
    return out


def test_cache_model_runs_and_is_consistent():
    if not os.path.exists(HIPCC):
        pytest.skip("needs hipcc")
    from paper_2301_11376_amd import binding, build_lib
    if not os.path.exists(binding.LIB_PATH):
        build_lib.build()
    libdir = os.path.dirname(binding.LIB_PATH)
    gb, cam, w, sc = workload("c1_128")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "l2_model")
        res = subprocess.run([HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17",
                              "-I", os.path.join(ROOT, "include"),
                              "-I", os.path.join(ROOT, "paper_2301_11376_amd", "csrc"),
                              os.path.join(ROOT, "tests", "l2_model.cpp"), "-L", libdir, "-lssvb",
                              f"-Wl,-rpath,{libdir}", "-o", exe], capture_output=True, text=True)
        assert res.returncode == 0, res.stderr
        files = []
        for k in ("depth", "normal", "radiance"):
            f = os.path.join(d, k)
            np.ascontiguousarray(gb[k]).tofile(f)
            files.append(f)
        runs = {}
        for order, layout in (("strip", "planar"), ("slice64", "planar"), ("strip", "packed"),
                              ("strip", "planar+d8x4")):
            args = [exe, *files, "128", "128", "0", str(w["slices"]), str(w["steps"]), str(w["radius"]),
                    str(w["thickness"]), str(w["seed"]), order, "1.0", layout]
            r = subprocess.run(args, capture_output=True, text=True, timeout=300)
            assert r.returncode == 0, r.stderr
            print(r.stdout)
            runs[(order, layout)] = parse(r.stdout)
    for rep in runs.values():
        hit, miss, req = rep["total"]
        assert 0.0 <= hit <= 1.0 and miss <= req
        for kind in ("depth", "normal", "radiance"):
            instr, lines, l2req, l2miss = rep[kind]
            assert lines <= 64 and l2miss <= l2req
        assert rep["normal"][0] > 0 and rep["radiance"][0] > 0
    # the same samples in every order
    assert runs[("strip", "planar")]["depth"][0] <= runs[("slice64", "planar")]["depth"][0]
    assert runs[("strip", "packed")]["radiance"][2] <= runs[("strip", "planar")]["radiance"][2]
    # a 2D depth layout changes addresses only: the same load instructions and samples
    assert runs[("strip", "planar+d8x4")]["depth"][0] == runs[("strip", "planar")]["depth"][0]
    assert runs[("strip", "planar+d8x4")]["normal"][:2] == runs[("strip", "planar")]["normal"][:2]
