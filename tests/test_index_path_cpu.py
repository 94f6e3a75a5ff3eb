"""CPU test of the gather kernels' complete index path (index_path_cpu.cpp): the kernels'
own __host__ __device__ index functions and the library's own frame constants (fill_frame,
build_batch, fill_denoise, ssvb_validate: the library's sources compiled in), all host code
under ASan and UBSan, over
every frame shape and launch shape the GPU suite uses (autotuner tiles, lanes per pixel
1-8, strips 1-8, full and half resolution, both mask widths, pitched buffers, 16384-pixel
frames): every tile is claimed once, every computed pixel reached by each of its lanes
once, every byte read or written inside its buffer, no int32 overflow in the lattice.
The same checks run on a reconstruction of the withdrawn interleaved strip walk."""
import os
import shutil
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "index_path_cpu.cpp")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


# the strip walk's frame shapes in two halves (the batches in the second), the
# interleaved reconstruction, two fuzz seeds
RUNS = {"strip0": ("--part", "0/2"), "strip1": ("--part", "1/2"), "interleaved": ("--interleaved", "--quick"),
        "fuzz7": ("--fuzz", "2000", "7"), "fuzz2024": ("--fuzz", "2000", "2024")}


CSRC = os.path.join(ROOT, "paper_2301_11376_amd", "csrc")
# the library's sources, built into the emulator with the sanitizers on their host code
# (the device code is built too, only because the kernels' launch stubs refer to it)
LIB_SOURCES = ["ssvb_kernels.hip", "ssvb_denoise.hip", "ssvb_api.cpp", "ssvb_server.cpp", "ssvb_sequence.cpp"]


@pytest.fixture(scope="module")
def emulator():
    """Builds the emulator (its own source and the library's, compiled in parallel, the
    host code under ASan and UBSan) and starts its five runs at once (they are independent,
    single threaded and take 20-30 s each); each test waits for its own."""
    if not os.path.exists(HIPCC) or shutil.which("ld") is None:
        pytest.skip("needs hipcc")
    common = ["-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
              "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all"]
    device = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    with tempfile.TemporaryDirectory() as d:
        jobs = {os.path.join(d, "index_path.o"): ["-x", "hip", "--cuda-host-only", *common, "-c", SRC]}
        for src in LIB_SOURCES:
            extra = device if src.endswith(".hip") else []
            jobs[os.path.join(d, src + ".o")] = [*extra, *common, "-c", os.path.join(CSRC, src)]
        builds = {o: subprocess.Popen([HIPCC, *args, "-o", o], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                      text=True) for o, args in jobs.items()}
        for o, b in builds.items():
            out, _ = b.communicate(timeout=600)
            assert b.returncode == 0, out
        exe = os.path.join(d, "index_path")
        res = subprocess.run([HIPCC, "-Xarch_host", "-fsanitize=address,undefined", "--hip-link", *jobs, "-o", exe],
                             capture_output=True, text=True)
        assert res.returncode == 0, res.stdout + res.stderr
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
        procs = {k: subprocess.Popen([exe, *a], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
                 for k, a in RUNS.items()}
        try:
            yield procs
        finally:
            for p in procs.values():
                if p.poll() is None:
                    p.kill()
                p.communicate()


def run(procs, key):
    out, err = procs[key].communicate(timeout=900)
    print(out)
    assert procs[key].returncode == 0, out + err
    assert " 0 failed" in out
    return out


def test_strip_walk_index_path(emulator):
    """The library's walk, every launch shape of the autotuner on every frame up to 1080p
    (four shapes on the 4K frame); the slice-major order (items over chunks of 1, 7, 64 and
    65,536 tiles: each (tile, slice) once, each pixel's partial record once and in bounds,
    the reduction's grid); on the frames up to 400k pixels also the half-resolution fill and
    every denoiser pass on real buffers of exactly the frames' spans."""
    outs = [run(emulator, "strip0"), run(emulator, "strip1")]
    counts = [[int(v) for v in re.search(r"(\d+) frame launches, (\d+) batches, (\d+) slice-major items, "
                                         r"(\d+) upsampled and (\d+) denoised cells", o).groups()] for o in outs]
    frames, batches, items, up, dn = (a + b for a, b in zip(*counts))
    assert frames > 1000 and batches > 100 and items > 0 and up > 0 and dn > 0


def test_interleaved_walk_reconstruction_index_path(emulator):
    """The reconstructed interleaved walk (strips 0, 8, 16, ... then 1, 9, ...) with the
    strip widths 1, 2 and 4 and the lp = 1 tiles: in bounds and a bijection as well."""
    run(emulator, "interleaved")


@pytest.mark.parametrize("seed", [7, 2024])
def test_validated_inputs_keep_the_index_path_in_bounds(emulator, seed):
    """2,000 random inputs (frames from 0x0 to 16384-wide strips, cameras with any principal
    point and focal lengths from 1e-3 to 1e5, every parameter over its range, FP16 / FP32,
    3 / 4 channels, pitches up to the 4 GiB span, forced and default launch shapes), each
    field now and then outside what the library accepts: every input ssvb_validate accepts
    runs the whole per-frame emulation (tiles, lanes, every texel's 32-bit offsets exact,
    outputs in bounds), the slice-major order with a chunk drawn from the seed, and the
    lattice check; the small ones also run in random batches of
    up to 64 frames under a random context launch shape (descriptor, packed list, cursor),
    and through the half-resolution fill and every denoiser pass on real buffers of exactly
    their spans (the sanitizer reports any access outside them)."""
    out = run(emulator, f"fuzz{seed}")
    m = re.search(r"fuzz: (\d+) inputs, (\d+) accepted \((\d+) emulated\), (\d+) rejected, (\d+) batches", out)
    n, acc, emu, rej, bat = (int(v) for v in m.groups())
    assert acc + rej == n and acc >= 0.4 * n and emu >= 0.9 * acc and bat >= 10
    m = re.search(r"(\d+) upsampled and (\d+) denoised cells", out)
    assert int(m.group(1)) > 0 and int(m.group(2)) > 0
