"""CPU tests of the gather kernels' per-pixel code, built for the host (host_gather.cpp).

csrc/ssvb_pixel.h holds everything a kernel thread computes for its pixel; its functions
are __host__ __device__, so the same source runs here on the CPU, with the frame constants
and tables the library derives.  These tests hold that code to the FP64 oracle with the
GPU parity tests' bar (masks equal, every mismatch traced to a near-tie endpoint, AO / GI /
ambient within 1e-3) on the same cases, and check that the batch kernel's run-time
dispatch instance gives the single-frame instance's results bit for bit.  The device
differs only in its primitives (the hardware reciprocal, FP contraction), so this shows
the kernel source right, not the GPU's rounding."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O
import parity as PY
from gbuffer_scene import make_camera, make_scene, render_gbuffer, workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def host():
    if not os.path.exists(HIPCC):
        pytest.skip("needs hipcc")
    from paper_2301_11376_amd import binding, build_lib
    if not os.path.exists(binding.LIB_PATH):
        build_lib.build()
    libdir = os.path.dirname(binding.LIB_PATH)
    with tempfile.TemporaryDirectory() as d:
        so = os.path.join(d, "host_gather.so")
        cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", "-fPIC", "-shared",
               "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2301_11376_amd", "csrc"),
               os.path.join(ROOT, "tests", "host_gather.cpp"), "-L", libdir, "-lssvb", f"-Wl,-rpath,{libdir}",
               "-o", so]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stdout + res.stderr
        L = ctypes.CDLL(so)
        B = binding
        L.host_gather.restype = ctypes.c_int32
        L.host_gather.argtypes = [ctypes.POINTER(B.ssvb_image)] * 3 + [
            ctypes.POINTER(B.ssvb_camera), ctypes.POINTER(B.ssvb_params), ctypes.POINTER(B.ssvb_outputs),
            ctypes.c_int32]
        L.host_gather_slices.restype = ctypes.c_int32
        L.host_gather_slices.argtypes = L.host_gather.argtypes
        f32p = ctypes.POINTER(ctypes.c_float)
        L.host_endpoints.restype = ctypes.c_int32
        L.host_endpoints.argtypes = L.host_gather.argtypes[:6] + [f32p]
        L.host_atan2.restype = None
        L.host_atan2.argtypes = [f32p, f32p, f32p, ctypes.c_int64]
        u32p, i32p = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_int32)
        L.host_mask_range.restype = ctypes.c_int32
        L.host_mask_range.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, u32p]
        L.host_mask_cover.restype = ctypes.c_int32
        L.host_mask_cover.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p, u32p, i32p]
        yield L


def _image(a, pad=0):
    """ssvb_image of a host array (optionally in rows padded by `pad` elements)."""
    from paper_2301_11376_amd import binding as B
    a = np.ascontiguousarray(a)
    if pad:
        H, W = a.shape[:2]
        buf = np.zeros((H, W + pad) + a.shape[2:], a.dtype)
        buf[:, :W] = a
        a = buf[:, :W]
    ch = 1 if a.ndim == 2 else a.shape[2]
    dt = B.F16 if a.dtype == np.float16 else B.F32
    return B.ssvb_image(a.ctypes.data, a.strides[0], dt, ch), a


def run_host(L, gb, cam, masks=True, generic=False, pad=0, chunk=None, **kw):
    """The host build on a frame: the single-frame (or with ``generic`` the batch) instance,
    or with ``chunk`` the slice-major order over chunks of that many tiles."""
    from paper_2301_11376_amd import binding as B
    H, W = gb["depth"].shape
    d, da = _image(gb["depth"], pad)
    n, na = _image(gb["normal"], pad)
    r, ra = _image(gb["radiance"], pad)
    bc, _ = PY.cams(cam)
    bp, _ = PY.params(**kw)
    words = kw["slices"] * kw.get("sectors", 32) // 32
    out = {"ao": np.full((H, W), np.nan, np.float32), "gi": np.full((H, W, 3), np.nan, np.float32),
           "ambient": np.full((H, W, 3), np.nan, np.float32)}
    if masks:
        out["masks"] = np.full((H, W, words), 0xDEADBEEF, np.uint32)
    o = B.ssvb_outputs(out["ao"].ctypes.data, out["gi"].ctypes.data, out["ambient"].ctypes.data,
                       out["masks"].ctypes.data if masks else None, 0, 0, 0, 0)
    c, p = bc.to_c(), bp.to_c()
    fn, last = (L.host_gather, int(generic)) if chunk is None else (L.host_gather_slices, int(chunk))
    st = fn(ctypes.byref(d), ctypes.byref(n), ctypes.byref(r), ctypes.byref(c), ctypes.byref(p), ctypes.byref(o),
            last)
    assert st == 0, st
    return out


def host_case(L, gb, cam, report=None, pixels=None, bar=None, **kw):
    """The host build against the oracle, and the batch instance against the single-frame
    instance (bit for bit).  ``bar`` overrides compare()'s agreement / max_bad."""
    g = run_host(L, gb, cam, **kw)
    gen = run_host(L, gb, cam, generic=True, **kw)
    for k in g:
        assert np.array_equal(g[k].view(np.uint32), gen[k].view(np.uint32)), ("generic instance", k)
    _, oc = PY.cams(cam)
    _, op = PY.params(**kw)
    ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, pixels=pixels, return_masks=True)
    PY.compare(g, ref, gb, oc, op, pixels=pixels, report=report, **(bar or {}))
    return g


def test_host_c1_full_frame(host):
    gb, cam, w, sc = workload("c1_128")
    rep = {}
    host_case(host, gb, cam, report=rep, slices=2, steps=8, radius=2.0, thickness=0.5, noise=O.NOISE_HASH, seed=1,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    print(rep)
    assert rep["mask_agreement"] == 1.0


@pytest.mark.parametrize("name", sorted(PY.VARIANTS))
def test_host_variants(host, name):
    gb, cam, sc = PY.tiny()
    host_case(host, gb, cam, ambient_sh=tuple(sc.ambient_sh.reshape(-1)), **PY.VARIANTS[name])


@pytest.mark.parametrize("fp16,channels", [(False, 4), (True, 3), (True, 4)])
def test_host_formats(host, fp16, channels):
    gb, cam, sc = PY.tiny(fp16=fp16, channels=channels)
    host_case(host, gb, cam, slices=3, steps=6, radius=1.3, thickness=0.3, noise=O.NOISE_R2, seed=2,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))


@pytest.mark.parametrize("shape", [(67, 45), (1, 1), (1, 37), (37, 1), (129, 3)])
def test_host_ragged_shapes(host, shape):
    W, H = shape
    sc = make_scene(21, 40, 20)
    cam = make_camera(W, H, fov_y_deg=60, pitch_deg=-25)
    gb = render_gbuffer(sc, cam, cache=False)
    host_case(host, gb, cam, slices=3, steps=5, radius=1.0, noise=O.NOISE_HASH, seed=3,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))


def test_host_pitched_buffers(host):
    """Rows padded in every input: the same results as dense rows, bit for bit."""
    gb, cam, sc = PY.tiny()
    kw = dict(slices=3, steps=6, radius=1.3, thickness=0.3, noise=O.NOISE_R2, seed=2,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    a = run_host(host, gb, cam, **kw)
    b = run_host(host, gb, cam, pad=13, **kw)
    for k in a:
        assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), k


@pytest.mark.parametrize("sectors", [32, 128])
def test_host_quadratic_probe(host, sectors):
    gb, cam, sc = PY.tiny()
    sh = np.random.default_rng(31).uniform(-1.0, 1.0, (9, 3))
    sh[0] = 1.5
    host_case(host, gb, cam, slices=4, steps=6, radius=1.5, thickness=0.4, noise=O.NOISE_R2, seed=31,
              ambient_samples=8, sectors=sectors, ambient_sh=tuple(sh.reshape(-1)))


@pytest.mark.parametrize("fp16", [False, True])
def test_host_sectors128_c1(host, fp16):
    gb, cam, w, sc = workload("c1_128")
    if fp16:
        gb = dict(gb, normal=gb["normal"].astype(np.float16), radiance=gb["radiance"].astype(np.float16))
    rep = {}
    host_case(host, gb, cam, report=rep, slices=2, steps=8, radius=2.0, thickness=0.5, noise=O.NOISE_HASH, seed=1,
              sectors=128, ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    print(rep)


def test_host_background(host):
    """A frame of sky only: AO 1, GI 0, ambient 0, masks 0 everywhere."""
    cam = make_camera(19, 11, fov_y_deg=60, pitch_deg=0)
    gb = {"depth": np.zeros((11, 19), np.float32), "normal": np.zeros((11, 19, 3), np.float32),
          "radiance": np.ones((11, 19, 3), np.float32)}
    g = run_host(host, gb, cam, slices=3, steps=4, radius=1.0, noise=O.NOISE_HASH, seed=1)
    assert np.all(g["ao"] == 1) and np.all(g["gi"] == 0) and np.all(g["ambient"] == 0) and np.all(g["masks"] == 0)


@pytest.mark.parametrize("name", sorted(PY.HALF_CASES))
@pytest.mark.parametrize("size", [(64, 48), (67, 45)])
def test_host_half_resolution(host, name, size):
    """Half resolution: the gathered (even, even) pixels are the full-resolution run's bit
    for bit; the upsampler matches the oracle's FP64 one on the same gathered values within
    1e-5; the whole image matches the oracle's half-resolution result within 1e-3."""
    gb, cam, sc = PY.tiny(*size)
    kw = dict(PY.HALF_CASES[name], ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    full = host_case(host, gb, cam, **kw)
    half = run_host(host, gb, cam, masks=False, resolution=2, **kw)
    for k in ("ao", "gi", "ambient"):
        assert np.array_equal(half[k][0::2, 0::2].view(np.uint32), full[k][0::2, 0::2].view(np.uint32)), k
    a, g, m = O.bilateral_upsample(gb["depth"], half["ao"].astype(np.float64), half["gi"].astype(np.float64),
                                   half["ambient"].astype(np.float64))
    assert max(np.abs(half["ao"] - a).max(), np.abs(half["gi"] - g).max(), np.abs(half["ambient"] - m).max()) <= 1e-5
    _, oc = PY.cams(cam)
    _, op = PY.params(resolution=2, **kw)
    ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op)
    for k in ("ao", "gi", "ambient"):
        assert np.abs(half[k] - ref[k]).max() <= 1e-3, k


def test_host_c2_1080p_sampled(host):
    """The whole 1920x1080 frame through the host build; the oracle checks a seeded sample
    of 3,000 pixels plus the corners and the last row and column."""
    gb, cam, w, sc = workload("c2_1080p")
    H, W = gb["depth"].shape
    rep = {}
    kw = dict(slices=4, steps=16, radius=3.0, thickness=0.5, noise=O.NOISE_R2, seed=2,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    g = run_host(host, gb, cam, **kw)
    pix = PY.sample_pixels(H, W, 3000, 2)
    _, oc = PY.cams(cam)
    _, op = PY.params(**kw)
    ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, pixels=pix, return_masks=True)
    PY.compare(g, ref, gb, oc, op, pixels=pix, report=rep)
    print(rep)


@pytest.mark.parametrize("case", range(48))
def test_host_random_cases(host, case):
    """48 seeded random frames (1x1 to 40x30, scenes with sky, FP16 / FP32, 3 / 4 channels)
    and parameter sets (criterion, noise, thickness 0 / finite / inf, slope, radius caps,
    sub-pixel steps, quadratic steps, 32 / 128 sectors, N_a): the host build against the
    oracle, every mismatch traced to near-tie endpoints and outputs within 1e-3; one in four
    also at half resolution (gathered pixels those of the traced full-resolution run bit for
    bit, the upsampler the oracle's FP64 one within 1e-5), and another one in four in the
    slice-major order too.  The 99.9 % mask agreement floor
    is not applied: these
    scenes are axis-aligned planes, so under PSEUDOCODE whole rows of samples lie exactly
    in a pixel's tangent plane, on a hemisphere edge, where the ceiling of a zero width
    is decided by the last bit of either side's FP64 rounding."""
    rng = np.random.default_rng(1000 + case)
    gb, cam, kw = PY.random_case(rng)
    H, W = gb["depth"].shape
    full = host_case(host, gb, cam, bar=dict(agreement=0.0, max_bad=H * W), **kw)
    if case % 4 == 1:
        # the slice-major order over chunks of 1-7 tiles: the same masks and AO, GI and
        # ambient within FP32 rounding of the other grouping
        so = run_host(host, gb, cam, chunk=1 + case % 7, **kw)
        assert np.array_equal(so["masks"], full["masks"])
        assert np.array_equal(so["ao"].view(np.uint32), full["ao"].view(np.uint32))
        for k in ("gi", "ambient"):
            np.testing.assert_allclose(so[k], full[k], rtol=5e-6, atol=1e-6, err_msg=k)
    if case % 4 == 3:
        half = run_host(host, gb, cam, masks=False, resolution=2, **kw)
        for k in ("ao", "gi", "ambient"):
            assert np.array_equal(half[k][0::2, 0::2].view(np.uint32), full[k][0::2, 0::2].view(np.uint32)), k
        a, g, m = O.bilateral_upsample(gb["depth"], half["ao"].astype(np.float64),
                                       half["gi"].astype(np.float64), half["ambient"].astype(np.float64))
        assert max(np.abs(half["ao"] - a).max(), np.abs(half["gi"] - g).max(),
                   np.abs(half["ambient"] - m).max()) <= 1e-5


SLICE_CASES = {
    "hash_t04": (PY.VARIANTS["hash_t04"], (64, 48)),
    "r2_tinf": (PY.VARIANTS["r2_tinf"], (67, 45)),
    "pseudo_128": (dict(slices=3, steps=6, radius=1.3, thickness=0.3, noise=O.NOISE_R2, seed=2, sectors=128,
                        hit_criterion=1), (37, 29)),
    "quad_8dirs": (dict(slices=8, steps=5, radius=1.5, thickness=0.4, noise=O.NOISE_HASH, seed=4,
                        step_distribution=1, ambient_samples=8), (40, 9)),
    "half_res": (dict(PY.HALF_CASES["uniform"], resolution=2), (67, 45)),
    "one_pixel": (dict(slices=2, steps=3, radius=1.0, noise=O.NOISE_HASH, seed=5), (1, 1)),
}


def slice_order_case(L, name, chunks=(1, 3, 64)):
    """The slice-major order against the pixel-major run of the same instance (the batch
    kernel's): masks and AO bit for bit (each slice's mask is the same march, and the AO adds
    the same per-slice terms in the same order), GI and ambient within FP32 rounding of a
    different summation order; every chunk size gives the same outputs bit for bit (the
    partial sums do not depend on the order items run in).  The partial buffer starts as
    NaN, so a (pixel, slice) no item covered would show."""
    kw, (W, H) = SLICE_CASES[name]
    gb, cam, sc = PY.tiny(W, H)
    kw = dict(kw, ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    half = kw.get("resolution", 1) == 2
    ref = run_host(L, gb, cam, masks=not half, generic=True, **kw)
    runs = [run_host(L, gb, cam, masks=not half, chunk=c, **kw) for c in chunks]
    for got in runs[1:]:
        for k in got:
            assert np.array_equal(got[k].view(np.uint32), runs[0][k].view(np.uint32)), ("chunk", k)
    got = runs[0]
    for k in ("ao", "gi", "ambient"):
        assert np.all(np.isfinite(got[k])), k
    if not half:
        assert np.array_equal(got["masks"], ref["masks"])
        assert np.array_equal(got["ao"].view(np.uint32), ref["ao"].view(np.uint32))
    else:
        assert np.abs(got["ao"] - ref["ao"]).max() <= 1e-6
    for k in ("gi", "ambient"):
        np.testing.assert_allclose(got[k], ref[k], rtol=2e-6, atol=1e-7, err_msg=k)
    return got, gb, cam, kw


@pytest.mark.parametrize("name", sorted(SLICE_CASES))
def test_host_slice_order(host, name):
    """Slice-major order (ssvb_set_slice_order) against the pixel-major run, and against
    the oracle with the parity bar (full resolution) or within 1e-3 (half)."""
    got, gb, cam, kw = slice_order_case(host, name)
    _, oc = PY.cams(cam)
    _, op = PY.params(**kw)
    if kw.get("resolution", 1) == 2:
        ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op)
        for k in ("ao", "gi", "ambient"):
            assert np.abs(got[k] - ref[k]).max() <= 1e-3, k
    else:
        ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, return_masks=True)
        H, W = gb["depth"].shape
        PY.compare(got, ref, gb, oc, op, agreement=0.0 if H * W < 100 else PY.MASK_AGREEMENT)


def test_host_slice_order_1080p_band(host):
    """A 270-row band across the middle of the 1920x1080 workload frame (its own camera
    cropped, 2,040 tiles: four chunks of 64 tiles per die's run, the last one shorter) in
    both orders: masks and AO equal bit for bit, GI and ambient within the GPU test's bar
    for the two orders (5e-6 relative, 1e-6 absolute)."""
    import dataclasses
    gb, cam, w, sc = workload("c2_1080p")
    r0, r1 = 405, 675
    gb = {k: np.ascontiguousarray(v[r0:r1]) for k, v in gb.items()}
    cam = dataclasses.replace(cam, height=r1 - r0, cy=float(np.float32(cam.cy - r0)))
    kw = dict(slices=4, steps=16, radius=3.0, thickness=0.5, noise=O.NOISE_R2, seed=2,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    a = run_host(host, gb, cam, generic=True, **kw)
    b = run_host(host, gb, cam, chunk=64, **kw)
    assert np.array_equal(a["masks"], b["masks"])
    assert np.array_equal(a["ao"].view(np.uint32), b["ao"].view(np.uint32))
    for k in ("gi", "ambient"):
        d = np.abs(a[k].astype(np.float64) - b[k])
        print(f"{k}: max |difference| {d.max():.3g}, on {np.mean(d > 0):.3f} of the values")
        np.testing.assert_allclose(b[k], a[k], rtol=5e-6, atol=1e-6, err_msg=k)


def test_host_slice_order_background(host):
    """A frame of sky in slice-major order: the reduction writes AO 1, GI 0, ambient 0 and
    empty masks (no item writes a background pixel's partial sums)."""
    cam = make_camera(19, 11, fov_y_deg=60, pitch_deg=0)
    gb = {"depth": np.zeros((11, 19), np.float32), "normal": np.zeros((11, 19, 3), np.float32),
          "radiance": np.ones((11, 19, 3), np.float32)}
    g = run_host(host, gb, cam, chunk=2, slices=3, steps=4, radius=1.0, noise=O.NOISE_HASH, seed=1)
    assert np.all(g["ao"] == 1) and np.all(g["gi"] == 0) and np.all(g["ambient"] == 0) and np.all(g["masks"] == 0)


def test_atan2_error_bound(host):
    """The kernels' FP32 arc tangent (octant reduction to r = min / max, odd degree-13
    minimax polynomial) against FP64 atan2 of the same FP32 arguments, over a dense sweep of
    r in [0, 1] in every octant of the upper half plane, at random magnitudes, and at the
    special arguments (y = 0, x = 0, y = |x|, x = -inf): |error| < 3.3e-7 rad for the
    polynomial alone (r exact, first octant) and < 5.5e-7 rad everywhere (the rounding of r,
    and pi/2 - a and pi - a rounded to FP32, whose ulp near pi is 2.4e-7).  The host's
    exact division stands in for the device's reciprocal (about 1 ulp of r more)."""
    rng = np.random.default_rng(5)
    r = np.linspace(0.0, 1.0, 400001)
    ys, xs = [], []
    for a, b in ((r, 1.0), (1.0, r), (r, -1.0), (1.0, -r)):
        scale = 10.0 ** rng.uniform(-18, 18, r.size)
        ys.append(np.broadcast_to(a, r.shape) * scale)
        xs.append(np.broadcast_to(b, r.shape) * scale)
    ys.append(np.array([0.0, 0.0, 1.0, 1.0, 1.0, 0.0, 3.0, 1e-30]))
    xs.append(np.array([1.0, -1.0, 0.0, 1.0, -1.0, -np.inf, -np.inf, 1e30]))
    y = np.ascontiguousarray(np.concatenate(ys), np.float32)
    x = np.ascontiguousarray(np.concatenate(xs), np.float32)
    out = np.empty_like(y)
    f32p = ctypes.POINTER(ctypes.c_float)
    host.host_atan2(y.ctypes.data_as(f32p), x.ctypes.data_as(f32p), out.ctypes.data_as(f32p), y.size)
    err = np.abs(out.astype(np.float64) - np.arctan2(y.astype(np.float64), x.astype(np.float64)))
    assert np.all(np.isfinite(out)) and err.max() < 5.5e-7, err.max()
    # the polynomial alone: r exact (x = 1), first octant
    r32 = np.ascontiguousarray(r, np.float32)
    one = np.ones_like(r32)
    poly = np.empty_like(r32)
    host.host_atan2(r32.ctypes.data_as(f32p), one.ctypes.data_as(f32p), poly.ctypes.data_as(f32p), r32.size)
    perr = np.abs(poly.astype(np.float64) - np.arctan(r32.astype(np.float64))).max()
    assert perr < 3.3e-7, perr


ENDPOINT_CASES = {
    "hash_t04": dict(slices=4, steps=12, radius=1.5, thickness=0.4, noise=O.NOISE_HASH, seed=3),
    "r2_tinf": dict(slices=2, steps=8, radius=3.0, thickness=float("inf"), noise=O.NOISE_R2, seed=4),
    "pseudocode": dict(slices=2, steps=8, radius=1.0, thickness=0.2, noise=O.NOISE_HASH, seed=5, hit_criterion=1),
    "slope_quad": dict(slices=3, steps=10, radius=2.0, thickness=0.1, thickness_slope=0.05, noise=O.NOISE_R2,
                       seed=6, step_distribution=1),
}


@pytest.mark.parametrize("sectors", [32, 128])
@pytest.mark.parametrize("name", sorted(ENDPOINT_CASES))
def test_host_endpoint_error_within_guard(host, name, sectors):
    """Every sample's FP32 sector arguments (the kernels' own code) against the oracle's
    FP64 ones: the same samples skipped, and every argument within 2^-16 sectors (in units
    of the mask's sectors), half the band in which the kernels re-decide in FP64 (2^-15
    sectors, scaled with N_b), so the exact decision covers every rounding the FP32 path
    can get wrong.  The GPU test of the same hook holds the device to the same bar."""
    from paper_2301_11376_amd import binding as B
    gb, cam, sc = PY.tiny()
    kw = dict(ENDPOINT_CASES[name], sectors=sectors)
    H, W = gb["depth"].shape
    d, da = _image(gb["depth"])
    n, na = _image(gb["normal"])
    r, ra = _image(gb["radiance"])
    bc, oc = PY.cams(cam)
    bp, op = PY.params(**kw)
    ao, gi, am = np.zeros((H, W), np.float32), np.zeros((H, W, 3), np.float32), np.zeros((H, W, 3), np.float32)
    o = B.ssvb_outputs(ao.ctypes.data, gi.ctypes.data, am.ctypes.data, None, 0, 0, 0, 0)
    ep = np.full((H, W, kw["slices"], 2, kw["steps"], 2), np.nan, np.float32)
    c, p = bc.to_c(), bp.to_c()
    st = host.host_endpoints(ctypes.byref(d), ctypes.byref(n), ctypes.byref(r), ctypes.byref(c), ctypes.byref(p),
                             ctypes.byref(o), ep.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    assert st == 0, st
    ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, return_endpoints=True)["endpoints"]
    assert np.array_equal(np.isnan(ep), np.isnan(ref))
    ok = np.isfinite(ref)
    err = np.abs(ep[ok] - ref[ok]).max()
    print(f"{name}, {sectors} sectors: max endpoint error {err:.3e} sectors over {ok.sum()} values")
    assert ok.sum() > 1000 and err < 2.0 ** -16 * (sectors // 32), err


def _words(bits, nb):
    """A Python int of sector bits as N_b / 32 little-endian 32-bit words."""
    return [(bits >> (32 * i)) & 0xFFFFFFFF for i in range(nb // 32)]


@pytest.mark.parametrize("nb", [32, 64, 128])
def test_mask_range_exhaustive(host, nb):
    """Every sector range [a, b), 0 <= a <= b <= N_b, against the bits it names."""
    out = (ctypes.c_uint32 * (nb // 32))()
    for a in range(nb + 1):
        for b in range(a, nb + 1):
            assert host.host_mask_range(nb, a, b, out) == 0
            assert list(out) == _words(((1 << b) - 1) ^ ((1 << a) - 1), nb), (a, b)


@pytest.mark.parametrize("nb", [32, 64, 128])
def test_mask_cover_sequences(host, nb):
    """Seeded sequences of ranges ORed in order: each step's newly covered count is the
    number of its sectors not in the union so far, and the final words and count are the
    union's (short, long, empty and full ranges mixed)."""
    rng = np.random.default_rng(nb)
    for trial in range(400):
        n = int(rng.integers(1, 40))
        a = rng.integers(0, nb + 1, n)
        w = np.where(rng.random(n) < 0.7, rng.integers(0, 6, n), rng.integers(0, nb + 1, n))
        b = np.minimum(a + w, nb)
        a32, b32 = a.astype(np.int32), b.astype(np.int32)
        fresh = np.zeros(n, np.int32)
        words = (ctypes.c_uint32 * (nb // 32))()
        count = ctypes.c_int32()
        i32p = ctypes.POINTER(ctypes.c_int32)
        assert host.host_mask_cover(nb, a32.ctypes.data_as(i32p), b32.ctypes.data_as(i32p), n,
                                    fresh.ctypes.data_as(i32p), words, ctypes.byref(count)) == 0
        union = 0
        for j in range(n):
            r = ((1 << int(b[j])) - 1) ^ ((1 << int(a[j])) - 1)
            assert fresh[j] == bin(r & ~union).count("1"), (trial, j)
            union |= r
        assert list(words) == _words(union, nb) and count.value == bin(union).count("1")
