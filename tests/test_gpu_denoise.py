"""GPU: edge-aware a-trous denoising (ssvb_denoise) against the oracle.

Tolerance: the filter's outputs are convex combinations of its inputs, so FP32 errors
enter through the weights.  The view-space positions carry a relative FP32 rounding of a
few ulp, so the plane distance d = n_p . (P_q - P_p) / (sigma z_p) is off by up to about
4e-7 |r| / sigma ~ 1.2e-5 (|r| <= 1.5, sigma = 0.05), which moves exp(-d^2) by 2 d
times that, relative; over the taps an output moves by at most about 1e-4 of the
spread of its inputs.  The bar is 1e-4 x max(1, max |input|), absolute.
"""
import sys

import numpy as np
import pytest

import oracle as O
import parity as PY
from gbuffer_scene import make_camera, make_scene, render_gbuffer

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2301_11376_amd import Context
    c = Context(0)
    yield c
    c.close()


def scene(W, H, seed, fp16=False, ch=3, background=False):
    sc = make_scene(seed, 30, 15)
    pitch = 0.0 if background else -35.0
    cam = make_camera(W, H, fov_y_deg=70, pitch_deg=pitch)
    dt = np.float16 if fp16 else np.float32
    gb = render_gbuffer(sc, cam, normal_dtype=dt, radiance_dtype=dt, channels=ch, cache=False)
    return gb, cam


def signal(H, W, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return {"ao": rng.uniform(0, 1, (H, W)).astype(np.float32),
            "gi": (scale * rng.uniform(0, 1, (H, W, 3))).astype(np.float32),
            "ambient": (scale * rng.uniform(0, 1, (H, W, 3))).astype(np.float32)}


def run(ctx, gb, cam, sig, pitched=False, **kw):
    import torch
    H, W = gb["depth"].shape
    t = PY.to_device(gb)
    bc, _ = PY.cams(cam)
    src = {k: torch.from_numpy(v).cuda() for k, v in sig.items()}
    if pitched:
        # row pitch wider than the row: views into larger buffers
        def wide(shape):
            full = torch.full((shape[0], shape[1] + 7) + tuple(shape[2:]), -5.0, device="cuda")
            return full[:, :shape[1]]
        src = {k: wide(v.shape).copy_(v) for k, v in src.items()}
        out = {k: wide(v.shape) for k, v in src.items()}
        tmp = {k: wide(v.shape) for k, v in src.items()}
        got = ctx.denoise(t["depth"], t["normal"], bc, src, out=out, tmp=tmp, **kw)
    else:
        got = ctx.denoise(t["depth"], t["normal"], bc, src, **kw)
    torch.cuda.synchronize()
    after = {k: v.cpu().numpy() for k, v in src.items()}
    for k in sig:
        assert np.array_equal(after[k], sig[k]), "input modified"
    return {k: v.cpu().numpy() for k, v in got.items()}


def oracle(gb, cam, sig, **kw):
    _, oc = PY.cams(cam)
    a, g, m = O.denoise(gb["depth"], gb["normal"], oc, sig["ao"], sig["gi"], sig["ambient"], **kw)
    return {"ao": a, "gi": g, "ambient": m}


def check(got, ref, sig, what):
    bar = 1e-4 * max(1.0, max(float(np.abs(v).max()) for v in sig.values()))
    err = max(float(np.abs(got[k].astype(np.float64) - ref[k]).max()) for k in ref)
    log(f"  {what}: max |GPU - oracle| = {err:.2e} (bar {bar:.1e})")
    assert err <= bar, what


CASES = {
    "default": dict(),
    "one pass": dict(passes=1),
    "three passes": dict(passes=3),
    "no normal term": dict(normal_power=0),
    "odd power": dict(normal_power=3, plane_sigma=0.02),
    "no plane term": dict(plane_sigma=float("inf"), normal_power=128),
    "half resolution": dict(resolution=2),
    "half resolution, three passes": dict(resolution=2, passes=3),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("size", [(67, 45), (40, 33)])
def test_denoise_matches_oracle(ctx, name, size):
    W, H = size
    gb, cam = scene(W, H, 3)
    sig = signal(H, W, 5)
    log(f"denoise {name} {W}x{H}")
    kw = CASES[name]
    check(run(ctx, gb, cam, sig, **kw), oracle(gb, cam, sig, **kw), sig, name)


@pytest.mark.parametrize("fmt", ["f16-3", "f32-4", "f16-4"])
def test_denoise_formats(ctx, fmt):
    gb, cam = scene(53, 38, 4, fp16=fmt.startswith("f16"), ch=int(fmt[-1]))
    sig = signal(38, 53, 6, scale=3.0)
    log(f"denoise normals {fmt}")
    check(run(ctx, gb, cam, sig), oracle(gb, cam, sig), sig, fmt)


def test_denoise_pitched_and_background(ctx):
    gb, cam = scene(61, 40, 7, background=True)
    fg = np.isfinite(gb["depth"]) & (gb["depth"] > 0)
    assert (~fg).sum() > 100 and fg.sum() > 100
    sig = signal(40, 61, 8)
    for kw in (dict(), dict(passes=3), dict(resolution=2)):
        got = run(ctx, gb, cam, sig, pitched=True, **kw)
        check(got, oracle(gb, cam, sig, **kw), sig, f"pitched, background {kw}")
        if kw.get("resolution", 1) == 1:
            for k in sig:
                assert np.array_equal(got[k][~fg], sig[k][~fg]), k   # background keeps its input


@pytest.mark.parametrize("size", [(1, 1), (1, 37), (37, 1), (17, 16), (16, 17), (129, 3)])
def test_denoise_ragged(ctx, size):
    W, H = size
    gb, cam = scene(W, H, 9)
    sig = signal(H, W, 10)
    for kw in (dict(passes=3), dict(resolution=2)):
        check(run(ctx, gb, cam, sig, **kw), oracle(gb, cam, sig, **kw), sig, f"{W}x{H} {kw}")


def test_denoise_after_gather(ctx):
    """The chain the paper times: the gather, then the denoiser, on the same frame; the
    GPU chain against the oracle chain within the gather's own bar (1e-3)."""
    gb, cam = scene(64, 48, 11)
    bc, oc = PY.cams(cam)
    kw = dict(slices=3, steps=6, radius=1.5, thickness=0.4, noise=O.NOISE_HASH, seed=2)
    bp, op = PY.params(**kw)
    t = PY.to_device(gb)
    g = ctx.compute(t["depth"], t["normal"], t["radiance"], bc, bp)
    dn = ctx.denoise(t["depth"], t["normal"], bc, g)
    ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op)
    a, gi, m = O.denoise(gb["depth"], gb["normal"], oc, ref["ao"], ref["gi"], ref["ambient"])
    import torch
    torch.cuda.synchronize()
    for k, r in (("ao", a), ("gi", gi), ("ambient", m)):
        err = float(np.abs(dn[k].cpu().numpy() - r).max())
        log(f"  chain {k}: {err:.2e}")
        assert err <= 1e-3, k


def test_denoise_1080p(ctx):
    """The 1080p workload's own G-buffer, every pixel (the oracle takes a few seconds)."""
    from gbuffer_scene import workload
    gb, cam, w, _ = workload("c2_1080p")
    H, W = gb["depth"].shape
    sig = signal(H, W, 12)
    log("denoise 1080p")
    check(run(ctx, gb, cam, sig), oracle(gb, cam, sig), sig, "1080p")


def test_denoise_rejects(ctx):
    import torch
    from paper_2301_11376_amd import SSVBError
    gb, cam = scene(24, 16, 13)
    t = PY.to_device(gb)
    bc, _ = PY.cams(cam)
    src = {k: torch.from_numpy(v).cuda() for k, v in signal(16, 24, 14).items()}
    for bad in (dict(passes=0), dict(passes=4), dict(normal_power=-1), dict(normal_power=129),
                dict(plane_sigma=0.0), dict(plane_sigma=float("nan")), dict(resolution=3)):
        with pytest.raises(SSVBError) as e:
            ctx.denoise(t["depth"], t["normal"], bc, src, **bad)
        assert e.value.status == 1, bad
    with pytest.raises(SSVBError):      # out aliases in
        ctx.denoise(t["depth"], t["normal"], bc, src, out=src)
    other = {k: torch.empty_like(v) for k, v in src.items()}
    with pytest.raises(SSVBError):      # tmp aliases out
        ctx.denoise(t["depth"], t["normal"], bc, src, out=other, tmp=other)
    ctx.denoise(t["depth"], t["normal"], bc, src, passes=1, out=other)   # one pass needs no tmp
    torch.cuda.synchronize()


def test_denoise_takes_compute_output_with_masks(ctx):
    """The dict ssvb_compute's binding returns (slice masks included) can be denoised as
    it is; the masks play no part."""
    import torch
    gb, cam = scene(40, 30, 15)
    bc, _ = PY.cams(cam)
    bp, _ = PY.params(slices=2, steps=6, radius=1.5, thickness=0.4, noise=O.NOISE_HASH, seed=4)
    t = PY.to_device(gb)
    with_masks = ctx.compute(t["depth"], t["normal"], t["radiance"], bc, bp, masks=True)
    plain_out = {k: v.clone() for k, v in with_masks.items() if k != "masks"}
    a = ctx.denoise(t["depth"], t["normal"], bc, with_masks)
    b = ctx.denoise(t["depth"], t["normal"], bc, plain_out)
    torch.cuda.synchronize()
    for k in ("ao", "gi", "ambient"):
        assert torch.equal(a[k], b[k]), k
