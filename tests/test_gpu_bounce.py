"""GPU: multi-bounce light injection (ssvb_inject_bounce) against the oracle."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import parity as PY
from gbuffer_scene import crease_gbuffer, make_camera

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


def scene():
    cam = make_camera(48, 32, fov_y_deg=70, pitch_deg=-30)
    gb = crease_gbuffer(cam, D=3.0, alpha=math.radians(60))
    return gb, cam


KW = dict(slices=4, steps=8, radius=2.0, thickness=float("inf"), noise=O.NOISE_FIXED)


def close(gpu, ref, f16):
    """FP32: within a few FP32 roundings; FP16: within one FP16 rounding of the FP64 value."""
    gpu = gpu.astype(np.float64)
    if f16:
        return np.all(np.abs(gpu - ref) <= np.spacing(np.abs(ref).astype(np.float16)).astype(np.float64))
    return np.all(np.abs(gpu - ref) <= 4 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64) + 1e-30)


@pytest.mark.parametrize("fmt", ["f32-3", "f16-3", "f32-4", "f16-4", "mixed"])
def test_inject_matches_oracle(ctx, fmt):
    import torch
    gb, cam = scene()
    H, W = gb["depth"].shape
    bc, _ = PY.cams(cam)
    bp, _ = PY.params(**KW)
    t = PY.to_device(gb)
    gi = ctx.compute(t["depth"], t["normal"], t["radiance"], bc, bp)["gi"]
    rng = np.random.default_rng(3)
    ch = 4 if fmt.endswith("-4") else 3
    d_np = rng.uniform(0, 2, (H, W, ch)).astype(np.float32)
    a_np = rng.uniform(0, 1, (H, W, ch)).astype(np.float32)
    dt_d = np.float16 if fmt in ("f16-3", "f16-4") else np.float32
    dt_a = np.float16 if fmt in ("f16-3", "f16-4", "mixed") else np.float32
    d_np, a_np = d_np.astype(dt_d), a_np.astype(dt_a)
    direct = torch.from_numpy(d_np).cuda()
    albedo = torch.from_numpy(a_np).cuda()
    out_dt = torch.float16 if fmt == "mixed" else direct.dtype
    out = torch.empty((H, W, ch), dtype=out_dt, device="cuda")
    ctx.inject_bounce(direct, albedo, gi, 0.8, out=out)
    torch.cuda.synchronize()
    ref = O.inject_bounce(d_np, a_np, gi.cpu().numpy(), 0.8)
    got = out.cpu().numpy()
    assert close(got[..., :3], ref, out_dt == torch.float16), fmt
    if ch == 4:
        assert np.array_equal(got[..., 3].astype(np.float32), d_np[..., 3].astype(out.cpu().numpy().dtype).astype(np.float32))
    # in place: next is direct
    inplace = direct.clone()
    if out_dt == direct.dtype:
        ctx.inject_bounce(inplace, albedo, gi, 0.8, out=inplace)
        torch.cuda.synchronize()
        assert torch.equal(inplace, out)


def test_multi_bounce_loop(ctx):
    """Three frames of feedback on the lit crease: each frame's GI matches the oracle's
    loop within the FP32 bar."""
    import torch
    gb, cam = scene()
    H, W = gb["depth"].shape
    bc, oc = PY.cams(cam)
    bp, op = PY.params(**KW)
    t = PY.to_device(gb)
    albedo_np = np.full((H, W, 3), 0.7, np.float32)
    albedo = torch.from_numpy(albedo_np).cuda()
    light = t["radiance"].clone()
    light_ref = gb["radiance"]
    for frame in range(3):
        gi = ctx.compute(t["depth"], t["normal"], light, bc, bp)["gi"]
        ref = O.compute(gb["depth"], gb["normal"], light_ref, oc, op)
        torch.cuda.synchronize()
        err = np.abs(gi.cpu().numpy() - ref["gi"]).max()
        log(f"frame {frame}: max GI error {err:.2e}")
        assert err <= 1e-3
        light = ctx.inject_bounce(t["radiance"], albedo, gi, 0.9)
        light_ref = O.inject_bounce(gb["radiance"], albedo_np, ref["gi"], 0.9).astype(np.float32)


def test_inject_rejects(ctx):
    import torch
    from paper_2301_11376_amd import SSVBError
    d = torch.zeros((8, 8, 3), device="cuda")
    a = torch.zeros((8, 8, 3), device="cuda")
    g = torch.zeros((8, 8, 3), device="cuda")
    with pytest.raises(SSVBError) as e:
        ctx.inject_bounce(d, a, g, -0.5)
    assert e.value.status == 1
    with pytest.raises(SSVBError) as e:
        ctx.inject_bounce(d, a, g, float("nan"))
    assert e.value.status == 1
    with pytest.raises(SSVBError) as e:
        ctx.inject_bounce(d, a, g, 0.5, out=torch.zeros((8, 8, 4), device="cuda"))
    assert e.value.status == 1
