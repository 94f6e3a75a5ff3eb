"""GPU: frame sequences (ssvb_sequence_*): multi-bounce feedback through the sequence's own
light buffer and the noise seed advanced per frame, against the oracle's sequence and
against the same steps composed from ssvb_inject_bounce and ssvb_compute."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import parity as PY
from gbuffer_scene import crease_gbuffer, make_camera, make_scene, render_gbuffer

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


def lit_scene(fp16=False, channels=3):
    """A 64x48 view into a box scene lit by the sun: the direct light has shadows and
    coloured albedos, so the bounce changes the GI noticeably."""
    sc = make_scene(7, 40, 20)
    cam = make_camera(64, 48, fov_y_deg=60, pitch_deg=-25)
    dt = np.float16 if fp16 else np.float32
    gb = render_gbuffer(sc, cam, normal_dtype=dt, radiance_dtype=dt, channels=channels, cache=False)
    return gb, cam, sc


def kw_of(sc, **extra):
    kw = dict(slices=3, steps=6, radius=1.5, thickness=0.4, noise=O.NOISE_R2, seed=5,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    kw.update(extra)
    return kw


def test_sequence_against_oracle(ctx):
    """Four frames, gain 0.9, FP32 light: each frame's masks, AO, GI and ambient against the
    oracle's sequence (masks exact up to traced near-ties, outputs within 1e-3)."""
    import torch
    from paper_2301_11376_amd import Sequence
    gb, cam, sc = lit_scene()
    H, W = gb["depth"].shape
    albedo_np = np.random.default_rng(2).uniform(0.2, 0.8, (H, W, 3)).astype(np.float32)
    kw = kw_of(sc)
    bc, oc = PY.cams(cam)
    bp, op = PY.params(**kw)
    t = PY.to_device(gb)
    albedo = torch.from_numpy(albedo_np).cuda()
    frames = [dict(depth=gb["depth"], normal=gb["normal"], direct=gb["radiance"], albedo=albedo_np)] * 4
    ref = O.bounce_sequence(frames, oc, op, 0.9, return_masks=True)
    seq = Sequence(ctx, W, H)
    try:
        for n in range(4):
            out = seq.step(t["depth"], t["normal"], t["radiance"], albedo, bc, bp, 0.9, masks=True)
            torch.cuda.synchronize()
            gpu = {k: v.cpu().numpy() for k, v in out.items()}
            gpu["masks"] = gpu["masks"].view(np.uint32)
            light = seq.light().cpu().numpy()
            torch.cuda.synchronize()
            assert np.abs(light - ref[n]["light"]).max() <= 1e-3, n
            from dataclasses import replace
            gb_n = dict(gb, radiance=ref[n]["light"].astype(np.float32))
            rep = {}
            PY.compare(gpu, ref[n], gb_n, oc, replace(op, seed=kw["seed"] + n), report=rep)
            log(f"frame {n}: {rep['mask_agreement']:.6f} masks, max err {rep['max_err']}")
        assert seq.frame == 4
    finally:
        seq.close()


@pytest.mark.parametrize("light_dtype,resolution,fp16_inputs", [("f32", 1, False), ("f16", 1, False),
                                                                  ("f32", 2, True)])
def test_sequence_equals_composition(ctx, light_dtype, resolution, fp16_inputs):
    """Every step equals, bit for bit, ssvb_inject_bounce into a light image of the same
    type followed by ssvb_compute with seed + n; reset starts again at frame 0."""
    import torch
    from paper_2301_11376_amd import Sequence, Params
    gb, cam, sc = lit_scene(fp16=fp16_inputs, channels=4 if fp16_inputs else 3)
    H, W = gb["depth"].shape
    albedo = torch.full((H, W, 3), 0.65, device="cuda")
    kw = kw_of(sc, resolution=resolution, noise=O.NOISE_HASH, seed=0xFFFFFFFE)  # the seed wraps at frame 2
    bc, _ = PY.cams(cam)
    t = PY.to_device(gb)
    ldt = torch.float16 if light_dtype == "f16" else torch.float32
    seq = Sequence(ctx, W, H, light_dtype=light_dtype)
    try:
        for rep in range(2):
            gi_prev = torch.zeros((H, W, 3), device="cuda")
            for n in range(3):
                light = torch.empty((H, W, 3), dtype=ldt, device="cuda")
                ctx.inject_bounce(t["radiance"], albedo, gi_prev, 0.8, out=light)
                pn = Params(**dict(kw, seed=(kw["seed"] + n) % (1 << 32)))
                want = ctx.compute(t["depth"], t["normal"], light, bc, pn)
                got = seq.step(t["depth"], t["normal"], t["radiance"], albedo, bc, Params(**kw), 0.8)
                got_light = seq.light()
                torch.cuda.synchronize()
                assert torch.equal(got_light, light), (rep, n)
                for k in ("ao", "gi", "ambient"):
                    assert torch.equal(got[k], want[k]), (rep, n, k)
                gi_prev = want["gi"]
            assert seq.frame == 3
            seq.reset()
            assert seq.frame == 0
        log(f"{light_dtype} light, resolution {resolution}: 2 x 3 frames bit-identical to the composition")
    finally:
        seq.close()


def test_sequence_feedback_converges(ctx):
    """The lit crease with FIXED noise (the same slices every frame): the GI grows frame
    after frame to a fixed point (reached exactly in FP32 within a few frames), as the
    oracle's sequence does."""
    import torch
    from paper_2301_11376_amd import Sequence
    cam = make_camera(48, 32, fov_y_deg=70, pitch_deg=-30)
    gb = crease_gbuffer(cam, D=3.0, alpha=math.radians(60))
    H, W = gb["depth"].shape
    kw = dict(slices=4, steps=8, radius=2.0, thickness=float("inf"), noise=O.NOISE_FIXED)
    bc, oc = PY.cams(cam)
    bp, op = PY.params(**kw)
    t = PY.to_device(gb)
    alb_np = np.full((H, W, 3), 0.7, np.float32)
    albedo = torch.from_numpy(alb_np).cuda()
    frames = [dict(depth=gb["depth"], normal=gb["normal"], direct=gb["radiance"], albedo=alb_np)] * 6
    ref = O.bounce_sequence(frames, oc, op, 0.9)
    seq = Sequence(ctx, W, H)
    try:
        sums = []
        for n in range(6):
            out = seq.step(t["depth"], t["normal"], t["radiance"], albedo, bc, bp, 0.9)
            torch.cuda.synchronize()
            gi = out["gi"].cpu().numpy()
            assert np.abs(gi - ref[n]["gi"]).max() <= 1e-3, n
            sums.append(float(gi.sum()))
        inc = np.diff(sums)
        log(f"GI sums {sums}")
        # rises, never falls, and settles (in FP32 the fixed point is reached exactly
        # within a few frames, after which the increments are 0)
        assert inc[0] > 0 and np.all(inc >= 0) and inc[-1] < 1e-2 * inc[0]
    finally:
        seq.close()


def test_sequence_rejects(ctx):
    """Arguments are checked before anything is launched; a refused step leaves the frame
    counter where it was."""
    import torch
    from paper_2301_11376_amd import Sequence, Params, SSVBError, Camera
    gb, cam, sc = lit_scene()
    H, W = gb["depth"].shape
    bc, _ = PY.cams(cam)
    t = PY.to_device(gb)
    albedo = torch.full((H, W, 3), 0.5, device="cuda")
    p = Params(**kw_of(sc))
    with pytest.raises(SSVBError) as e:
        Sequence(ctx, 0, 16)
    assert e.value.status == 1
    seq = Sequence(ctx, W, H)
    try:
        with pytest.raises(SSVBError) as e:
            seq.step(t["depth"], t["normal"], t["radiance"], albedo, bc, p, -1.0)
        assert e.value.status == 1
        with pytest.raises(SSVBError) as e:
            seq.step(t["depth"], t["normal"], t["radiance"], albedo, bc, p, float("inf"))
        assert e.value.status == 1
        small = Camera(W - 1, H, cam.fx, cam.fy, cam.cx, cam.cy, tuple(cam.view_to_world))
        with pytest.raises((SSVBError, ValueError)):
            seq.step(t["depth"][:, :W - 1], t["normal"][:, :W - 1], t["radiance"][:, :W - 1], albedo[:, :W - 1],
                     small, p, 0.5)
        assert seq.frame == 0
        seq.step(t["depth"], t["normal"], t["radiance"], albedo, bc, p, 0.5)
        torch.cuda.synchronize()
        assert seq.frame == 1
    finally:
        seq.close()
