"""GPU: batched persistent path, launch shapes and the autotuner.

A frame in a batch must produce exactly what ssvb_compute writes for it with the same
launch shape (same device code, same frame constants); every launch shape must meet the
oracle's tolerances; the autotuner must return and remember a valid shape.
"""
import sys

import numpy as np
import pytest

import oracle as O
import parity as PY
from gbuffer_scene import make_camera, make_scene, render_gbuffer

pytestmark = pytest.mark.gpu

INF = float("inf")


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


def scene_frames(specs):
    """specs: list of (W, H, seed, fp16, channels, kw); returns host G-buffers, cameras, params."""
    out = []
    for W, H, seed, fp16, ch, kw in specs:
        sc = make_scene(seed, 40, 20)
        cam = make_camera(W, H, fov_y_deg=60, pitch_deg=-25)
        dt = np.float16 if fp16 else np.float32
        gb = render_gbuffer(sc, cam, normal_dtype=dt, radiance_dtype=dt, channels=ch, cache=False)
        kw = dict(kw, ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
        out.append((gb, cam, kw))
    return out


MIXED = [
    (67, 45, 1, False, 3, dict(slices=3, steps=5, radius=1.2, thickness=0.4, noise=O.NOISE_HASH, seed=1)),
    (128, 72, 2, True, 4, dict(slices=2, steps=8, radius=2.0, thickness=INF, noise=O.NOISE_R2, seed=2)),
    (33, 91, 3, False, 4, dict(slices=8, steps=3, radius=0.8, thickness=0.1, noise=O.NOISE_HASH, seed=3,
                               hit_criterion=1)),
    (200, 113, 4, True, 3, dict(slices=4, steps=16, radius=3.0, thickness=0.5, thickness_slope=0.05,
                                noise=O.NOISE_R2, seed=4)),
    (1, 1, 5, False, 3, dict(slices=1, steps=1, radius=1.0, noise=O.NOISE_FIXED)),
    (96, 64, 6, False, 3, dict(slices=5, steps=7, radius=1.5, thickness=0.3, noise=O.NOISE_HASH, seed=6,
                               ambient_samples=8, step_distribution=1)),
]

# 128-sector and half-resolution frames, mixed in with 32-sector full-resolution ones
MODES = [
    (80, 50, 7, False, 3, dict(slices=3, steps=6, radius=1.5, thickness=0.3, noise=O.NOISE_HASH, seed=7,
                               sectors=128, ambient_samples=8)),
    (71, 47, 8, True, 4, dict(slices=2, steps=6, radius=1.8, thickness=0.4, noise=O.NOISE_R2, seed=8,
                              resolution=2)),
    (64, 41, 9, False, 3, dict(slices=2, steps=5, radius=1.2, thickness=INF, noise=O.NOISE_HASH, seed=9,
                               sectors=128, resolution=2, hit_criterion=1)),
    (57, 38, 10, True, 3, dict(slices=4, steps=4, radius=1.0, thickness=0.2, noise=O.NOISE_FIXED,
                               sectors=128, step_distribution=1)),
]


def run_plain(ctx, gb, cam, kw):
    bc, _ = PY.cams(cam)
    bp, _ = PY.params(**kw)
    return PY.gpu_run(ctx, gb, bc, bp, masks=kw.get("resolution", 1) == 1)


def assert_same(g, ref, what):
    assert set(g) == set(ref), what
    for k in g:
        assert np.array_equal(g[k].view(np.uint8), ref[k].view(np.uint8)), (what, k)


def run_batch(ctx, items):
    import torch
    from paper_2301_11376_amd import Context
    args, outs = [], []
    for gb, cam, kw in items:
        t = PY.to_device(gb)
        H, W = gb["depth"].shape
        bc, _ = PY.cams(cam)
        bp, _ = PY.params(**kw)
        out = Context.alloc_outputs(H, W, kw["slices"], "cuda", masks=kw.get("resolution", 1) == 1,
                                    sectors=kw.get("sectors", 32))
        for v in out.values():
            v.fill_(-7)
        args.append((t["depth"], t["normal"], t["radiance"], bc, bp, out))
        outs.append(out)
    ctx.compute_batch(args)
    torch.cuda.synchronize()
    res = []
    for out in outs:
        r = {k: v.cpu().numpy() for k, v in out.items()}
        if "masks" in r:
            r["masks"] = r["masks"].view(np.uint32)
        res.append(r)
    return res


def test_batch_equals_plain_bitwise(ctx):
    items = scene_frames(MIXED)
    log(f"batch of {len(items)} mixed frames")
    got = run_batch(ctx, items)
    for (gb, cam, kw), g in zip(items, got):
        assert_same(g, run_plain(ctx, gb, cam, kw), (cam.width, cam.height))


@pytest.mark.parametrize("mix", ["modes", "mixed+modes", "half-only", "128-only"])
def test_batch_modes_equal_plain_bitwise(ctx, mix):
    """Batches holding 128-sector and half-resolution frames (each set of frame kinds
    replays its own graph): every frame as ssvb_compute writes it."""
    specs = {"modes": MODES, "mixed+modes": [m for pair in zip(MIXED, MODES) for m in pair] + MIXED[4:],
             "half-only": [MODES[1], MODES[2]], "128-only": [MODES[0], MODES[3]]}[mix]
    items = scene_frames(specs)
    log(f"batch {mix}: {len(items)} frames")
    got = run_batch(ctx, items)
    for (gb, cam, kw), g in zip(items, got):
        assert_same(g, run_plain(ctx, gb, cam, kw), (cam.width, cam.height, kw.get("sectors", 32),
                                                     kw.get("resolution", 1)))


def test_batch_against_oracle(ctx):
    items = scene_frames(MIXED[:4] + MODES)
    got = run_batch(ctx, items)
    for (gb, cam, kw), g in zip(items, got):
        log(f"batch frame {cam.width}x{cam.height} sectors {kw.get('sectors', 32)} "
            f"resolution {kw.get('resolution', 1)} vs oracle")
        _, oc = PY.cams(cam)
        _, op = PY.params(**kw)
        if kw.get("resolution", 1) == 2:
            ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op)
            for k in ("ao", "gi", "ambient"):
                assert np.abs(g[k] - ref[k]).max() <= 1e-3, k
        else:
            ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, return_masks=True)
            PY.compare(g, ref, gb, oc, op)


def test_batch_chunks_and_repeats(ctx):
    """More than 64 frames (several graph replays, both descriptor slots reused) and the
    same batch twice: identical results."""
    base = scene_frames([(48, 32, 9, False, 3, dict(slices=2, steps=4, radius=1.0, noise=O.NOISE_HASH, seed=0))])[0]
    items = []
    for i in range(70):
        gb, cam, kw = base
        items.append((gb, cam, dict(kw, seed=i, slices=1 + i % 4)))
    log("batch of 70 frames, twice")
    a = run_batch(ctx, items)
    b = run_batch(ctx, items)
    for i, (x, y) in enumerate(zip(a, b)):
        for k in x:
            assert np.array_equal(x[k].view(np.uint8), y[k].view(np.uint8)), (i, k)
    for i in (0, 37, 69):
        gb, cam, kw = items[i]
        ref = run_plain(ctx, gb, cam, kw)
        for k in ("ao", "gi", "ambient", "masks"):
            assert np.array_equal(a[i][k].view(np.uint8), ref[k].view(np.uint8)), (i, k)


def test_batch_empty(ctx):
    ctx.compute_batch([])


SHAPES = [(32, 8, 4, 1), (16, 16, 2, 1), (64, 4, 8, 1), (16, 8, 4, 2), (8, 8, 4, 4), (8, 4, 2, 8), (4, 8, 8, 8)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_launch_shapes_meet_oracle(ctx, shape):
    gb, cam, kw = scene_frames([(75, 53, 11, False, 3, dict(slices=6, steps=6, radius=1.4, thickness=0.4,
                                                            noise=O.NOISE_R2, seed=5))])[0]
    log(f"launch shape {shape}")
    ctx.set_launch(shape)
    try:
        bc, oc = PY.cams(cam)
        bp, op = PY.params(**kw)
        got = ctx.get_launch(bc, bp)  # the strip is clamped to the frame's tile columns
        assert got[:2] == shape[:2] and got[3] == shape[3]
        assert got[2] == min(shape[2], -(-cam.width // shape[0]))
        g = PY.gpu_run(ctx, gb, bc, bp)
    finally:
        ctx.set_launch(None)
    ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, return_masks=True)
    PY.compare(g, ref, gb, oc, op)


def test_autotune(ctx):
    import torch
    from paper_2301_11376_amd import Context
    gb, cam, kw = scene_frames([(160, 96, 12, False, 3, dict(slices=4, steps=8, radius=2.0, noise=O.NOISE_HASH,
                                                             seed=1))])[0]
    bc, _ = PY.cams(cam)
    bp, _ = PY.params(**kw)
    t = PY.to_device(gb)
    out = Context.alloc_outputs(96, 160, 4, "cuda")
    shape, ms = ctx.autotune(t["depth"], t["normal"], t["radiance"], bc, bp, out)
    log(f"autotune: {shape} {ms:.4f} ms")
    assert shape[0] * shape[1] * shape[3] == 256 and ms > 0
    assert ctx.get_launch(bc, bp) == shape
    torch.cuda.synchronize()


def test_batch_full_sizes(ctx):
    """One batch holding the headline frames at full size (1920x1080 FP32 with two sample
    counts, 3840x2160 FP16 at its 8 x 32 samples, 128x128, and the 1080p frame at half
    resolution and at 128 sectors): every frame equals its single-frame launch bit for
    bit, and the oracle agrees on a seeded sample of pixels."""
    import torch
    from gbuffer_scene import workload
    from paper_2301_11376_amd import Context
    specs = []
    for name, kw in (("c2_1080p", dict(slices=4, steps=16, radius=3.0, thickness=0.5, noise=O.NOISE_R2, seed=2)),
                     ("c3_4k_fp16", dict(slices=8, steps=32, radius=8.0, noise=O.NOISE_R2, seed=3)),
                     ("c1_128", dict(slices=2, steps=8, radius=2.0, thickness=0.5, noise=O.NOISE_HASH, seed=1)),
                     ("c2_1080p", dict(slices=2, steps=8, radius=3.0, thickness=0.5, noise=O.NOISE_R2, seed=9)),
                     ("c2_1080p", dict(slices=2, steps=16, radius=4.0, thickness=0.2, noise=O.NOISE_R2, seed=7,
                                       step_distribution=1, resolution=2)),
                     ("c2_1080p", dict(slices=2, steps=8, radius=3.0, thickness=0.5, noise=O.NOISE_HASH, seed=5,
                                       sectors=128))):
        gb, cam, w, sc = workload(name)
        kw = dict(kw, ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
        if "thickness" not in kw:
            kw["thickness"] = w["thickness"]
        specs.append((gb, cam, kw))
    log(f"batch of {len(specs)} full-size frames")
    args, outs = [], []
    for gb, cam, kw in specs:
        H, W = gb["depth"].shape
        t = PY.to_device(gb)
        bc, _ = PY.cams(cam)
        bp, _ = PY.params(**kw)
        out = Context.alloc_outputs(H, W, kw["slices"], "cuda")
        args.append((t["depth"], t["normal"], t["radiance"], bc, bp, out))
        outs.append(out)
    ctx.compute_batch(args)
    torch.cuda.synchronize()
    for i, ((gb, cam, kw), out) in enumerate(zip(specs, outs)):
        got = {k: v.cpu().numpy() for k, v in out.items()}
        ref_plain = run_plain(ctx, gb, cam, dict(kw))
        ref_plain.pop("masks", None)
        assert_same(got, ref_plain, (i, cam.width, cam.height))
        H, W = gb["depth"].shape
        ys, xs = PY.sample_pixels(H, W, 300, 10 + i)
        if kw.get("resolution", 1) == 2:
            # the gathered pixels of a half-resolution frame are the full-resolution gather's
            ys, xs = ys - ys % 2, xs - xs % 2
        _, oc = PY.cams(cam)
        _, op = PY.params(**dict(kw, resolution=1))
        ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, pixels=(ys, xs))
        err = max(float(np.abs(got[k][ys, xs] - ref[k]).max()) for k in ("ao", "gi", "ambient"))
        log(f"  frame {i} {cam.width}x{cam.height} {kw.get('sectors', 32)} sectors, resolution "
            f"{kw.get('resolution', 1)}: max |error| at {len(ys)} sampled pixels {err:.2e}")
        assert err <= 1e-3, i


def test_batch_packed_edge_cases(ctx):
    """Packed lists with one-tile frames, split points inside frames and a heavy frame
    among light ones (costs from 1 x 1 to 16 x 64 samples per pixel), 128-sector and
    half-resolution frames mixed in: every frame equals its single-frame launch."""
    rng = np.random.default_rng(17)
    specs = []
    for i in range(60):
        W, H = int(rng.integers(1, 40)), int(rng.integers(1, 24))
        kw = dict(slices=int(rng.integers(1, 5)), steps=int(rng.integers(1, 9)), radius=float(rng.uniform(0.5, 3)),
                  thickness=float(rng.uniform(0.1, 1.0)), noise=O.NOISE_HASH, seed=i)
        if i % 7 == 3:
            kw["sectors"] = 128
        if i % 11 == 5 and W > 1 and H > 1:
            kw["resolution"] = 2
        specs.append((W, H, 20 + i % 3, bool(i % 2), 3, kw))
    specs.insert(30, (150, 90, 9, False, 3, dict(slices=16, steps=64, radius=4.0, thickness=0.5,
                                                  noise=O.NOISE_R2, seed=99)))
    items = scene_frames(specs)
    log(f"packed edge cases: {len(items)} frames")
    got = run_batch(ctx, items)
    for i, ((gb, cam, kw), g) in enumerate(zip(items, got)):
        assert_same(g, run_plain(ctx, gb, cam, kw), (i, cam.width, cam.height))
