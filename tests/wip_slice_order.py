"""GPU: the slice-major work order of ssvb_compute (ssvb_set_slice_order) against the
default order on the same frames and against the oracle.

Held out of collection until it has passed on the GPU: run it by naming the file
(python -m pytest tests/wip_slice_order.py -m gpu).  Bars: masks and AO equal to the default
order's bit for bit (the same per-slice march; the AO adds multiples of 1/N_b, exact in
any order), GI and ambient within FP32 rounding of a different grouping of the same
terms (5e-6 relative, 1e-6 absolute), every chunk size the same outputs bit for bit, and
the oracle's parity bar."""
import sys

import numpy as np
import pytest

import oracle as O
import parity as PY
from gbuffer_scene import make_camera, workload

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


def host_copy(out):
    """Outputs on the host; the masks as unsigned words, as the oracle returns them."""
    res = {k: v.cpu().numpy() for k, v in out.items()}
    if "masks" in res:
        res["masks"] = res["masks"].view(np.uint32)
    return res


def both_orders(ctx, gb, cam, kw, chunks=(1, 64, 65536), masks=True):
    """Outputs of the default order and of the slice-major order at each chunk size."""
    import torch
    bc, _ = PY.cams(cam)
    bp, _ = PY.params(**kw)
    t = PY.to_device(gb)
    ref = ctx.compute(t["depth"], t["normal"], t["radiance"], bc, bp, masks=masks)
    torch.cuda.synchronize()
    ref = host_copy(ref)
    runs = []
    try:
        for c in chunks:
            ctx.set_slice_order(c)
            got = ctx.compute(t["depth"], t["normal"], t["radiance"], bc, bp, masks=masks)
            torch.cuda.synchronize()
            runs.append(host_copy(got))
    finally:
        ctx.set_slice_order(0)
    return ref, runs


def check_orders(ref, runs, bitwise_ao=True):
    for got in runs[1:]:
        for k in got:
            assert np.array_equal(got[k].view(np.uint32), runs[0][k].view(np.uint32)), ("chunk", k)
    got = runs[0]
    for k in ("ao", "gi", "ambient"):
        assert np.all(np.isfinite(got[k])), k
    if "masks" in got:
        assert np.array_equal(got["masks"], ref["masks"])
    if bitwise_ao:
        assert np.array_equal(got["ao"].view(np.uint32), ref["ao"].view(np.uint32))
    else:
        assert np.abs(got["ao"] - ref["ao"]).max() <= 1e-6
    # the same FP32 terms summed in another grouping: at the 1080p and 4K workloads the host
    # build of both orders differs by at most 1.9e-7 absolute and 6e-7 relative; the bar
    # leaves a factor of about 5-10 for the device's own contraction choices
    for k in ("gi", "ambient"):
        np.testing.assert_allclose(got[k], ref[k], rtol=5e-6, atol=1e-6, err_msg=k)
    return got


CASES = {
    "hash_t04": (PY.VARIANTS["hash_t04"], (64, 48)),
    "r2_tinf": (PY.VARIANTS["r2_tinf"], (67, 45)),
    "pseudo_128": (dict(slices=3, steps=6, radius=1.3, thickness=0.3, noise=O.NOISE_R2, seed=2, sectors=128,
                        hit_criterion=1), (37, 29)),
    "quad_8dirs": (dict(slices=8, steps=5, radius=1.5, thickness=0.4, noise=O.NOISE_HASH, seed=4,
                        step_distribution=1, ambient_samples=8), (40, 9)),
    "one_pixel": (dict(slices=2, steps=3, radius=1.0, noise=O.NOISE_HASH, seed=5), (1, 1)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_slice_order_small(ctx, name):
    kw, (W, H) = CASES[name]
    log(f"slice order {name} {W}x{H}")
    gb, cam, sc = PY.tiny(W, H)
    kw = dict(kw, ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    ref, runs = both_orders(ctx, gb, cam, kw)
    got = check_orders(ref, runs)
    _, oc = PY.cams(cam)
    _, op = PY.params(**kw)
    oref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, return_masks=True)
    PY.compare(got, oref, gb, oc, op, agreement=0.0 if W * H < 100 else PY.MASK_AGREEMENT)


def test_slice_order_half_resolution(ctx):
    gb, cam, sc = PY.tiny(67, 45)
    log("slice order half resolution 67x45")
    kw = dict(PY.HALF_CASES["uniform"], resolution=2, ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    ref, runs = both_orders(ctx, gb, cam, kw, masks=False)
    got = check_orders(ref, runs)
    _, oc = PY.cams(cam)
    _, op = PY.params(**kw)
    oref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op)
    for k in ("ao", "gi", "ambient"):
        assert np.abs(got[k] - oref[k]).max() <= 1e-3, k


def test_slice_order_background(ctx):
    log("slice order sky frame 19x11")
    cam = make_camera(19, 11, fov_y_deg=60, pitch_deg=0)
    gb = {"depth": np.zeros((11, 19), np.float32), "normal": np.zeros((11, 19, 3), np.float32),
          "radiance": np.ones((11, 19, 3), np.float32)}
    ref, runs = both_orders(ctx, gb, cam, dict(slices=3, steps=4, radius=1.0, noise=O.NOISE_HASH, seed=1))
    got = check_orders(ref, runs)
    assert np.all(got["ao"] == 1) and np.all(got["gi"] == 0) and np.all(got["masks"] == 0)


def test_slice_order_1080p_sampled(ctx):
    """The 1920x1080 workload frame in slice-major order (chunk 256): against the default
    order over the whole frame, and the oracle on a seeded sample of 3,000 pixels."""
    gb, cam, w, sc = workload("c2_1080p")
    log("slice order 1920x1080")
    H, W = gb["depth"].shape
    kw = dict(slices=4, steps=16, radius=3.0, thickness=0.5, noise=O.NOISE_R2, seed=2,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    ref, runs = both_orders(ctx, gb, cam, kw, chunks=(256,))
    got = check_orders(ref, runs)
    pix = PY.sample_pixels(H, W, 3000, 2)
    _, oc = PY.cams(cam)
    _, op = PY.params(**kw)
    oref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, pixels=pix, return_masks=True)
    PY.compare(got, oref, gb, oc, op, pixels=pix)


def test_slice_order_4k_fp16_sampled(ctx):
    """The 3840x2160 FP16 workload frame in slice-major order (chunk 256): against the
    default order over the whole frame (masks not requested), and the oracle on the same
    FP16 values on a seeded sample of 800 pixels plus the corners."""
    gb, cam, w, sc = workload("c3_4k_fp16")
    log("slice order 3840x2160 fp16")
    H, W = gb["depth"].shape
    kw = dict(slices=8, steps=32, radius=8.0, thickness=w["thickness"], noise=O.NOISE_R2, seed=3,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    ref, runs = both_orders(ctx, gb, cam, kw, chunks=(256,), masks=False)
    got = check_orders(ref, runs)
    pix = PY.sample_pixels(H, W, 800, 3)
    _, oc = PY.cams(cam)
    _, op = PY.params(**kw)
    oref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, pixels=pix)
    ys, xs = pix
    for k in ("ao", "gi", "ambient"):
        err = np.abs(got[k][ys, xs] - oref[k]).max()
        log(f"  {k}: max |error| {err:.3e} against the oracle")
        assert err <= 1e-3, k


def test_slice_order_buffer_growth_two_streams(ctx):
    """On a fresh context: a small frame, then a larger one (the partial buffer grows while
    the first may still run), then the small one again, alternating two streams with no
    host synchronisation, the outputs allocated beforehand: each result equals the same
    frame's result run alone."""
    import torch
    from paper_2301_11376_amd import Context
    log("slice order buffer growth, two streams")
    frames = []
    for W, H in ((40, 30), (96, 64), (40, 30)):
        gb, cam, sc = PY.tiny(W, H)
        kw = dict(slices=3, steps=6, radius=1.3, thickness=0.3, noise=O.NOISE_R2, seed=2,
                  ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
        bc, _ = PY.cams(cam)
        bp, _ = PY.params(**kw)
        frames.append((PY.to_device(gb), bc, bp, W, H))
    alone = []
    try:
        ctx.set_slice_order(16)
        for t, bc, bp, W, H in frames:
            out = ctx.compute(t["depth"], t["normal"], t["radiance"], bc, bp)
            torch.cuda.synchronize()
            alone.append(host_copy(out))
    finally:
        ctx.set_slice_order(0)
    fresh = Context(0)
    try:
        fresh.set_slice_order(16)
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        outs = [Context.alloc_outputs(H, W, 3, "cuda") for _, _, _, W, H in frames]
        torch.cuda.synchronize()
        for i, (t, bc, bp, W, H) in enumerate(frames):
            fresh.compute(t["depth"], t["normal"], t["radiance"], bc, bp, out=outs[i], stream=streams[i % 2])
        torch.cuda.synchronize()
    finally:
        fresh.close()
    for a, o in zip(alone, outs):
        for k in ("ao", "gi", "ambient"):
            assert np.array_equal(o[k].cpu().numpy().view(np.uint32), a[k].view(np.uint32)), k


def test_slice_order_rejects(ctx):
    """Chunk sizes outside [0, 65536] are refused and leave the order as it was."""
    import torch
    from paper_2301_11376_amd import SSVBError
    gb, cam, sc = PY.tiny(40, 30)
    kw = dict(slices=3, steps=6, radius=1.3, thickness=0.3, noise=O.NOISE_R2, seed=2)
    ref, _ = both_orders(ctx, gb, cam, kw, chunks=())
    for bad in (-1, 65537, 1 << 30):
        with pytest.raises(SSVBError) as e:
            ctx.set_slice_order(bad)
        assert e.value.status == 1
    # still the default order: the same outputs bit for bit
    bc, _ = PY.cams(cam)
    bp, _ = PY.params(**kw)
    t = PY.to_device(gb)
    out = ctx.compute(t["depth"], t["normal"], t["radiance"], bc, bp, masks=True)
    torch.cuda.synchronize()
    out = host_copy(out)
    for k in ref:
        assert np.array_equal(out[k].view(np.uint32), ref[k].view(np.uint32)), k
