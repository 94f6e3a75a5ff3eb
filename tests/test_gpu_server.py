"""GPU: the request loop (ssvb_server_*).

Every served frame must equal, bit for bit, what ssvb_compute writes for it alone (same
launch shape, same device code); frames must be admitted within the HBM budget, rounds
must overlap when requests arrive while another round is on the device, and the error
paths must report the documented status codes.
"""
import sys
import time

import numpy as np
import pytest

import oracle as O
import parity as PY
from gbuffer_scene import make_camera, make_scene, render_gbuffer, plane_gbuffer

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


def footprint(W, H, nbytes_px, rbytes_px):
    up = lambda n: (n + 255) // 256 * 256
    px = W * H
    return up(px * 4) + up(px * nbytes_px) + up(px * rbytes_px) + up(px * 4) + 2 * up(px * 12)


SPECS = [  # W, H, scene seed, fp16, channels, params
    (67, 45, 1, False, 3, dict(slices=3, steps=5, radius=1.2, thickness=0.4, noise=O.NOISE_HASH, seed=1)),
    (128, 72, 2, True, 4, dict(slices=2, steps=8, radius=2.0, thickness=float("inf"), noise=O.NOISE_R2, seed=2)),
    (33, 91, 3, False, 4, dict(slices=8, steps=3, radius=0.8, thickness=0.1, noise=O.NOISE_HASH, seed=3,
                               hit_criterion=1)),
    (200, 113, 4, True, 3, dict(slices=4, steps=16, radius=3.0, thickness=0.5, thickness_slope=0.05,
                                noise=O.NOISE_R2, seed=4)),
    (96, 64, 6, False, 3, dict(slices=5, steps=7, radius=1.5, thickness=0.3, noise=O.NOISE_HASH, seed=6,
                               ambient_samples=8)),
    (160, 90, 7, True, 3, dict(slices=7, steps=9, radius=2.5, thickness=0.6, noise=O.NOISE_R2, seed=7)),
]


def make_items(specs):
    out = []
    for W, H, seed, fp16, ch, kw in specs:
        sc = make_scene(seed, 40, 20)
        cam = make_camera(W, H, fov_y_deg=60, pitch_deg=-25)
        dt = np.float16 if fp16 else np.float32
        gb = render_gbuffer(sc, cam, normal_dtype=dt, radiance_dtype=dt, channels=ch, cache=False)
        out.append((gb, cam, dict(kw, ambient_sh=tuple(sc.ambient_sh.reshape(-1)))))
    return out


def device_request(gb, cam, kw, pinned=False):
    import torch
    from paper_2301_11376_amd import Context
    H, W = gb["depth"].shape
    if pinned:
        t = {k: torch.from_numpy(np.ascontiguousarray(v)).pin_memory() for k, v in gb.items()}
        out = {"ao": torch.empty((H, W), pin_memory=True), "gi": torch.empty((H, W, 3), pin_memory=True),
               "ambient": torch.empty((H, W, 3), pin_memory=True)}
    else:
        t = PY.to_device(gb)
        out = Context.alloc_outputs(H, W, kw["slices"], "cuda")
    for v in out.values():
        v.fill_(float("nan"))
    bc, _ = PY.cams(cam)
    bp, _ = PY.params(**kw)
    return t, bc, bp, out


def host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def plain(ctx, gb, cam, kw):
    bc, _ = PY.cams(cam)
    bp, _ = PY.params(**kw)
    return PY.gpu_run(ctx, gb, bc, bp, masks=False)


def same(a, b, what):
    for k in ("ao", "gi", "ambient"):
        assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), (what, k)


def test_served_equals_plain(ctx):
    import torch
    from paper_2301_11376_amd import Server
    items = make_items(SPECS)
    srv = Server(ctx, 512 << 20, streams=2)
    try:
        reqs = []
        for i, (gb, cam, kw) in enumerate(items):
            t, bc, bp, out = device_request(gb, cam, kw)
            torch.cuda.synchronize()
            reqs.append((srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out), out))
            if i % 2:
                time.sleep(0.001)
        log(f"submitted {len(reqs)} requests")
        for tk, _ in reqs:
            lat = srv.wait(tk, 60000)
            assert lat >= 0
        for (tk, out), (gb, cam, kw) in zip(reqs, items):
            assert srv.poll(tk)[0]
            same(host(out), plain(ctx, gb, cam, kw), (cam.width, cam.height))
            srv.release(tk)
        st = srv.stats()
        log(f"stats {st}")
        assert st["completed"] == len(items) and st["failed"] == 0
        assert st["arena_in_use"] == 0 and 0 < st["arena_peak"] <= st["arena_bytes"]
        assert st["frames_in_rounds"] == len(items) and st["rounds"] >= 1
    finally:
        srv.close()


def test_served_against_oracle(ctx):
    import torch
    from paper_2301_11376_amd import Server
    gb, cam, kw = make_items(SPECS[:1])[0]
    srv = Server(ctx, 64 << 20)
    try:
        t, bc, bp, out = device_request(gb, cam, kw)
        torch.cuda.synchronize()
        tk = srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out)
        srv.wait(tk, 60000)
        srv.release(tk)
    finally:
        srv.close()
    _, oc = PY.cams(cam)
    _, op = PY.params(**kw)
    ref = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, return_masks=True)
    got = host(out)
    got["masks"] = PY.gpu_run(ctx, gb, *PY.cams(cam)[:1], PY.params(**kw)[0])["masks"]
    PY.compare(got, ref, gb, oc, op)


def test_admission_within_budget(ctx):
    """A budget that holds two of these frames at a time: all eight finish, the arena
    never holds more than the budget, and each result equals the plain launch's."""
    import torch
    from paper_2301_11376_amd import Server
    spec = (160, 90, 7, False, 3, dict(slices=3, steps=6, radius=2.0, thickness=0.5, noise=O.NOISE_HASH, seed=0))
    gb, cam, kw = make_items([spec])[0]
    fp = footprint(160, 90, 12, 12)
    srv = Server(ctx, 2 * fp + 1000, streams=2)
    try:
        reqs = []
        for i in range(8):
            k = dict(kw, seed=i)
            t, bc, bp, out = device_request(gb, cam, k)
            torch.cuda.synchronize()
            reqs.append((srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out), out, k))
        for tk, out, k in reqs:
            srv.wait(tk, 60000)
            same(host(out), plain(ctx, gb, cam, k), k["seed"])
            srv.release(tk)
        st = srv.stats()
        log(f"stats {st}")
        assert st["completed"] == 8 and st["arena_peak"] <= 2 * fp + 1000 and st["rounds"] >= 4
        assert st["max_round_frames"] <= 2
    finally:
        srv.close()


def big_plane(W, H):
    cam = make_camera(W, H, fov_y_deg=60, pitch_deg=-25)
    gb = plane_gbuffer(cam, (0.0, 1.0, 0.3), (0.0, -1.5, -4.0))
    return gb, cam


def test_rounds_overlap_and_alone_equals_mix(ctx):
    """A long frame is on the device when small ones arrive: they are admitted and start
    on the second stream while it runs; every frame equals its result served alone."""
    import torch
    from paper_2301_11376_amd import Server
    gb_big, cam_big = big_plane(2560, 1440)
    kw_big = dict(slices=8, steps=32, radius=4.0, thickness=0.5, noise=O.NOISE_R2, seed=9)
    small = make_items(SPECS[:4])
    srv = Server(ctx, 2 << 30, streams=2)
    try:
        # alone
        alone = []
        for gb, cam, kw in [(gb_big, cam_big, kw_big)] + small:
            t, bc, bp, out = device_request(gb, cam, kw)
            torch.cuda.synchronize()
            tk = srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out)
            srv.wait(tk, 60000)
            srv.release(tk)
            alone.append(host(out))
        st0 = srv.stats()
        # in the mix
        reqs = []
        prepared = [device_request(gb, cam, kw) for gb, cam, kw in [(gb_big, cam_big, kw_big)] + small]
        torch.cuda.synchronize()
        for i, (t, bc, bp, out) in enumerate(prepared):
            reqs.append((srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out), out))
            if i == 0:
                time.sleep(0.002)  # the long frame is on the device by now
        for tk, _ in reqs:
            srv.wait(tk, 60000)
        st = srv.stats()
        log(f"stats {st}")
        for (tk, out), ref in zip(reqs, alone):
            same(host(out), ref, tk)
            srv.release(tk)
        assert st["max_running_rounds"] >= 2
        assert st["admitted_while_running"] > st0["admitted_while_running"]
    finally:
        srv.close()


def test_submit_orders_after_caller_stream(ctx):
    """Inputs written and outputs cleared by work still queued on the caller's stream,
    submitted with no host synchronisation: the server waits for that work (an event
    recorded on the caller's stream at submission), so the results equal plain launches
    on the final inputs (device buffers, read and written in place)."""
    import torch
    from paper_2301_11376_amd import Server
    items = make_items(SPECS[:2])
    refs = [host(plain(ctx, gb, cam, kw)) for gb, cam, kw in items]
    srv = Server(ctx, 256 << 20)
    try:
        for rep in range(2):
            reqs = []
            for (gb, cam, kw), ref in zip(items, refs):
                t, bc, bp, out = device_request(gb, cam, kw, pinned=False)
                src = {k: v.clone() for k, v in t.items()}
                for v in t.values():
                    v.zero_()  # depth 0: every pixel background until the copy below lands
                torch.cuda.synchronize()
                # tens of milliseconds of queued work, then the real inputs
                a = torch.randn(4096, 4096, device="cuda")
                for _ in range(12):
                    a = torch.mm(a, a) * 1e-2
                for k in t:
                    t[k].copy_(src[k])
                for v in out.values():
                    v.fill_(float("nan"))
                reqs.append((srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out), out, ref, t, src))
            for tk, out, ref, _, _ in reqs:
                srv.wait(tk, 60000)
                same(host(out), ref, (rep, tk))
                srv.release(tk)
            log(f"rep {rep}: {len(reqs)} requests ordered after the caller's stream")
    finally:
        srv.close()


def test_pinned_host_buffers(ctx):
    from paper_2301_11376_amd import Server
    items = make_items(SPECS[3:5])
    srv = Server(ctx, 256 << 20)
    try:
        reqs = []
        for gb, cam, kw in items:
            t, bc, bp, out = device_request(gb, cam, kw, pinned=True)
            reqs.append((srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out), out))
        for (tk, out), (gb, cam, kw) in zip(reqs, items):
            srv.wait(tk, 60000)
            same(host(out), plain(ctx, gb, cam, kw), cam.width)
            srv.release(tk)
    finally:
        srv.close()


def test_error_paths(ctx):
    import torch
    from paper_2301_11376_amd import Server, SSVBError
    gb, cam, kw = make_items(SPECS[:1])[0]
    srv = Server(ctx, footprint(67, 45, 12, 12))
    try:
        t, bc, bp, out = device_request(gb, cam, kw)
        torch.cuda.synchronize()
        # fits exactly
        tk = srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out)
        srv.wait(tk, 60000)
        with pytest.raises(SSVBError) as e:
            srv.release(tk + 1000)
        assert e.value.status == 7
        srv.release(tk)
        with pytest.raises(SSVBError) as e:
            srv.poll(tk)
        assert e.value.status == 7
        # larger than the whole arena
        gb2, cam2, kw2 = make_items(SPECS[3:4])[0]
        t2, bc2, bp2, out2 = device_request(gb2, cam2, kw2)
        with pytest.raises(SSVBError) as e:
            srv.submit(t2["depth"], t2["normal"], t2["radiance"], bc2, bp2, out2)
        assert e.value.status == 3
        # masks are not served
        out_m = dict(out, masks=torch.empty((45, 67, kw["slices"]), dtype=torch.int32, device="cuda"))
        with pytest.raises(SSVBError) as e:
            srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out_m)
        assert e.value.status == 1
        # an empty frame finishes at once
        from paper_2301_11376_amd import Camera
        z = torch.empty((0, 0), device="cuda")
        z3 = torch.empty((0, 0, 3), device="cuda")
        tk0 = srv.submit(z, z3, z3, Camera(0, 0, 1.0, 1.0, 0.0, 0.0), bp, {"ao": z, "gi": z3, "ambient": z3})
        assert srv.poll(tk0)[0]
        srv.release(tk0)
        assert srv.stats()["failed"] == 0
    finally:
        srv.close()
    # the budget must hold something
    with pytest.raises(SSVBError) as e:
        Server(ctx, 16)
    assert e.value.status == 1


def test_wait_timeout(ctx):
    import torch
    from paper_2301_11376_amd import Server, SSVBError
    gb, cam = big_plane(2560, 1440)
    kw = dict(slices=8, steps=32, radius=4.0, thickness=0.5, noise=O.NOISE_R2, seed=3)
    srv = Server(ctx, 1 << 30)
    try:
        t, bc, bp, out = device_request(gb, cam, kw)
        torch.cuda.synchronize()
        tk = srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out)
        with pytest.raises(SSVBError) as e:
            srv.wait(tk, 0.0)
        assert e.value.status == 6
        with pytest.raises(SSVBError) as e:
            srv.release(tk)
        assert e.value.status == 5
        srv.wait(tk, 60000)
        srv.release(tk)
    finally:
        srv.close()


def test_mixed_residency(ctx):
    """Buffers in device memory are used in place, those in host memory staged through the
    arena: every mix gives the per-frame launch's result."""
    import torch
    from paper_2301_11376_amd import Server
    gb, cam, kw = make_items(SPECS[3:4])[0]
    H, W = gb["depth"].shape
    ref = plain(ctx, gb, cam, kw)
    bc, _ = PY.cams(cam)
    bp, _ = PY.params(**kw)
    dev = PY.to_device(gb)
    pin = {k: torch.from_numpy(np.ascontiguousarray(v)).pin_memory() for k, v in gb.items()}
    srv = Server(ctx, 256 << 20)
    try:
        for mix in [("cuda", "pin", "cuda", "pin"), ("pin", "cuda", "pin", "cuda"), ("cuda", "cuda", "cuda", "pin")]:
            src = [dev if m == "cuda" else pin for m in mix[:3]]
            if mix[3] == "cuda":
                out = {"ao": torch.empty((H, W), device="cuda"), "gi": torch.empty((H, W, 3), device="cuda"),
                       "ambient": torch.empty((H, W, 3), device="cuda")}
            else:
                out = {"ao": torch.empty((H, W), pin_memory=True), "gi": torch.empty((H, W, 3), pin_memory=True),
                       "ambient": torch.empty((H, W, 3), pin_memory=True)}
            for v in out.values():
                v.fill_(float("nan"))
            torch.cuda.synchronize()
            tk = srv.submit(src[0]["depth"], src[1]["normal"], src[2]["radiance"], bc, bp, out)
            srv.wait(tk, 60000)
            srv.release(tk)
            same(host(out), ref, mix)
    finally:
        srv.close()


def test_served_modes(ctx):
    """128 sectors, half resolution and quadratic steps are served like any frame: the
    results equal ssvb_compute's bit for bit, in one mixed round or alone."""
    import torch
    from paper_2301_11376_amd import Server
    items = make_items(SPECS[:4])
    extra = [dict(sectors=128), dict(resolution=2), dict(step_distribution=1, sectors=128), dict(resolution=2,
                                                                                               step_distribution=1)]
    srv = Server(ctx, 512 << 20, streams=2)
    try:
        reqs = []
        for (gb, cam, kw), ex in zip(items, extra):
            kw = dict(kw, **ex)
            t, bc, bp, out = device_request(gb, cam, kw)
            torch.cuda.synchronize()
            reqs.append((srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out), out, gb, cam, kw))
        for tk, out, gb, cam, kw in reqs:
            srv.wait(tk, 60000)
            same(host(out), plain(ctx, gb, cam, kw), kw)
            srv.release(tk)
        assert srv.stats()["failed"] == 0
    finally:
        srv.close()


def test_many_tiny_requests(ctx):
    """150 tiny requests (1x1 to 39x23, 32 or 128 sectors, full or half resolution) in
    few large rounds of packed frames: every result equals ssvb_compute's."""
    import torch
    from paper_2301_11376_amd import Server
    rng = np.random.default_rng(23)
    specs = []
    for i in range(150):
        W, H = int(rng.integers(1, 40)), int(rng.integers(1, 24))
        kw = dict(slices=int(rng.integers(1, 5)), steps=int(rng.integers(1, 9)), radius=float(rng.uniform(0.5, 3)),
                  thickness=float(rng.uniform(0.1, 1.0)), noise=O.NOISE_R2, seed=i)
        if i % 5 == 2:
            kw["sectors"] = 128
        if i % 9 == 4 and W > 1 and H > 1:
            kw["resolution"] = 2
        specs.append((W, H, 30 + i % 2, bool(i % 3 == 0), 3, kw))
    items = make_items(specs)
    srv = Server(ctx, 256 << 20)
    try:
        reqs = []
        for gb, cam, kw in items:
            t, bc, bp, out = device_request(gb, cam, kw)
            reqs.append((t, out, gb, cam, kw, bc, bp))
        torch.cuda.synchronize()
        tks = [srv.submit(t["depth"], t["normal"], t["radiance"], bc, bp, out) for t, out, gb, cam, kw, bc, bp in reqs]
        for tk, (t, out, gb, cam, kw, bc, bp) in zip(tks, reqs):
            srv.wait(tk, 60000)
            same(host(out), plain(ctx, gb, cam, kw), (cam.width, cam.height))
            srv.release(tk)
        st = srv.stats()
        log(f"tiny requests: {st['rounds']} rounds, largest {st['max_round_frames']} frames")
        assert st["failed"] == 0 and st["completed"] >= len(items)
    finally:
        srv.close()
