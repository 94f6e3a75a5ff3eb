"""Benchmark of the visibility-bitmask gather on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2_1080p]
                [--no-batch] [--no-serve] [--no-autotune] [--no-table2]
                [--serve-requests N] [--serve-sweep] [--no-cpu-baseline]

One step = one pass of the whole hot path (ssvb_compute: AO, GI and ambient of one
frame) over a seeded synthetic 1920x1080 G-buffer already resident in HBM.  Prints one
JSON line with Gsamples/s (a sample is one depth fetch of one pixel, slice, side and
step: px * N_d * 2 * N_s per frame), ms per frame, the roofline of the gather kernel and
the FP64 oracle timed on a bounded sample on the host cores.  Two more legs run the
mixed-frame workloads: a batch of 64 frames of mixed resolution and sample counts (one
graph launch against 64 plain launches) and a Poisson request stream through the
request loop (p50 / p99 latency, frames/s).

Everything the host renders or computes on the CPU (scene pools, the oracle) runs in
forked worker processes before this process touches the GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
import traceback

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
SERVE_BUDGET = 64 << 30  # HBM budget of the request loop
SERVE_STREAMS = 1  # compute streams of the request loop (concurrent rounds measured slower)
HOST_WORKERS = 16  # CPU share of one GPU on the benchmark hosts


def algorithmic_bytes(W, H, nd, ns, fp16):
    """Bytes the method itself moves per frame: every sample reads depth + normal +
    radiance (28 B, or 16 B with FP16 normal and radiance), every pixel reads its own
    depth + normal and writes AO + GI + ambient (44 B, or 38 B)."""
    px = W * H
    samples = px * nd * 2 * ns
    per_sample = 16 if fp16 else 28
    per_px = 38 if fp16 else 44
    return samples, samples * per_sample + px * per_px


def samples_of(f):
    return f["width"] * f["height"] * f["slices"] * 2 * f["steps"]


def device_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in ("ssvb_kernels.hip", "ssvb_pixel.h", "ssvb_internal.h"):
        with open(os.path.join(ROOT, "paper_2301_11376_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name, shape):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE passes
    (scaled by the copy calibration), or None when the device code or the launch shape has
    changed since."""
    path = os.path.join(ROOT, "profiles", f"gather_frame_{workload_name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if (rec.get("device_source_sha256") != device_source_sha256() or rec.get("workload") != workload_name
            or rec.get("launch_shape") != list(shape)):
        return None
    return rec["traffic_bytes_per_launch"]


# ---------------------------------------------------------------------------------------
# cpu_baseline leg: the FP64 oracle as it stands, on row bands, one process per band.  Its
# runs give the timed baseline (a bounded band of each workload, median of 3) and the
# reference outputs the GPU's per-output error is reported against.
# ---------------------------------------------------------------------------------------

# rows per band of the timed baseline (HOST_WORKERS bands, centred in the frame): about
# 63 M samples each at 1080p and 4K, the whole frame at 128x128
TIMED_ROWS = {"c1_128": None, "c2_1080p": 16, "c3_4k_fp16": 2}
# rows of the 4K frame whose outputs are compared with the oracle (centred)
C3_PARITY_ROWS = 135


def oracle_params(O, w, scene):
    return O.Params(slices=w["slices"], steps=w["steps"], radius=w["radius"], thickness=w["thickness"],
                    noise=O.NOISE_NAMES[w["noise"]], seed=w["seed"],
                    ambient_sh=tuple(float(v) for v in scene.ambient_sh.reshape(-1)))


def oracle_camera(O, cam):
    return O.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, tuple(cam.view_to_world))


def cpu_baseline_leg(loaded, workers, names):
    """Timed oracle bands (median of 3 per workload) and the oracle's outputs for the error
    report: the whole 128x128 and 1080p frames (with slice masks) and a centred band of the
    4K frame on its FP16 inputs (with masks) and on the FP32 originals."""
    import oracle as O
    from oracle.bands import compute_rows
    base, refs = {}, {}
    for name in names:
        gb, cam, w, scene = loaded[name][:4]
        H, W = gb["depth"].shape
        oc, prm = oracle_camera(O, cam), oracle_params(O, w, scene)
        rows = TIMED_ROWS[name]
        r0, r1 = (0, H) if rows is None else ((H - workers * rows) // 2, (H - workers * rows) // 2 + workers * rows)
        runs = []
        for _ in range(3):
            res, wall, cpu = compute_rows(gb, oc, prm, r0, r1, workers, return_masks=rows is None)
            runs.append((wall, cpu))
        if rows is None:
            refs[name] = {"rows": (0, H), "fp": res}
        samples = (r1 - r0) * W * w["slices"] * 2 * w["steps"]
        walls = sorted(r[0] for r in runs)
        med = walls[1]
        base[name] = {"value": samples / med / 1e9, "unit": "Gsamples/s", "cores": min(workers, r1 - r0),
                      "kind": "oracle",
                      "sample": f"rows {r0}..{r1 - 1} of the {W}x{H} frame ({(r1 - r0) * W} px, {samples} samples) in "
                                f"{min(workers, r1 - r0)} bands, one single-threaded NumPy FP64 process per band; "
                                f"median of 3 runs ({', '.join(f'{x:.2f}' for x in walls)} s wall)",
                      "single_process_value": samples / float(np.median([r[1] for r in runs])) / 1e9}
        print(f"cpu baseline {name}: {base[name]['value']:.4f} Gsamples/s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    if "c2_1080p" in names:
        gb, cam, w, scene = loaded["c2_1080p"][:4]
        H = gb["depth"].shape[0]
        res, _, _ = compute_rows(gb, oracle_camera(O, cam), oracle_params(O, w, scene), 0, H, workers,
                                 return_masks=True)
        refs["c2_1080p"] = {"rows": (0, H), "fp": res}
    if "c3_4k_fp16" in names:
        gb, cam, w, scene, gb32 = loaded["c3_4k_fp16"]
        H = gb["depth"].shape[0]
        r0 = (H - C3_PARITY_ROWS) // 2
        oc, prm = oracle_camera(O, cam), oracle_params(O, w, scene)
        res16, _, _ = compute_rows(gb, oc, prm, r0, r0 + C3_PARITY_ROWS, workers, return_masks=True)
        res32, _, _ = compute_rows(gb32, oc, prm, r0, r0 + C3_PARITY_ROWS, workers)
        refs["c3_4k_fp16"] = {"rows": (r0, r0 + C3_PARITY_ROWS), "fp": res16, "fp32_originals": res32}
    print(f"oracle reference outputs in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return base, refs


def error_report(gpu, ref, masks=True):
    """Per output: mean, p99 and max of |GPU - FP64 oracle| over every element (AO per
    pixel, GI and ambient per pixel and channel); with masks, the fraction of pixels whose
    slice masks all equal the oracle's."""
    rep = {}
    for k in ("ao", "gi", "ambient"):
        d = np.abs(gpu[k].astype(np.float64) - ref[k]).reshape(-1)
        rep[k] = {"mean": float(d.mean()), "p99": float(np.percentile(d, 99)), "max": float(d.max())}
    if masks:
        g = gpu["masks"].reshape(ref["masks"].shape).view(np.uint32)
        rep["mask_agreement"] = float((g == ref["masks"]).all(axis=-1).mean())
    return rep


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# ---------------------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------------------

def to_params(Params, NOISE_NAMES, f, scene):
    return Params(slices=f["slices"], steps=f["steps"], radius=f["radius"], thickness=f["thickness"],
                  noise=NOISE_NAMES[f["noise"]], seed=f["noise_seed"],
                  ambient_sh=tuple(float(v) for v in scene.ambient_sh.reshape(-1)))


def camera_of(Camera, W, H):
    from gbuffer_scene import make_camera
    c = make_camera(W, H)
    return Camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, tuple(c.view_to_world))


def timed(fn, stream, reps):
    """Median, min and all of `reps` HIP-event timings (ms) of fn() on `stream`."""
    import torch
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts)), float(np.min(ts)), ts


def stream_copy_gbs(mib=1024, reps=20):
    """Measured device-to-device copy bandwidth (bytes read + written per second), the
    practical ceiling beside the 8 TB/s spec figure: median of `reps` event-timed copies."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    s = torch.cuda.current_stream()
    for a, b in ev:
        a.record(s)
        dst.copy_(src)
        b.record(s)
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    del src, dst
    return 2 * n * 4 / (ms * 1e-3) / 1e9


BATCH_WORKLOADS = {
    "mixed": "64 frames, resolution uniform over 1280x720 / 1920x1080 / 2560x1440 / 3840x2160, slices {2,4,8}, "
             "steps {8,16,32}, FP32 G-buffers, radius 3, t 0.5, R2 noise, scenes from 4 procedural seeds per "
             "resolution (64 boxes, 32 thin planes), draw seed 4",
    "small": "64 frames, resolution uniform over 256x144 / 320x180 / 480x270 / 640x360, slices {2,4}, steps {8,16}, "
             "FP32 G-buffers, radius 3, t 0.5, R2 noise, scenes from 2 procedural seeds per resolution "
             "(64 boxes, 32 thin planes), draw seed 6",
}


def batch_frames(kind):
    from gbuffer_scene import mixed_batch, small_batch
    return mixed_batch() if kind == "mixed" else small_batch()


def batch_leg(ctx, pool, autotune, kind="mixed"):
    """64 frames: 64 plain launches on one stream against one graph launch of the
    persistent batch kernel, both with the autotuned shape of each frame's class."""
    import torch
    from paper_2301_11376_amd import Camera, Context, Params, NOISE_NAMES
    frames = batch_frames(kind)
    dev = torch.device("cuda:0")
    base = {}
    for f in frames:
        k = (f["scene_seed"], f["width"], f["height"])
        if k not in base:
            gb, _ = pool[k]
            base[k] = {n: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for n, v in gb.items()}
    items_plain, items_batch = [], []
    for f in frames:
        k = (f["scene_seed"], f["width"], f["height"])
        t = {n: v.clone() for n, v in base[k].items()}  # every frame its own G-buffer in HBM
        cam = camera_of(Camera, f["width"], f["height"])
        p = to_params(Params, NOISE_NAMES, f, pool[k][1])
        oa = Context.alloc_outputs(f["height"], f["width"], f["slices"], dev)
        ob = Context.alloc_outputs(f["height"], f["width"], f["slices"], dev)
        items_plain.append((t["depth"], t["normal"], t["radiance"], cam, p, oa))
        items_batch.append((t["depth"], t["normal"], t["radiance"], cam, p, ob))
    del base
    tuned = 0
    if autotune:
        seen = set()
        for it in items_plain:
            cls = (it[3].width, it[3].height, it[4].slices, it[4].steps)
            if cls in seen:
                continue
            seen.add(cls)
            ctx.autotune(*it)
            tuned += 1
        torch.cuda.synchronize()
        print(f"autotuned {tuned} frame classes", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()

    # arguments marshalled once, outside the timed region, for both paths
    fa_plain, fa_batch = ctx.frames(items_plain), ctx.frames(items_batch)

    def plain():
        ctx.compute_each(fa_plain)

    def batched():
        ctx.compute_batch(fa_batch)

    plain(), batched()
    torch.cuda.synchronize()
    identical = all(torch.equal(a[5][n], b[5][n]) for a, b in zip(items_plain, items_batch)
                    for n in ("ao", "gi", "ambient"))
    # the two paths alternate, run by run, so that drift of the clock or the box falls on
    # both; every run is kept so the speed-up can be read against the spread
    p_all, b_all = [], []
    for _ in range(7):
        p_all += timed(plain, stream, 1)[2]
        b_all += timed(batched, stream, 1)[2]
    p_med, p_min, p_max = float(np.median(p_all)), min(p_all), max(p_all)
    b_med, b_min, b_max = float(np.median(b_all)), min(b_all), max(b_all)
    samples = sum(samples_of(f) for f in frames)
    res = {"workload": BATCH_WORKLOADS[kind],
           "frames": len(frames), "samples": samples, "autotuned_classes": tuned,
           "plain_ms": p_med, "plain_min_ms": p_min, "plain_max_ms": p_max, "plain_runs_ms": p_all,
           "batched_ms": b_med, "batched_min_ms": b_min, "batched_max_ms": b_max, "batched_runs_ms": b_all,
           "speedup": p_med / b_med, "speedup_range": [p_min / b_max, p_max / b_min],
           "speedup_outside_spread": bool(p_min > b_max or p_max < b_min),
           "plain_gsamples_s": samples / p_med / 1e6,
           "batched_gsamples_s": samples / b_med / 1e6, "bit_identical_to_plain": bool(identical)}
    print(f"batch ({kind}): plain {p_med:.2f} ms, batched {b_med:.2f} ms, x{p_med / b_med:.3f}, identical {identical}",
          file=sys.stderr, flush=True)
    del items_plain, items_batch
    torch.cuda.empty_cache()
    return res


# Section 4.3, Table 2 (1920x1080, thickness 0.2): samples per side, radius, step
# distribution, and the paper's sampling time on its GPU (context only)
TABLE2 = [("a", 8, 1.0, "uniform", 1, 0.9), ("b", 8, 4.0, "uniform", 1, 1.7), ("c", 16, 4.0, "uniform", 1, 2.3),
          ("d", 16, 4.0, "quadratic", 1, 2.6), ("e", 32, 4.0, "quadratic", 1, 4.0),
          ("f", 16, 4.0, "quadratic", 2, 0.97)]


def table2_leg(ctx, t, c, scene, slices):
    """The rows of Table 2 on the 1080p G-buffer: N_s, radius, step distribution and
    resolution from the table, `slices` slices, thickness 0.2, R2 noise; median of 20
    launches each (row f: the half-resolution gather plus the upsampling pass)."""
    import torch
    from paper_2301_11376_amd import Params, NOISE_R2, STEPS_UNIFORM, STEPS_QUADRATIC
    H, W = t["depth"].shape
    out = {"ao": torch.empty((H, W), device="cuda"), "gi": torch.empty((H, W, 3), device="cuda"),
           "ambient": torch.empty((H, W, 3), device="cuda")}
    stream = torch.cuda.current_stream()
    rows = []
    for name, ns, radius, dist, res, paper_ms in TABLE2:
        p = Params(slices=slices, steps=ns, radius=radius, thickness=0.2, noise=NOISE_R2, seed=7,
                   step_distribution=STEPS_QUADRATIC if dist == "quadratic" else STEPS_UNIFORM,
                   resolution=res, ambient_sh=tuple(float(v) for v in scene.ambient_sh.reshape(-1)))
        fn = lambda: ctx.compute(t["depth"], t["normal"], t["radiance"], c, p, out=out)
        fn()
        med, mn, _ = timed(fn, stream, 20)
        samples = ((W + res - 1) // res) * ((H + res - 1) // res) * slices * 2 * ns
        rows.append({"row": name, "steps_per_side": ns, "radius": radius, "steps": dist,
                     "resolution": "half" if res == 2 else "full", "ms": med,
                     "gsamples_s": samples / med / 1e6, "paper_sampling_ms_rtx2080": paper_ms})
    # the denoising column: the default denoiser on the gather's outputs at each resolution
    dn = {}
    for res in (1, 2):
        tmp = {k: torch.empty_like(v) for k, v in out.items()}
        dst = {k: torch.empty_like(v) for k, v in out.items()}
        fn = lambda: ctx.denoise(t["depth"], t["normal"], c, out, resolution=res, out=dst, tmp=tmp)
        fn()
        dn[res] = timed(fn, stream, 20)[0]
    for r in rows:
        res = 2 if r["resolution"] == "half" else 1
        r["denoise_ms"] = dn[res]
        r["total_ms"] = r["ms"] + dn[res]
        r["paper_denoise_ms_rtx2080"] = 0.1 if res == 2 else 0.33
    return {"workload": f"1920x1080 G-buffer of the headline workload, {slices} slices, thickness 0.2, R2 noise; "
                        "Table 2's sample counts read as steps per side; the paper's times are for its own GI "
                        "shader on an RTX 2080 (context, not a target)", "rows": rows}


def denoise_leg(ctx, t, c, out, steps):
    """The denoiser (2 passes, normal power 16, plane sigma 0.05) on the 1080p frame's
    outputs: event-timed calls, and each pass's algorithmic bytes (depth 4 + normal 12 +
    seven input channels 28 + seven output channels 28 = 72 B per pixel, FP32 normals)."""
    import torch
    H, W = t["depth"].shape
    tmp = {k: torch.empty_like(v) for k, v in out.items()}
    dst = {k: torch.empty_like(v) for k, v in out.items()}
    stream = torch.cuda.current_stream()
    fn = lambda: ctx.denoise(t["depth"], t["normal"], c, out, out=dst, tmp=tmp)
    fn()
    med, mn, all_ms = timed(fn, stream, steps)
    p90 = float(np.percentile(all_ms, 90))
    nbytes = 2 * W * H * (4 + 12 + 28 + 28)
    gbs = nbytes / (med * 1e-3) / 1e9
    return {"workload": f"{W}x{H}, 2 passes (taps 1 and 2 pixels apart), normal power 16, plane sigma 0.05",
            "ms": med, "ms_min": mn, "ms_p90": p90, "paper_ms_rtx2080": 0.33,
            "algorithmic_bytes": nbytes, "achieved_gbs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}


def bounce_leg(ctx, t, out, steps):
    """Multi-bounce injection (next = direct + gain * albedo * GI) on the 1080p frame: the
    frame's radiance as the direct light, a constant albedo, its GI; median of `steps`
    event-timed calls; algorithmic bytes 12 + 12 + 12 read and 12 written per pixel (FP32,
    3 channels)."""
    import torch
    H, W = t["depth"].shape
    albedo = torch.full((H, W, 3), 0.6, device="cuda")
    nxt = torch.empty_like(t["radiance"])
    stream = torch.cuda.current_stream()
    fn = lambda: ctx.inject_bounce(t["radiance"], albedo, out["gi"], 0.8, out=nxt)
    fn()
    med, mn, _ = timed(fn, stream, steps)
    nbytes = W * H * 48
    gbs = nbytes / (med * 1e-3) / 1e9
    return {"workload": f"{W}x{H}, FP32 3-channel direct light and albedo, FP32 GI", "ms": med, "ms_min": mn,
            "algorithmic_bytes": nbytes, "achieved_gbs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}


def sequence_leg(ctx, t, c, p, steps):
    """Frame sequences on the 1080p frame (multi-bounce feedback through the library's own
    light buffer, gain 0.8 on a constant albedo, the seed advanced per frame): median of
    `steps` event-timed steps (injection, gather on the new light, copy of the GI), beside
    the same frame's gather alone."""
    import torch
    from paper_2301_11376_amd import Sequence
    H, W = t["depth"].shape
    albedo = torch.full((H, W, 3), 0.6, device="cuda")
    out = {"ao": torch.empty((H, W), device="cuda"), "gi": torch.empty((H, W, 3), device="cuda"),
           "ambient": torch.empty((H, W, 3), device="cuda")}
    stream = torch.cuda.current_stream()
    seq = Sequence(ctx, W, H)
    try:
        fn = lambda: seq.step(t["depth"], t["normal"], t["radiance"], albedo, c, p, 0.8, out=out)
        fn()
        med, mn, _ = timed(fn, stream, steps)
        frames = seq.frame
    finally:
        torch.cuda.synchronize()
        seq.close()
    gather = lambda: ctx.compute(t["depth"], t["normal"], t["radiance"], c, p, out=out)
    g_med = timed(gather, stream, steps)[0]
    return {"workload": f"{W}x{H}, FP32 light buffer, gain 0.8, constant albedo 0.6, {frames} frames",
            "ms_per_step": med, "ms_min": mn, "gather_ms": g_med, "overhead_vs_gather": med / g_med - 1.0}


def sectors_leg(ctx, t, c, p):
    """The headline frame with 128 visibility sectors against 32 (Section 4.1 reports a
    5-10 % overhead for 128 on its GPU); median of 20 launches each."""
    import dataclasses
    import torch
    H, W = t["depth"].shape
    out = {"ao": torch.empty((H, W), device="cuda"), "gi": torch.empty((H, W, 3), device="cuda"),
           "ambient": torch.empty((H, W, 3), device="cuda")}
    stream = torch.cuda.current_stream()
    ms = {}
    for nb in (32, 128):
        q = dataclasses.replace(p, sectors=nb)
        fn = lambda: ctx.compute(t["depth"], t["normal"], t["radiance"], c, q, out=out)
        fn()
        ms[nb] = timed(fn, stream, 20)[0]
    return {"ms_32": ms[32], "ms_128": ms[128], "overhead": ms[128] / ms[32] - 1.0,
            "paper_overhead": "5-10 % (Section 4.1, its GPU)"}


def serve_leg(ctx, pool, n_requests, rates):
    """Poisson stream through the request loop; G-buffers device-resident in a pool, the
    loop stages each request into its 64 GB arena and copies results to the request's
    output buffers."""
    import torch
    from gbuffer_scene import request_stream, as_format
    from paper_2301_11376_amd import Camera, Context, Params, Server, NOISE_NAMES
    reqs = request_stream(n_requests=n_requests)
    dev = torch.device("cuda:0")
    gbs = {}
    for r in reqs:
        k = (r["scene_seed"], r["width"], r["height"], r["fp16"])
        if k not in gbs:
            gb = as_format(pool[k[:3]][0], r["fp16"])
            gbs[k] = {n: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for n, v in gb.items()}
    cams = {}
    prm = []
    for r in reqs:
        if (r["width"], r["height"]) not in cams:
            cams[(r["width"], r["height"])] = camera_of(Camera, r["width"], r["height"])
        prm.append(to_params(Params, NOISE_NAMES, r, pool[(r["scene_seed"], r["width"], r["height"])][1]))
    free_out = {}

    def get_out(W, H):
        lst = free_out.setdefault((W, H), [])
        return lst.pop() if lst else Context.alloc_outputs(H, W, 1, dev)

    def args(i):
        r = reqs[i]
        g = gbs[(r["scene_seed"], r["width"], r["height"], r["fp16"])]
        return g, cams[(r["width"], r["height"])], prm[i]

    # plain launches of the same mix, back to back on one stream (no staging)
    stream = torch.cuda.current_stream()
    n_sat = min(300, len(reqs))
    plain_out = {}  # one output set per resolution: the launches are ordered on one stream
    outs = [plain_out.setdefault((reqs[i]["width"], reqs[i]["height"]),
                                 get_out(reqs[i]["width"], reqs[i]["height"])) for i in range(n_sat)]

    def plain():
        for i in range(n_sat):
            g, c, p = args(i)
            ctx.compute(g["depth"], g["normal"], g["radiance"], c, p, out=outs[i])
    plain()
    torch.cuda.synchronize()
    t_plain, _, _ = timed(plain, stream, 3)
    for key, o in plain_out.items():
        free_out[key].append(o)
    plain_fps = n_sat / (t_plain * 1e-3)

    srv = Server(ctx, SERVE_BUDGET, streams=SERVE_STREAMS)
    try:
        def run(schedule, count):
            """Submit requests 0..count-1 at host times `schedule` (s, relative); returns
            latencies (ms) in request order and the wall time."""
            pend, lat = {}, [None] * count
            t0 = time.perf_counter()
            i = 0
            while i < count or pend:
                now = time.perf_counter() - t0
                while i < count and schedule[i] <= now:
                    g, c, p = args(i)
                    o = get_out(c.width, c.height)
                    tk = srv.submit(g["depth"], g["normal"], g["radiance"], c, p, o)
                    pend[tk] = (i, o, (c.width, c.height))
                    i += 1
                    now = time.perf_counter() - t0
                for tk in list(pend):
                    done, lt = srv.poll(tk)
                    if done:
                        j, o, key = pend.pop(tk)
                        lat[j] = lt
                        srv.release(tk)
                        free_out[key].append(o)
                if i < count:
                    wait = schedule[i] - (time.perf_counter() - t0)
                    if wait > 0.0005:
                        time.sleep(min(wait - 0.0003, 0.002))
                else:
                    time.sleep(0.0002)
            return lat, time.perf_counter() - t0

        # saturated: the first n_sat requests submitted at once
        run([0.0] * n_sat, n_sat)  # warm-up (graphs, output buffers)
        _, wall_sat = run([0.0] * n_sat, n_sat)
        sat_fps = n_sat / wall_sat
        print(f"serve: plain {plain_fps:.1f} frames/s, saturated served {sat_fps:.1f} frames/s",
              file=sys.stderr, flush=True)
        results = []
        for frac in rates:
            lam = frac * sat_fps
            sched = np.cumsum([r["gap"] for r in reqs]) / lam
            sched -= sched[0]
            st0 = srv.stats()
            lat, wall = run(list(sched), len(reqs))
            st = srv.stats()
            first = 200 if len(lat) > 400 else 0
            keep = np.array(lat[first:])
            samples = sum(samples_of(r) for r in reqs)
            # where the tail comes from: latency per resolution (a large frame's own work
            # against small frames waiting behind it)
            by_res = {}
            for r, lt in zip(reqs[first:], lat[first:]):
                by_res.setdefault(f"{r['width']}x{r['height']}", []).append(lt)
            by_res = {k: {"n": len(v), "p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99))}
                      for k, v in sorted(by_res.items(), key=lambda kv: int(kv[0].split("x")[0]))}
            res = {"rate_fraction_of_saturated": frac, "rate_hz": lam, "requests": len(reqs),
                   "discarded_warmup": len(reqs) - len(keep), "p50_ms": float(np.percentile(keep, 50)),
                   "p99_ms": float(np.percentile(keep, 99)), "mean_ms": float(keep.mean()),
                   "frames_per_s": len(reqs) / wall, "gsamples_s": samples / wall / 1e9,
                   "rounds": st["rounds"] - st0["rounds"],
                   "frames_per_round": (st["frames_in_rounds"] - st0["frames_in_rounds"]) /
                                       max(1, st["rounds"] - st0["rounds"]),
                   "admitted_while_running": st["admitted_while_running"] - st0["admitted_while_running"],
                   "max_running_rounds": st["max_running_rounds"], "arena_peak_bytes": st["arena_peak"],
                   "by_resolution": by_res}
            print(f"serve at {frac:.2f} x saturated ({lam:.1f}/s): p50 {res['p50_ms']:.2f} ms, "
                  f"p99 {res['p99_ms']:.2f} ms, {res['frames_per_s']:.1f} frames/s", file=sys.stderr, flush=True)
            results.append(res)
    finally:
        srv.close()
    head = next((r for r in results if abs(r["rate_fraction_of_saturated"] - 0.7) < 1e-9), results[0])
    return {"workload": f"Poisson stream of {len(reqs)} requests (first 200 discarded), resolution uniform over "
                        "960x540 / 1280x720 / 1920x1080 / 2560x1440 / 3840x2160, slices 2..8, steps {8,16,32}, "
                        "FP16 or FP32 normals+radiance (p = 1/2), radius 3, t 0.5, R2 noise, 2 procedural scenes "
                        f"per resolution, draw seed 5; G-buffers device-resident, 64 GB HBM budget, {SERVE_STREAMS} stream(s)",
            "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "frames_per_s": head["frames_per_s"],
            "rate_hz": head["rate_hz"], "saturated_frames_per_s": sat_fps,
            "plain_frames_per_s": plain_fps, "served_vs_plain": sat_fps / plain_fps, "rates": results}


def frame_leg(ctx, name, gb, cam, w, scene, steps, warmup, own_noise=True, tune=False):
    """One workload's frame, inputs resident in HBM: `warmup` untimed launches, then `steps`
    launches timed by the host clock around the loop (ms/frame, Gsamples/s) and by HIP
    events on the stream the kernels run on (the gather kernel's duration, the roofline).
    With `tune` the library's autotuner first picks the frame class's launch shape (untimed),
    else the context's default shape runs."""
    import torch
    from paper_2301_11376_amd import Camera, Params, NOISE_NAMES
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in gb.items()}
    H, W = gb["depth"].shape
    out = {"ao": torch.empty((H, W), device=dev), "gi": torch.empty((H, W, 3), device=dev),
           "ambient": torch.empty((H, W, 3), device=dev)}
    c = Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, tuple(cam.view_to_world))
    p = Params(slices=w["slices"], steps=w["steps"], radius=w["radius"], thickness=w["thickness"],
               noise=NOISE_NAMES[w["noise"]], seed=w["seed"],
               ambient_sh=tuple(float(v) for v in scene.ambient_sh.reshape(-1)))
    stream = torch.cuda.current_stream()
    tuned_ms = None
    if tune:
        _, tuned_ms = ctx.autotune(t["depth"], t["normal"], t["radiance"], c, p, out)
        torch.cuda.synchronize()
    shape = ctx.get_launch(c, p, 3 if w["fp16"] else 0)
    for _ in range(warmup):
        ctx.compute(t["depth"], t["normal"], t["radiance"], c, p, out=out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        ctx.compute(t["depth"], t["normal"], t["radiance"], c, p, out=out)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_launch_ms = np.array([a.elapsed_time(b) for a, b in ev])
    ms = wall * 1e3 / steps
    samples, abytes = algorithmic_bytes(W, H, w["slices"], w["steps"], w["fp16"])
    kernel_ms = float(per_launch_ms.mean())
    achieved = abytes / (kernel_ms * 1e-3) / 1e9
    floor_bytes = W * H * ((4 + 6 + 6 if w["fp16"] else 4 + 12 + 12) + 28)
    print(f"{name}: timed {steps} steps: {ms:.3f} ms/frame wall, kernel mean {kernel_ms:.3f} ms "
          f"(p50 {np.percentile(per_launch_ms, 50):.3f}, p99 {np.percentile(per_launch_ms, 99):.3f})",
          file=sys.stderr, flush=True)
    res = {
        "workload": f"{name}: {W}x{H}, {w['slices']} slices x {w['steps']} steps per side, N_b 32, radius "
                    f"{w['radius']}, thickness {w['thickness']:.4g}, noise {w['noise']}, "
                    f"{'FP16' if w['fp16'] else 'FP32'} normals and radiance, procedural scene seed {w['seed']} "
                    f"({w['n_boxes']} boxes, {w['n_planes']} thin planes)",
        "samples_per_frame": samples, "pixels": W * H, "ms_per_frame": ms,
        "gsamples_s": samples / (ms * 1e-3) / 1e9, "steps": steps, "warmup": warmup,
        "kernel_ms": {"mean": kernel_ms, "p50": float(np.percentile(per_launch_ms, 50)),
                      "p90": float(np.percentile(per_launch_ms, 90)),
                      "p99": float(np.percentile(per_launch_ms, 99)), "min": float(per_launch_ms.min())},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(name, shape) if own_noise else None,
                     "traffic_unit": "B per launch", "algorithmic_bytes_per_launch": abytes,
                     "bytes_per_sample": 16 if w["fp16"] else 28, "bytes_per_pixel": 38 if w["fp16"] else 44,
                     "launch_shape": list(shape), "launch_shape_source": "autotuned" if tune else "default",
                     "autotune_best_ms": tuned_ms, "compulsory_floor_bytes": floor_bytes,
                     "compulsory_floor_ms": floor_bytes / (HBM_PEAK_GBS * 1e9) * 1e3},
    }
    return res, (t, c, p, out)


def run_leg(into, key, fn, *a, say=None, **k):
    """Run one leg after the headline into `into[key]`.  A Python-level failure (an exception
    from the leg, a status the library returned) is printed with its traceback and
    recorded as {"error": ...} under the key, so the measurements already taken still reach
    the JSON line; a device fault still ends the process.  `say` formats a progress line
    from the leg's result."""
    try:
        r = fn(*a, **k)
    except Exception as e:
        traceback.print_exc(file=sys.stderr)
        into[key] = {"error": f"{type(e).__name__}: {e}"}
        return None
    into[key] = r
    if say is not None:
        print(say(r), file=sys.stderr, flush=True)
    return r


def slice_order_leg(ctx, tensors, chunks, steps, warmup=3):
    """The same frame in slice-major order, once per chunk size in `chunks` (tiles; both
    kernels, the per-slice gather and the reduction, inside the timed region), against the
    default order timed the same way just before; the outputs of each run compared with the
    default order's (AO bit for bit, GI and ambient max |difference|)."""
    import torch
    t, c, p, out = tensors
    stream = torch.cuda.current_stream()

    def timed():
        for _ in range(warmup):
            ctx.compute(t["depth"], t["normal"], t["radiance"], c, p, out=out)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            ctx.compute(t["depth"], t["normal"], t["radiance"], c, p, out=out)
            b.record(stream)
        torch.cuda.synchronize()
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        return float(ms.mean()), float(np.percentile(ms, 50)), {k: v.clone() for k, v in out.items()}

    base_ms, base_p50, base = timed()
    res = {"default_order_ms": base_ms, "default_order_p50_ms": base_p50, "chunks": []}
    try:
        for chunk in chunks:
            ctx.set_slice_order(chunk)
            ms, p50, got = timed()
            r = {"chunk_tiles": chunk, "ms": ms, "p50_ms": p50, "speedup": base_ms / ms,
                 "ao_equal": bool(torch.equal(got["ao"], base["ao"])),
                 "gi_max_diff": float((got["gi"] - base["gi"]).abs().max()),
                 "ambient_max_diff": float((got["ambient"] - base["ambient"]).abs().max())}
            res["chunks"].append(r)
            print(f"slice order (chunk {chunk}): {ms:.3f} ms vs default order {base_ms:.3f} ms, AO equal "
                  f"{r['ao_equal']}, GI max diff {r['gi_max_diff']:.2e}", file=sys.stderr, flush=True)
    finally:
        ctx.set_slice_order(0)
    return res


def parity_leg(ctx, name, tensors, ref):
    """The workload's frame once more with slice masks, compared with the oracle's outputs
    from the cpu_baseline leg (the rows it computed)."""
    import torch
    t, c, p, _ = tensors
    o = ctx.compute(t["depth"], t["normal"], t["radiance"], c, p, masks=True)
    torch.cuda.synchronize()
    r0, r1 = ref["rows"]
    gpu = {k: v[r0:r1].cpu().numpy() for k, v in o.items()}
    del o
    rep = {"rows": [r0, r1], "vs_oracle_same_inputs": error_report(gpu, ref["fp"])}
    if "fp32_originals" in ref:
        rep["vs_oracle_fp32_originals"] = error_report(gpu, ref["fp32_originals"], masks=False)
    e = rep["vs_oracle_same_inputs"]
    print(f"parity {name}: masks {e['mask_agreement']:.6f}, max |err| AO {e['ao']['max']:.2e} "
          f"GI {e['gi']['max']:.2e} ambient {e['ambient']['max']:.2e}", file=sys.stderr, flush=True)
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2_1080p")
    ap.add_argument("--noise", choices=["hash", "r2", "fixed"], default=None,
                    help="replace the workload's noise (fixed: every pixel the same slice directions and "
                         "offsets, which shows what the per-pixel decorrelation costs in cache misses)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle: no cpu_baseline and no per-output error report")
    ap.add_argument("--no-c3", action="store_true", help="skip the 4K FP16 leg")
    ap.add_argument("--c3-steps", type=int, default=10)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-table2", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rates", default="0.5,0.7,0.9",
                    help="request rates as fractions of the saturated rate (p50 / p99 at each)")
    ap.add_argument("--slice-order", default="", metavar="TILES[,TILES...]",
                    help="also time the frame(s) in slice-major order over chunks of TILES tiles, once per "
                         "comma-separated size (empty: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="instead of the gather, run a plain device copy of MIB MiB (scales HBM counters)")
    args = ap.parse_args()
    args.slice_order = [int(v) for v in args.slice_order.split(",") if v.strip()]
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the gather has no multi-GPU path in this build "
              "(frames or row bands would shard with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.arange(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(args.steps, 1)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": max(args.steps, 1)}))
        return

    # ---- host work first (forked workers), before anything touches the GPU ----
    from gbuffer_scene import workload, request_stream, render_pool, render_gbuffer
    names = [args.workload]
    if args.workload == "c2_1080p" and not args.no_c3:
        names.append("c3_4k_fp16")
    if not args.no_cpu_baseline and "c1_128" not in names:
        names.insert(0, "c1_128")
    loaded = {}
    for n in names:
        gb_n, cam_n, w_n, sc_n = workload(n)
        own = w_n["noise"]
        if args.noise:
            w_n["noise"] = args.noise
        w_n["own_noise"] = own == w_n["noise"]
        extra = (render_gbuffer(sc_n, cam_n),) if w_n["fp16"] else ()  # FP32 originals
        loaded[n] = (gb_n, cam_n, w_n, sc_n) + extra
    keys = []
    if not args.no_batch:
        keys += [(f["scene_seed"], f["width"], f["height"]) for kind in BATCH_WORKLOADS for f in batch_frames(kind)]
    if not args.no_serve:
        keys += [(r["scene_seed"], r["width"], r["height"]) for r in request_stream(n_requests=args.serve_requests)]
    pool = {}
    if keys:
        t0 = time.perf_counter()
        pool = render_pool(keys, workers=min(HOST_WORKERS, os.cpu_count() or 1))
        print(f"rendered {len(pool)} pool frames in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    base, refs = None, {}
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        base, refs = cpu_baseline_leg(loaded, max(1, min(HOST_WORKERS, os.cpu_count() or 1)), names)

    # ---- GPU ----
    import torch
    from paper_2301_11376_amd import Context
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = Context(0)
    gb, cam, w, scene = loaded[args.workload][:4]
    head, tensors = frame_leg(ctx, args.workload, gb, cam, w, scene, args.steps, args.warmup, w["own_noise"])
    t, c, p, out = tensors
    copy_gbs = stream_copy_gbs()
    head["roofline"]["stream_copy_gbs"] = copy_gbs
    head["roofline"]["frac_of_stream_copy"] = head["roofline"]["achieved"] / copy_gbs
    result = {
        "metric": "Gsamples/s & ms/frame at 1080p vs HBM roofline; p50/p99 latency, mixed frames",
        "value": head["gsamples_s"],
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_frame"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" + ("+f16 normal/radiance" if w["fp16"] else ""),
        "data": "synthetic",
        "config": {"workload": head["workload"], "samples_per_frame": head["samples_per_frame"],
                   "pixels": head["pixels"], "parallelism": "single GPU",
                   "device": torch.cuda.get_device_name(dev) or torch.cuda.get_device_properties(dev).gcnArchName,
                   "hip": torch.version.hip},
        "kernel_ms": head["kernel_ms"],
        "roofline": head["roofline"],
    }
    if base is not None:
        cpu = dict(base[args.workload])
        cpu["gpu_speedup"] = result["value"] / cpu["value"]
        cpu["cpu_model"] = cpu_model()
        cpu["host_cpus"] = os.cpu_count()
        cpu["workloads"] = base
        result["cpu_baseline"] = cpu
    if args.slice_order:
        result["slice_order"] = {}
        run_leg(result["slice_order"], args.workload, slice_order_leg, ctx, tensors, args.slice_order, args.steps)
    parity = {}
    if args.workload in refs:
        run_leg(parity, args.workload, parity_leg, ctx, args.workload, tensors, refs[args.workload])
    if not args.no_table2 and args.workload == "c2_1080p":
        run_leg(result, "table2", table2_leg, ctx, t, c, scene, slices=1,
                say=lambda r: "table2: " + ", ".join(f"{x['row']} {x['ms']:.3f} ms" for x in r["rows"]))
        run_leg(result, "denoise", denoise_leg, ctx, t, c, out, 20, say=lambda r: f"denoise: {r['ms']:.3f} ms")
        run_leg(result, "bounce", bounce_leg, ctx, t, out, 20,
                say=lambda r: f"bounce: {r['ms']:.3f} ms, {r['achieved_gbs']:.0f} GB/s")
        run_leg(result, "sequence", sequence_leg, ctx, t, c, p, 20,
                say=lambda r: f"sequence: {r['ms_per_step']:.3f} ms per step, gather alone {r['gather_ms']:.3f} ms")
        run_leg(result, "sectors128", sectors_leg, ctx, t, c, p,
                say=lambda r: f"sectors: 32 {r['ms_32']:.3f} ms, 128 {r['ms_128']:.3f} ms")
    del t, out, tensors
    for n in names:
        if n == args.workload:
            continue
        gb_n, cam_n, w_n, sc_n = loaded[n][:4]
        if n == "c3_4k_fp16":
            # at 4K the default shape is not the fastest (the autotuner's pick measured 4 %
            # faster), so this leg runs the shape the library's autotuner picks
            legs = {}
            run_leg(legs, n, frame_leg, ctx, n, gb_n, cam_n, w_n, sc_n, args.c3_steps, 2, w_n["own_noise"],
                    tune=not args.no_autotune)
            if isinstance(legs[n], dict):  # the leg's error record
                result[n] = legs[n]
                torch.cuda.empty_cache()
                continue
            result[n], tens = legs[n]
            if args.slice_order:
                run_leg(result.setdefault("slice_order", {}), n, slice_order_leg, ctx, tens, args.slice_order,
                        args.c3_steps)
        else:
            from paper_2301_11376_amd import Camera, Params, NOISE_NAMES
            tt = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in gb_n.items()}
            cc = Camera(cam_n.width, cam_n.height, cam_n.fx, cam_n.fy, cam_n.cx, cam_n.cy,
                        tuple(cam_n.view_to_world))
            pp = Params(slices=w_n["slices"], steps=w_n["steps"], radius=w_n["radius"],
                        thickness=w_n["thickness"], noise=NOISE_NAMES[w_n["noise"]], seed=w_n["seed"],
                        ambient_sh=tuple(float(v) for v in sc_n.ambient_sh.reshape(-1)))
            tens = (tt, cc, pp, None)
        if n in refs:
            run_leg(parity, n, parity_leg, ctx, n, tens, refs[n])
        del tens
        torch.cuda.empty_cache()
    if parity:
        result["parity"] = parity
    if not args.no_batch:
        run_leg(result, "batch", batch_leg, ctx, pool, autotune=not args.no_autotune)
        run_leg(result, "batch_small", batch_leg, ctx, pool, autotune=not args.no_autotune, kind="small")
    if not args.no_serve:
        rates = [float(x) for x in args.serve_rates.split(",") if x.strip()]
        run_leg(result, "serving", serve_leg, ctx, pool, args.serve_requests, rates)
    run_leg({}, "close", ctx.close)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
