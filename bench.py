"""Benchmark of the visibility-bitmask gather on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2_1080p]

One step = one pass of the whole hot path (ssvb_compute: AO, GI and ambient of one
frame) over a seeded synthetic 1920x1080 G-buffer already resident in HBM.  Prints one
JSON line with Gsamples/s (a sample is one depth fetch of one pixel, slice, side and
step: px * N_d * 2 * N_s per frame), ms per frame, the roofline of the gather kernel
and the FP64 oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def algorithmic_bytes(W, H, nd, ns, fp16):
    """Bytes the method itself moves per frame: every sample reads depth + normal +
    radiance (28 B, or 16 B with FP16 normal and radiance), every pixel reads its own
    depth + normal and writes AO + GI + ambient (44 B, or 38 B)."""
    px = W * H
    samples = px * nd * 2 * ns
    per_sample = 16 if fp16 else 28
    per_px = 38 if fp16 else 44
    return samples, samples * per_sample + px * per_px


def device_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in ("ssvb_kernels.hip", "ssvb_internal.h"):
        with open(os.path.join(ROOT, "paper_2301_11376_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE passes
    (scaled by the copy calibration), or None when the device code has changed since."""
    path = os.path.join(ROOT, "profiles", f"gather_plain_{workload_name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("device_source_sha256") != device_source_sha256() or rec.get("workload") != workload_name:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(gb, cam, kw):
    """The FP64 oracle, as it stands, on a 128-row band of the frame (single process)."""
    import oracle as O
    H, W = gb["depth"].shape
    rows = min(128, H)
    y0 = (H - rows) // 2
    ys = np.repeat(np.arange(y0, y0 + rows), W)
    xs = np.tile(np.arange(W), rows)
    oc = O.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, tuple(cam.view_to_world))
    t0 = time.perf_counter()
    O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, O.Params(**kw), pixels=(ys, xs))
    dt = time.perf_counter() - t0
    samples = len(ys) * kw["slices"] * 2 * kw["steps"]
    return {"value": samples / dt / 1e9, "unit": "Gsamples/s", "cores": 1, "kind": "oracle",
            "sample": f"rows {y0}..{y0 + rows - 1} of the same frame ({len(ys)} px, {samples} samples), "
                      f"{dt:.1f} s single-threaded NumPy FP64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2_1080p")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="instead of the gather, run a plain device copy of MIB MiB (scales HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the gather has no multi-GPU path in this build "
              "(frames or row bands would shard with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.arange(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(args.steps, 1)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": max(args.steps, 1)}))
        return
    from gbuffer_scene import workload
    from paper_2301_11376_amd import Camera, Context, Params, NOISE_NAMES

    gb, cam, w, scene = workload(args.workload)
    kw = dict(slices=w["slices"], steps=w["steps"], radius=w["radius"], thickness=w["thickness"],
              noise=NOISE_NAMES[w["noise"]], seed=w["seed"], ambient_sh=tuple(float(v) for v in scene.ambient_sh.reshape(-1)))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in gb.items()}
    H, W = gb["depth"].shape
    out = {"ao": torch.empty((H, W), device=dev), "gi": torch.empty((H, W, 3), device=dev),
           "ambient": torch.empty((H, W, 3), device=dev)}
    ctx = Context(0)
    c = Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, tuple(cam.view_to_world))
    p = Params(**kw)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        ctx.compute(t["depth"], t["normal"], t["radiance"], c, p, out=out)
    torch.cuda.synchronize()
    print(f"warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        ctx.compute(t["depth"], t["normal"], t["radiance"], c, p, out=out)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_launch_ms = np.array([a.elapsed_time(b) for a, b in ev])
    ms = wall * 1e3 / args.steps
    samples, abytes = algorithmic_bytes(W, H, kw["slices"], kw["steps"], w["fp16"])
    kernel_ms = float(per_launch_ms.mean())
    achieved = abytes / (kernel_ms * 1e-3) / 1e9
    print(f"timed {args.steps} steps: {ms:.3f} ms/frame wall, kernel mean {kernel_ms:.3f} ms "
          f"(p50 {np.percentile(per_launch_ms, 50):.3f}, p99 {np.percentile(per_launch_ms, 99):.3f})",
          file=sys.stderr, flush=True)

    result = {
        "metric": "Gsamples/s & ms/frame at 1080p vs HBM roofline; p50/p99 latency, mixed frames",
        "value": samples / (ms * 1e-3) / 1e9,
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" + ("+f16 normal/radiance" if w["fp16"] else ""),
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {W}x{H}, {kw['slices']} slices x {kw['steps']} steps per side, "
                               f"N_b 32, radius {kw['radius']}, thickness {kw['thickness']:.4g}, noise {w['noise']}, "
                               f"procedural scene seed {w['seed']} ({w['n_boxes']} boxes, {w['n_planes']} thin planes)",
                   "samples_per_frame": samples, "pixels": W * H, "parallelism": "single GPU"},
        "kernel_ms": {"mean": kernel_ms, "p50": float(np.percentile(per_launch_ms, 50)),
                      "p99": float(np.percentile(per_launch_ms, 99)), "min": float(per_launch_ms.min())},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload), "traffic_unit": "B per launch",
                     "algorithmic_bytes_per_launch": abytes},
    }
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(gb, cam, kw)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
