"""Helpers shared by the parity tests: run the HIP path (or the host build of its per-pixel
code) and the oracle on the same seeded inputs, compare element by element and trace every
mismatch.

The bar: sector masks exact on >= 99.9 % of pixels, every mismatch explained by endpoints
within 1e-6 rad of a rounding boundary; AO, GI and ambient within 1e-3 absolute for FP32
inputs (the oracle reads the same FP32 / FP16 values the GPU reads, upcast exactly).  The
tracer (explain_pixel) replays a mismatched pixel in the oracle with near-tie roundings
flipped: a floor or ceiling argument just off an integer crosses it; one exactly on it
drops under a floor and rises under a ceiling (PSEUDOCODE's width).  Up to 10 near ties
every combination is replayed; with more, each mismatched slice is searched on its own for
flips whose sector sets OR to the device's slice mask, and the oracle replays the
candidates.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

import oracle as O
from gbuffer_scene import make_camera, make_scene, render_gbuffer

TOL_FP32 = 1e-3
MASK_AGREEMENT = 0.999
TIE_RAD = 1e-6                       # a mismatch must come from an endpoint this close


def tie_sectors(nb):
    """TIE_RAD in sector units of an N_b-sector mask."""
    return TIE_RAD * nb / math.pi


def packed_masks(m):
    """Oracle masks as the GPU stores them: uint32 [n, N_d] for N_b = 32 already; for more
    sectors a bool [n, N_d, N_b] array becomes [n, N_d * N_b / 32] words, sector k in bit
    k % 32 of word k / 32."""
    m = np.asarray(m)
    if m.dtype != bool:
        return m
    n, nd, nb = m.shape
    w = m.reshape(n, nd, nb // 32, 32).astype(np.uint64) << np.arange(32, dtype=np.uint64)
    return w.sum(axis=-1).astype(np.uint32).reshape(n, nd * (nb // 32))


def cams(cam):
    """(binding Camera, oracle Camera) of a gbuffer_scene CameraSpec."""
    from paper_2301_11376_amd import Camera
    return (Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, tuple(cam.view_to_world)),
            O.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, tuple(cam.view_to_world)))


def params(**kw):
    """(binding Params, oracle Params) with identical values."""
    from paper_2301_11376_amd import Params
    return Params(**kw), O.Params(**kw)


def to_device(gb, device="cuda"):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in gb.items()}


def gpu_run(ctx, gb, cam, prm, masks=True):
    import torch
    t = to_device(gb)
    out = ctx.compute(t["depth"], t["normal"], t["radiance"], cam, prm, masks=masks)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    if masks:
        res["masks"] = res["masks"].view(np.uint32)
    return res


def compare(gpu, ref, gb, ocam, oprm, pixels=None, tol=TOL_FP32, report=None, agreement=MASK_AGREEMENT,
            max_bad=200):
    """Compare GPU outputs with the oracle's; explain every mismatch by flipping near-tie
    roundings in an FP64 replay.  ``gpu`` holds full images, ``ref`` the oracle results at
    ``pixels`` (or full images).  At most ``max_bad`` pixels may differ and the masks must
    agree on at least ``agreement`` of them.  Returns a stats dict; raises AssertionError
    on failure."""
    if pixels is None:
        H, W = gb["depth"].shape
        ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        ys, xs = ys.reshape(-1), xs.reshape(-1)
        flat = lambda a: a.reshape((H * W,) + a.shape[2:])
        ref = {k: flat(v) for k, v in ref.items() if k in ("ao", "gi", "ambient", "masks", "valid")}
    else:
        ys, xs = pixels
    if "masks" in ref:
        ref = dict(ref, masks=packed_masks(ref["masks"]))
    g = {k: gpu[k][ys, xs] for k in ("ao", "gi", "ambient", "masks") if k in gpu}
    mask_eq = np.all(g["masks"] == ref["masks"], axis=-1) if "masks" in g else np.ones(len(ys), bool)
    err_ao = np.abs(g["ao"] - ref["ao"])
    err_gi = np.abs(g["gi"] - ref["gi"]).max(axis=-1)
    err_amb = np.abs(g["ambient"] - ref["ambient"]).max(axis=-1)
    bad = ~mask_eq | (err_ao > tol) | (err_gi > tol) | (err_amb > tol)
    stats = {
        "pixels": int(len(ys)),
        "mask_agreement": float(mask_eq.mean()),
        "mismatched_pixels": int(bad.sum()),
        "max_err": {"ao": float(err_ao.max(initial=0)), "gi": float(err_gi.max(initial=0)),
                    "ambient": float(err_amb.max(initial=0))},
        "mean_err": {"ao": float(err_ao.mean()), "gi": float(err_gi.mean()), "ambient": float(err_amb.mean())},
        "p99_err": {"ao": float(np.percentile(err_ao, 99)), "gi": float(np.percentile(err_gi, 99)),
                    "ambient": float(np.percentile(err_amb, 99))},
        "explained": 0,
    }
    unexplained = []
    for idx in np.flatnonzero(bad)[:max_bad]:
        if explain_pixel(gpu, gb, ocam, oprm, int(ys[idx]), int(xs[idx]), tol):
            stats["explained"] += 1
        else:
            unexplained.append((int(ys[idx]), int(xs[idx])))
    if report is not None:
        report.update(stats)
    assert bad.sum() <= max_bad, f"{bad.sum()} mismatched pixels: {stats}"
    assert not unexplained, f"unexplained mismatches at {unexplained[:10]}: {stats}"
    assert stats["mask_agreement"] >= agreement, stats
    return stats


def _flip(v, ceil):
    """Bias that moves the rounding of an endpoint argument ``v`` across its nearest integer:
    +1 below it, -1 above it; exactly on it, a floor drops (-1) and a ceiling rises (+1)."""
    r = np.round(v)
    if v != r:
        return 1 if v < r else -1
    return 1 if ceil else -1


def _near_ties(ep, oprm):
    """Near-tie endpoints of one pixel: a list of (index into ``ep``, bias).  A sector start
    exactly at 0 has no flip: an angle past the hemisphere edge is clamped back onto it."""
    pseudo = oprm.hit_criterion != O.ROUND
    dist = np.abs(ep - np.round(ep))
    out = []
    for pos in np.argwhere(np.isfinite(ep) & (dist < tie_sectors(oprm.sectors))):
        pos = tuple(int(p) for p in pos)
        v = ep[pos]
        f = _flip(v, pseudo and pos[-1] == 1)
        if pos[-1] == 0 and v == 0.0 and f < 0:
            continue
        out.append((pos, f))
    return out


def _replay(gpu, gb, ocam, oprm, y, x, bias, tol):
    """The oracle at pixel (y, x) with rounding biases: does it give the GPU's masks and
    outputs within ``tol``?"""
    rr = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam, oprm, pixels=([y], [x]),
                   return_masks=True, index_bias=bias[None])
    if not np.array_equal(packed_masks(rr["masks"])[0], gpu["masks"][y, x]):
        return False
    return bool(abs(rr["ao"][0] - gpu["ao"][y, x]) <= tol and np.abs(rr["gi"][0] - gpu["gi"][y, x]).max() <= tol
                and np.abs(rr["ambient"][0] - gpu["ambient"][y, x]).max() <= tol)


def _sample_bits(e, d, nb, pseudo):
    """Sector set (an int bit mask) of one sample from its endpoint arguments ``e`` and
    rounding biases ``d``: [floor, floor) under ROUND; start floor and width ceil under
    PSEUDOCODE.  Used only to steer the search; every candidate is replayed by the oracle."""
    a = math.floor(e[0]) + d[0]
    b = min(a + math.ceil(e[1]) + d[1], nb) if pseudo else math.floor(e[1]) + d[1]
    a, b = max(a, 0), min(b, nb)
    return ((1 << b) - (1 << a)) if b > a else 0


def _slice_solutions(ep_i, ties, target, nb, pseudo, limit=16):
    """Up to ``limit`` bias choices for one slice whose sample sets OR to ``target``: a
    depth-first search over the samples in march order (side +, then -, steps in order),
    each keeping its rounding or taking flips of its own near-tie endpoints, fewest flips
    first.  Returns a list of {(side, step): (bias0, bias1)}."""
    order = [(s, j) for s in range(ep_i.shape[0]) for j in range(ep_i.shape[1])]
    alts = []
    for s, j in order:
        e = ep_i[s, j]
        if not np.all(np.isfinite(e)):
            alts.append([((0, 0), 0)])
            continue
        t = ties.get((s, j), {})
        opts = {}
        for f0 in ((0,) if 0 not in t else (0, t[0])):
            for f1 in ((0,) if 1 not in t else (0, t[1])):
                bits = _sample_bits(e, (f0, f1), nb, pseudo)
                if bits & ~target:
                    continue
                if bits not in opts or abs(f0) + abs(f1) < sum(map(abs, opts[bits])):
                    opts[bits] = (f0, f1)
        alts.append(sorted(((d, b) for b, d in opts.items()), key=lambda db: sum(map(abs, db[0]))))
    suffix = [0] * (len(order) + 1)
    for k in range(len(order) - 1, -1, -1):
        suffix[k] = suffix[k + 1]
        for _, b in alts[k]:
            suffix[k] |= b
    out, dead, path = [], set(), []

    def dfs(k, covered):
        if len(out) >= limit:
            return True
        if (covered | suffix[k]) & target != target or (k, covered) in dead:
            return False
        if k == len(order):
            if covered == target:
                out.append({order[i]: d for i, d in enumerate(path) if d != (0, 0)})
                return True
            return False
        found = False
        for d, b in alts[k]:
            path.append(d)
            found |= dfs(k + 1, covered | b)
            path.pop()
            if len(out) >= limit:
                return True
        if not found:
            dead.add((k, covered))
        return found

    dfs(0, 0)
    return out


def explain_pixel(gpu, gb, ocam, oprm, y, x, tol):
    """Replay pixel (y, x) in FP64 with flipped near-tie roundings; True if one choice
    reproduces the GPU's masks exactly and its outputs within ``tol``.  Up to 10 near
    ties every combination is tried; beyond that (whole rows of samples exactly on a
    hemisphere edge) each mismatched slice is searched on its own for flips whose sector
    sets OR to the GPU's slice mask, and the candidates are replayed."""
    r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam, oprm, pixels=([y], [x]),
                  return_masks=True, return_endpoints=True)
    ep = r["endpoints"][0]
    near = _near_ties(ep, oprm)
    if not near:
        return False
    if len(near) <= 10:
        for flips in itertools.product((0, 1), repeat=len(near)):
            if not any(flips):
                continue
            bias = np.zeros(ep.shape, dtype=np.int64)
            for f, (pos, d) in zip(flips, near):
                if f:
                    bias[pos] = d
            if _replay(gpu, gb, ocam, oprm, y, x, bias, tol):
                return True
        return False
    nb, pseudo = oprm.sectors, oprm.hit_criterion != O.ROUND
    wpc = nb // 32
    mine = packed_masks(r["masks"])[0]
    theirs = gpu["masks"][y, x]
    per_slice = []
    for i in range(ep.shape[0]):
        if np.array_equal(mine[i * wpc:(i + 1) * wpc], theirs[i * wpc:(i + 1) * wpc]):
            continue
        target = sum(int(w) << (32 * k) for k, w in enumerate(theirs[i * wpc:(i + 1) * wpc]))
        ties = {}
        for pos, d in near:
            if pos[0] == i:
                ties.setdefault((pos[1], pos[2]), {})[pos[3]] = d
        sols = _slice_solutions(ep[i], ties, target, nb, pseudo)
        if not sols:
            return False
        per_slice.append((i, sols))
    if not per_slice:
        return False

    def bias_of(choice):
        bias = np.zeros(ep.shape, dtype=np.int64)
        for (i, sols), c in zip(per_slice, choice):
            for (s, j), (d0, d1) in sols[c].items():
                bias[i, s, j] = (d0, d1)
        return bias

    base = [0] * len(per_slice)
    if _replay(gpu, gb, ocam, oprm, y, x, bias_of(base), tol):
        return True
    for k, (_, sols) in enumerate(per_slice):
        for c in range(1, len(sols)):
            choice = list(base)
            choice[k] = c
            if _replay(gpu, gb, ocam, oprm, y, x, bias_of(choice), tol):
                return True
    return False


def sample_pixels(H, W, n, seed):
    """A seeded sample of pixels: random ones plus the four corners and the last row
    and column (ragged tails)."""
    rng = np.random.default_rng(seed)
    ys = rng.integers(0, H, n)
    xs = rng.integers(0, W, n)
    extra_y = np.array([0, 0, H - 1, H - 1] + [H - 1] * 8 + list(rng.integers(0, H, 8)))
    extra_x = np.array([0, W - 1, 0, W - 1] + list(rng.integers(0, W, 8)) + [W - 1] * 8)
    return np.concatenate([ys, extra_y]), np.concatenate([xs, extra_x])


# ----------------------------------------------------------------------------------------
# cases shared by the GPU parity tests and the CPU tests of the host build of the kernels
# ----------------------------------------------------------------------------------------
INF = float("inf")
_SCENES = {}


def tiny(width=64, height=48, fp16=False, channels=3, seed=7):
    key = (width, height, fp16, channels, seed)
    if key not in _SCENES:
        sc = make_scene(seed, 40, 20)
        cam = make_camera(width, height, fov_y_deg=60, pitch_deg=-25)
        dt = np.float16 if fp16 else np.float32
        gb = render_gbuffer(sc, cam, normal_dtype=dt, radiance_dtype=dt, channels=channels, cache=False)
        _SCENES[key] = (gb, cam, sc)
    return _SCENES[key]


VARIANTS = {
    "hash_t04": dict(slices=3, steps=6, radius=1.2, thickness=0.4, noise=O.NOISE_HASH, seed=11),
    "r2_tinf": dict(slices=4, steps=10, radius=2.5, thickness=INF, noise=O.NOISE_R2, seed=12),
    "fixed_thin": dict(slices=2, steps=9, radius=0.8, thickness=0.05, noise=O.NOISE_FIXED),
    "slope": dict(slices=2, steps=7, radius=1.5, thickness=0.1, thickness_slope=0.05, noise=O.NOISE_HASH, seed=13),
    "pseudocode": dict(slices=3, steps=6, radius=1.5, thickness=0.3, noise=O.NOISE_HASH, seed=14, hit_criterion=1),
    "one_slice_one_step": dict(slices=1, steps=1, radius=1.0, noise=O.NOISE_HASH, seed=15),
    "many_slices": dict(slices=16, steps=3, radius=1.0, noise=O.NOISE_R2, seed=16, ambient_samples=32),
    "ambient1": dict(slices=2, steps=4, radius=1.0, noise=O.NOISE_HASH, seed=17, ambient_samples=1),
    "capped_subpixel": dict(slices=2, steps=20, radius=4.0, noise=O.NOISE_HASH, seed=18, max_radius_px=6.0,
                            min_step_q4=2),
    "zero_thickness": dict(slices=2, steps=6, radius=1.5, thickness=0.0, noise=O.NOISE_HASH, seed=19),
    "quadratic_steps": dict(slices=3, steps=12, radius=2.0, thickness=0.3, noise=O.NOISE_R2, seed=20,
                            step_distribution=1),
    "sectors128": dict(slices=3, steps=8, radius=1.5, thickness=0.4, noise=O.NOISE_HASH, seed=41, sectors=128),
    "sectors128_pseudocode_tinf": dict(slices=2, steps=10, radius=2.0, thickness=INF, noise=O.NOISE_R2, seed=42,
                                       sectors=128, hit_criterion=1, ambient_samples=16),
    "sectors128_slope_quadratic": dict(slices=4, steps=6, radius=1.0, thickness=0.1, thickness_slope=0.05,
                                       noise=O.NOISE_HASH, seed=43, sectors=128, step_distribution=1,
                                       ambient_samples=32),
    "quadratic_pseudocode_tinf": dict(slices=2, steps=8, radius=1.5, thickness=INF, noise=O.NOISE_HASH, seed=21,
                                      step_distribution=1, hit_criterion=1),
    # the largest slice and step counts the library accepts
    "max_slices": dict(slices=64, steps=2, radius=1.0, thickness=0.3, noise=O.NOISE_HASH, seed=44, ambient_samples=32),
    "max_slices_128": dict(slices=64, steps=2, radius=1.0, thickness=0.3, noise=O.NOISE_R2, seed=45, sectors=128,
                           ambient_samples=32),
    "max_steps": dict(slices=1, steps=1024, radius=6.0, thickness=0.4, noise=O.NOISE_R2, seed=46, min_step_q4=1),
    "max_steps_quadratic": dict(slices=1, steps=1024, radius=6.0, thickness=INF, noise=O.NOISE_HASH, seed=47,
                                min_step_q4=1, step_distribution=1),
}


HALF_CASES = {
    "uniform": dict(slices=3, steps=6, radius=1.2, thickness=0.4, noise=O.NOISE_HASH, seed=31),
    "table2_f": dict(slices=2, steps=16, radius=4.0, thickness=0.2, noise=O.NOISE_R2, seed=32,
                     step_distribution=1),
}


# ----------------------------------------------------------------------------------------
# oracle references of the large-frame GPU parity tests
# ----------------------------------------------------------------------------------------
# Each is the oracle over row bands of a workload frame.  They are computed in forked
# processes when the test session's collection ends (tests/conftest.py), before any test
# initialises the GPU (a process that uses the GPU must not fork), and kept here; a test
# that finds none computes it in this process.
BAND_REFS = {}
C3_BAND_ROWS = 270


def band_cases():
    """name -> (G-buffer, camera, oracle params kwargs, first row, end row, masks)."""
    from gbuffer_scene import workload
    out = {}
    gb, cam, w, sc = workload("c2_1080p")
    kw = dict(slices=4, steps=16, radius=3.0, thickness=0.5, noise=O.NOISE_R2, seed=2,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    out["c2_full"] = (gb, cam, kw, 0, gb["depth"].shape[0], True)
    gb, cam, w, sc = workload("c3_4k_fp16")
    H = gb["depth"].shape[0]
    r0 = (H - C3_BAND_ROWS) // 2
    kw = dict(slices=8, steps=32, radius=8.0, thickness=w["thickness"], noise=O.NOISE_R2, seed=3,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    out["c3_band_fp16"] = (gb, cam, kw, r0, r0 + C3_BAND_ROWS, True)
    out["c3_band_fp32"] = (render_gbuffer(make_scene(3, 64, 32), cam), cam, kw, r0, r0 + C3_BAND_ROWS, False)
    return out


def compute_band_refs(names, workers, threads=False):
    """Fill BAND_REFS for `names` (the oracle over the cases' rows)."""
    import os
    import time
    from oracle.bands import compute_rows
    cases = band_cases()
    for n in names:
        if n in BAND_REFS:
            continue
        gb, cam, kw, r0, r1, masks = cases[n]
        _, oc = cams(cam)
        t0 = time.perf_counter()
        res, _, _ = compute_rows(gb, oc, O.Params(**kw), r0, r1, workers, return_masks=masks, threads=threads)
        BAND_REFS[n] = res
        print(f"oracle reference {n}: rows {r0}..{r1 - 1} in {time.perf_counter() - t0:.1f} s "
              f"({'threads' if threads else 'processes'}, {workers})", flush=True)
    return {n: BAND_REFS[n] for n in names}


def random_case(rng):
    """A seeded random frame and parameter set over the library's whole parameter space."""
    W, H = int(rng.integers(1, 41)), int(rng.integers(1, 31))
    fp16 = bool(rng.integers(2))
    ch = int(rng.choice([3, 4]))
    sc = make_scene(int(rng.integers(1000)), int(rng.integers(5, 40)), int(rng.integers(0, 20)))
    cam = make_camera(W, H, fov_y_deg=float(rng.uniform(40, 100)), pitch_deg=float(rng.uniform(-60, 0)))
    dt = np.float16 if fp16 else np.float32
    gb = render_gbuffer(sc, cam, normal_dtype=dt, radiance_dtype=dt, channels=ch, cache=False)
    sectors = int(rng.choice([32, 128]))
    na = int(rng.choice([n for n in (1, 2, 4, 8, 16, 32) if sectors % n == 0]))
    kw = dict(slices=int(rng.integers(1, 9)), steps=int(rng.integers(1, 21)), sectors=sectors,
              ambient_samples=na, radius=float(rng.uniform(0.2, 4.0)),
              thickness=float(rng.choice([0.0, INF, rng.uniform(0.01, 1.0)])),
              thickness_slope=float(rng.choice([0.0, rng.uniform(0.0, 0.1)])),
              max_radius_px=float(rng.choice([0.0, rng.uniform(1.0, 30.0)])),
              min_step_q4=int(rng.choice([16, int(rng.integers(1, 17))])),
              step_distribution=int(rng.integers(2)), hit_criterion=int(rng.integers(2)),
              noise=int(rng.integers(3)), seed=int(rng.integers(0, 1 << 32)),
              ambient_sh=tuple(rng.uniform(-1.0, 1.0, 27)))
    return gb, cam, kw
