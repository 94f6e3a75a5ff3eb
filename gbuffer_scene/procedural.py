"""Procedural scenes and an analytic ray caster that writes a single-layer G-buffer.

Conventions (shared by every consumer of these arrays):
  * view space: x right, y up, camera looking down -z; image y grows downward;
    pixel (x, y) has its centre at (x + 0.5, y + 0.5);
  * the ray through pixel coordinates (X, Y) is r = ((X - cx)/fx, -(Y - cy)/fy, -1),
    so a point at linear view depth z along it is z * r;
  * depth is linear view depth (-z_view) in float32; 0 marks background;
  * normals are unit view-space normals; radiance is RGB direct light (albedo times
    Lambert times a hard shadow), the kind of light buffer Section 4.3 of the paper uses.
World space is y-up.  Everything is drawn from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

_EPS = 1e-9


@dataclass(frozen=True)
class CameraSpec:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    view_to_world: tuple  # 9 floats, row-major R with world_dir = R @ view_dir
    position: tuple = (0.0, 1.6, 0.0)

    @property
    def R(self) -> np.ndarray:
        return np.asarray(self.view_to_world, dtype=np.float64).reshape(3, 3)


@dataclass
class Scene:
    boxes_min: np.ndarray  # [N, 3] world
    boxes_max: np.ndarray  # [N, 3]
    albedo: np.ndarray  # [N + 1, 3]; row 0 is the ground plane
    light_dir: np.ndarray  # [3] unit, pointing toward the light
    seed: int = 0
    ambient_sh: np.ndarray = field(default_factory=lambda: np.zeros((9, 3)))


def _f32(v: float) -> float:
    return float(np.float32(v))


def make_camera(width: int, height: int, fov_y_deg: float = 90.0, pitch_deg: float = -50.0,
                yaw_deg: float = 0.0, position=(0.0, 1.6, 0.0)) -> CameraSpec:
    """Pinhole camera with vertical field of view ``fov_y_deg`` and square pixels."""
    f = (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)
    p = math.radians(pitch_deg)
    y = math.radians(yaw_deg)
    rx = np.array([[1, 0, 0], [0, math.cos(p), -math.sin(p)], [0, math.sin(p), math.cos(p)]])
    ry = np.array([[math.cos(y), 0, math.sin(y)], [0, 1, 0], [-math.sin(y), 0, math.cos(y)]])
    R = ry @ rx
    return CameraSpec(width, height, _f32(f), _f32(f), _f32(width / 2.0), _f32(height / 2.0),
                      tuple(float(np.float32(v)) for v in R.reshape(-1)), tuple(position))


def _ambient_sh(rng) -> np.ndarray:
    """An L2 real-SH sky probe: a constant term of 0.3 plus a seeded upward gradient."""
    y00 = 0.5 * math.sqrt(1.0 / math.pi)
    y1 = math.sqrt(3.0 / (4.0 * math.pi))
    sh = np.zeros((9, 3))
    sh[0] = 0.3 / y00 * rng.uniform(0.8, 1.2, 3)
    sh[1] = rng.uniform(0.05, 0.2, 3) / y1  # Y_{1,-1} is proportional to world y
    sh[2:] = rng.uniform(-0.02, 0.02, (7, 3))
    return sh


def make_scene(seed: int, n_boxes: int, n_planes: int) -> Scene:
    """Ground plane y = 0, ``n_boxes`` boxes standing on it and ``n_planes`` thin slabs."""
    rng = np.random.default_rng(seed)
    mins, maxs = [], []
    for _ in range(n_boxes):
        size = rng.uniform(0.2, 1.5, 3)
        c = np.array([rng.uniform(-6, 6), 0.0, rng.uniform(-14, -2)])
        mins.append([c[0] - size[0] / 2, 0.0, c[2] - size[2] / 2])
        maxs.append([c[0] + size[0] / 2, size[1], c[2] + size[2] / 2])
    for _ in range(n_planes):
        thin_axis = int(rng.integers(0, 3))
        long_edges = rng.uniform(0.5, 2.5, 2)
        raised = rng.uniform(0.0, 1.0) if rng.uniform() < 0.5 else 0.0
        c = np.array([rng.uniform(-6, 6), 0.0, rng.uniform(-14, -2)])
        size = np.empty(3)
        others = [a for a in range(3) if a != thin_axis]
        size[thin_axis] = 0.02
        size[others[0]] = long_edges[0]
        size[others[1]] = long_edges[1]
        mins.append([c[0] - size[0] / 2, raised, c[2] - size[2] / 2])
        maxs.append([c[0] + size[0] / 2, raised + size[1], c[2] + size[2] / 2])
    n = n_boxes + n_planes
    albedo = rng.uniform(0.1, 0.9, (n + 1, 3))
    el = math.radians(rng.uniform(30, 60))
    az = math.radians(rng.uniform(0, 360))
    light = np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    return Scene(np.asarray(mins, dtype=np.float64).reshape(n, 3),
                 np.asarray(maxs, dtype=np.float64).reshape(n, 3), albedo, light, seed,
                 _ambient_sh(rng))


# ----------------------------------------------------------------------------------------
# analytic ray casting
# ----------------------------------------------------------------------------------------

def _pixel_rays(cam: CameraSpec, ys: np.ndarray, xs: np.ndarray) -> np.ndarray:
    r = np.empty(ys.shape + (3,))
    r[..., 0] = (xs + 0.5 - cam.cx) / cam.fx
    r[..., 1] = -(ys + 0.5 - cam.cy) / cam.fy
    r[..., 2] = -1.0
    return r


def _safe_inv(d: np.ndarray) -> np.ndarray:
    out = np.empty_like(d)
    small = np.abs(d) < 1e-300
    out[~small] = 1.0 / d[~small]
    out[small] = np.where(np.signbit(d[small]), -1e300, 1e300)
    return out


def _slab(origin, inv_d, bmin, bmax):
    """Ray/box slab test. Returns (t_enter, t_exit, entry_axis)."""
    t1 = (bmin - origin) * inv_d
    t2 = (bmax - origin) * inv_d
    tlo = np.minimum(t1, t2)
    thi = np.maximum(t1, t2)
    axis = np.argmax(tlo, axis=-1)
    t_enter = np.max(tlo, axis=-1)
    t_exit = np.min(thi, axis=-1)
    return t_enter, t_exit, axis


def _project_bbox(cam: CameraSpec, pts_world: np.ndarray, margin: int = 2):
    """Screen rectangle covering world points, or None if any lies behind the camera."""
    R = cam.R
    pv = (pts_world - np.asarray(cam.position)) @ R  # R^T applied to each row
    if np.any(pv[:, 2] > -0.05):
        return None
    zd = -pv[:, 2]
    X = pv[:, 0] / zd * cam.fx + cam.cx
    Y = -pv[:, 1] / zd * cam.fy + cam.cy
    x0 = max(int(math.floor(X.min())) - margin, 0)
    x1 = min(int(math.ceil(X.max())) + margin, cam.width)
    y0 = max(int(math.floor(Y.min())) - margin, 0)
    y1 = min(int(math.ceil(Y.max())) + margin, cam.height)
    if x0 >= x1 or y0 >= y1:
        return (0, 0, 0, 0)
    return (y0, y1, x0, x1)


def _corners(bmin, bmax):
    return np.array([[bmin[0] if i & 1 == 0 else bmax[0],
                      bmin[1] if i & 2 == 0 else bmax[1],
                      bmin[2] if i & 4 == 0 else bmax[2]] for i in range(8)])


def render_gbuffer(scene: Scene, cam: CameraSpec, normal_dtype=np.float32,
                   radiance_dtype=np.float32, channels: int = 3, cache: bool = True):
    """Ray-cast ``scene`` through ``cam``.  Returns dict(depth, normal, radiance)."""
    key = None
    cache_dir = os.environ.get("SSVB_SCENE_CACHE", "/tmp/ssvb_scene_cache")
    if cache:
        key = (f"s{scene.seed}_n{len(scene.boxes_min)}_{cam.width}x{cam.height}_"
               f"{abs(hash((cam.fx, cam.fy, cam.cx, cam.cy, cam.view_to_world, cam.position))) % (1 << 40):x}")
        path = os.path.join(cache_dir, key + ".npz")
        if os.path.exists(path):
            try:
                with np.load(path, allow_pickle=False) as z:
                    depth, nrm, rad = z["depth"], z["normal"], z["radiance"]
                return _finish(depth, nrm, rad, normal_dtype, radiance_dtype, channels)
            except Exception:
                pass
    H, W = cam.height, cam.width
    R = cam.R
    O = np.asarray(cam.position, dtype=np.float64)
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    d = _pixel_rays(cam, ys, xs) @ R.T  # world-space direction, not normalised
    inv_d = _safe_inv(d)

    # ground plane y = 0
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = np.where(d[..., 1] < -1e-12, -O[1] / d[..., 1], np.inf)
    tbest = tg
    obj = np.where(np.isfinite(tg), 0, -1)
    nrm_w = np.zeros((H, W, 3))
    nrm_w[..., 1] = 1.0

    for b in range(len(scene.boxes_min)):
        bmin, bmax = scene.boxes_min[b], scene.boxes_max[b]
        rect = _project_bbox(cam, _corners(bmin, bmax))
        y0, y1, x0, x1 = rect if rect is not None else (0, H, 0, W)
        if y0 >= y1 or x0 >= x1:
            continue
        sl = (slice(y0, y1), slice(x0, x1))
        te, tx, ax = _slab(O, inv_d[sl], bmin, bmax)
        hit = (tx >= te) & (te > 1e-6) & (te < tbest[sl])
        if not np.any(hit):
            continue
        tb = tbest[sl]
        tb[hit] = te[hit]
        ob = obj[sl]
        ob[hit] = b + 1
        n_sub = nrm_w[sl]
        dsub = d[sl]
        nn = np.zeros(hit.shape + (3,))
        sign = -np.sign(np.take_along_axis(dsub, ax[..., None], axis=-1)[..., 0])
        np.put_along_axis(nn, ax[..., None], sign[..., None], axis=-1)
        n_sub[hit] = nn[hit]

    geom = obj >= 0
    depth = np.where(geom, tbest, 0.0)
    P = O + depth[..., None] * d   # sky rays (no hit, tbest = inf) get 0 here, then 0 below
    P = np.where(geom[..., None], P, 0.0)

    # hard shadows toward the directional light
    L = scene.light_dir
    lit = geom.copy()
    P_off = P + 1e-4 * nrm_w
    for b in range(len(scene.boxes_min)):
        bmin, bmax = scene.boxes_min[b], scene.boxes_max[b]
        c = _corners(bmin, bmax)
        ground = c - (c[:, 1:2] / max(L[1], 1e-6)) * L[None, :]
        rect = _project_bbox(cam, np.concatenate([c, ground]))
        y0, y1, x0, x1 = rect if rect is not None else (0, H, 0, W)
        if y0 >= y1 or x0 >= x1:
            continue
        sl = (slice(y0, y1), slice(x0, x1))
        inv_l = _safe_inv(np.broadcast_to(L, P_off[sl].shape).copy())
        te, tx, _ = _slab(P_off[sl], inv_l, bmin, bmax)
        occl = (tx >= np.maximum(te, 0.0)) & (obj[sl] != b + 1)
        lit[sl] &= ~occl

    albedo = scene.albedo[np.maximum(obj, 0)]
    ndl = np.maximum(0.0, nrm_w @ L)
    rad = np.where(geom[..., None], albedo * (ndl * lit)[..., None], 0.0)
    nrm_v = nrm_w @ R  # R^T n for each pixel
    nrm_v = np.where(geom[..., None], nrm_v, 0.0)

    depth = depth.astype(np.float32)
    if cache and key is not None:
        try:
            os.makedirs(cache_dir, exist_ok=True)
            tmp = os.path.join(cache_dir, key + f".{os.getpid()}.tmp.npz")
            np.savez(tmp, depth=depth, normal=nrm_v.astype(np.float32), radiance=rad.astype(np.float32))
            os.replace(tmp, os.path.join(cache_dir, key + ".npz"))
        except OSError:
            pass
    return _finish(depth, nrm_v.astype(np.float32), rad.astype(np.float32), normal_dtype,
                   radiance_dtype, channels)


def _finish(depth, nrm, rad, normal_dtype, radiance_dtype, channels):
    H, W = depth.shape
    def widen(a, dt):
        out = np.zeros((H, W, channels), dtype=dt)
        out[..., :3] = a.astype(dt)  # float16: round to nearest even
        return out
    return {"depth": np.ascontiguousarray(depth, dtype=np.float32),
            "normal": widen(nrm, normal_dtype),
            "radiance": widen(rad, radiance_dtype)}


# ----------------------------------------------------------------------------------------
# analytic scenes for the pins
# ----------------------------------------------------------------------------------------

def plane_gbuffer(cam: CameraSpec, normal_view, point_view, albedo=(0.5, 0.5, 0.5)):
    """G-buffer of the infinite plane {P : n . (P - P0) = 0} in view space.

    Pixels whose ray misses the plane (or hits it behind the camera) are background.
    Radiance is the constant ``albedo`` on the plane.
    """
    n = np.asarray(normal_view, dtype=np.float64)
    n = n / np.linalg.norm(n)
    P0 = np.asarray(point_view, dtype=np.float64)
    H, W = cam.height, cam.width
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    r = _pixel_rays(cam, ys, xs)
    den = r @ n
    with np.errstate(divide="ignore", invalid="ignore"):
        z = np.where(np.abs(den) > 1e-12, (P0 @ n) / den, 0.0)
    geom = z > 0
    depth = np.where(geom, z, 0.0).astype(np.float32)
    nrm = np.where(geom[..., None], n, 0.0).astype(np.float32)
    rad = np.where(geom[..., None], np.asarray(albedo, dtype=np.float64), 0.0).astype(np.float32)
    return {"depth": depth, "normal": nrm, "radiance": rad}


def crease_gbuffer(cam: CameraSpec, D: float, alpha: float, hinge_x: float = 0.0):
    """Fronto-parallel floor z_view = -D with a half-plane wall hinged on x_view = hinge_x.

    The wall rises toward the camera at angle ``alpha`` (radians) from the floor for
    x_view >= hinge_x:  z_view = -D + (x_view - hinge_x) tan(alpha).  The visible surface
    is the nearer of the two (a concave crease).  Radiance is 1 on the wall, 0 on the floor.
    """
    H, W = cam.height, cam.width
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    r = _pixel_rays(cam, ys, xs)
    ta = math.tan(alpha)
    # floor: z * r_z = -D  ->  z = D
    z_floor = np.full((H, W), D)
    # wall: -z = -D + (z r_x - hinge_x) tan(alpha)  ->  z (1 + r_x tan a) = D + hinge_x tan a
    den = 1.0 + r[..., 0] * ta
    with np.errstate(divide="ignore", invalid="ignore"):
        z_wall = np.where(den > 1e-12, (D + hinge_x * ta) / den, np.inf)
    on_wall = (z_wall * r[..., 0] >= hinge_x) & (z_wall < z_floor) & (z_wall > 0)
    depth = np.where(on_wall, z_wall, z_floor).astype(np.float32)
    n_floor = np.array([0.0, 0.0, 1.0])
    n_wall = np.array([-math.sin(alpha), 0.0, math.cos(alpha)])
    nrm = np.where(on_wall[..., None], n_wall, n_floor).astype(np.float32)
    rad = np.where(on_wall[..., None], 1.0, 0.0) * np.ones(3)
    return {"depth": depth, "normal": nrm, "radiance": rad.astype(np.float32)}


# ----------------------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------------------

WORKLOADS = {
    # 128x128, 8 boxes + 4 thin planes, FP32, 2 slices x 8 steps per side, t 0.5, radius 2
    "c1_128": dict(width=128, height=128, seed=1, n_boxes=8, n_planes=4, slices=2, steps=8,
                   thickness=0.5, radius=2.0, noise="hash", fp16=False),
    # 1920x1080, 64 boxes + 32 thin planes, FP32, 4 slices x 16 steps, t 0.5, radius 3
    "c2_1080p": dict(width=1920, height=1080, seed=2, n_boxes=64, n_planes=32, slices=4, steps=16,
                     thickness=0.5, radius=3.0, noise="r2", fp16=False),
    # 3840x2160, FP16 normals and radiance, 8 slices x 32 steps, radius 8, t ~ U[0.1, 1.0]
    "c3_4k_fp16": dict(width=3840, height=2160, seed=3, n_boxes=64, n_planes=32, slices=8, steps=32,
                       thickness=None, radius=8.0, noise="r2", fp16=True),
}


def workload(name: str, channels: int = 3):
    """Return (gbuffer dict, camera, sampling dict, scene) for a named workload."""
    w = dict(WORKLOADS[name])
    scene = make_scene(w["seed"], w["n_boxes"], w["n_planes"])
    cam = make_camera(w["width"], w["height"])
    dt = np.float16 if w["fp16"] else np.float32
    gb = render_gbuffer(scene, cam, normal_dtype=dt, radiance_dtype=dt, channels=channels)
    if w["thickness"] is None:
        w["thickness"] = float(np.float32(np.random.default_rng(w["seed"]).uniform(0.1, 1.0)))
    return gb, cam, w, scene


# ----------------------------------------------------------------------------------------
# mixed-resolution batches and request streams
# ----------------------------------------------------------------------------------------

BATCH_RESOLUTIONS = [(1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)]
SERVE_RESOLUTIONS = [(960, 540), (1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)]
POOL_SEED0 = 100  # scene seeds of the frame pools: 100, 101, ...


def mixed_batch(seed: int = 4, n_frames: int = 64, pool: int = 4):
    """Draws of a batch of mixed frames: resolution uniform over BATCH_RESOLUTIONS,
    slices uniform over {2, 4, 8}, steps over {8, 16, 32}, FP32 G-buffers, the scene
    one of ``pool`` seeds per resolution, noise seed = frame index; radius 3, t 0.5, R2."""
    rng = np.random.default_rng(seed)
    frames = []
    for i in range(n_frames):
        W, H = BATCH_RESOLUTIONS[int(rng.integers(len(BATCH_RESOLUTIONS)))]
        nd = int(rng.choice([2, 4, 8]))
        ns = int(rng.choice([8, 16, 32]))
        sc = POOL_SEED0 + int(rng.integers(pool))
        frames.append(dict(width=W, height=H, scene_seed=sc, slices=nd, steps=ns, noise_seed=i, fp16=False,
                           radius=3.0, thickness=0.5, noise="r2"))
    return frames


SMALL_RESOLUTIONS = [(256, 144), (320, 180), (480, 270), (640, 360)]


def small_batch(seed: int = 6, n_frames: int = 64, pool: int = 2):
    """Draws of a batch of small frames (probes, thumbnails, distant views): resolution
    uniform over SMALL_RESOLUTIONS, slices over {2, 4}, steps over {8, 16}, FP32
    G-buffers, the scene one of ``pool`` seeds per resolution, noise seed = frame index;
    radius 3, t 0.5, R2."""
    rng = np.random.default_rng(seed)
    frames = []
    for i in range(n_frames):
        W, H = SMALL_RESOLUTIONS[int(rng.integers(len(SMALL_RESOLUTIONS)))]
        nd = int(rng.choice([2, 4]))
        ns = int(rng.choice([8, 16]))
        sc = POOL_SEED0 + int(rng.integers(pool))
        frames.append(dict(width=W, height=H, scene_seed=sc, slices=nd, steps=ns, noise_seed=i, fp16=False,
                           radius=3.0, thickness=0.5, noise="r2"))
    return frames


def request_stream(seed: int = 5, n_requests: int = 2000, pool: int = 2):
    """Draws of a served request stream: resolution uniform over SERVE_RESOLUTIONS, slices
    uniform over 2..8, steps over {8, 16, 32}, FP16 or FP32 normals and radiance with
    probability 1/2, scene one of ``pool`` seeds per resolution, noise seed = request
    index, and a unit-rate exponential gap before each arrival (divide by the rate)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_requests):
        W, H = SERVE_RESOLUTIONS[int(rng.integers(len(SERVE_RESOLUTIONS)))]
        nd = int(rng.integers(2, 9))
        ns = int(rng.choice([8, 16, 32]))
        fp16 = bool(rng.integers(2))
        sc = POOL_SEED0 + int(rng.integers(pool))
        gap = float(rng.exponential(1.0))
        reqs.append(dict(width=W, height=H, scene_seed=sc, slices=nd, steps=ns, noise_seed=i, fp16=fp16,
                         radius=3.0, thickness=0.5, noise="r2", gap=gap))
    return reqs


def _render_one(key):
    seed, W, H = key
    render_gbuffer(make_scene(seed, 64, 32), make_camera(W, H), cache=True)
    return key


def render_pool(keys, workers: int = 8):
    """Render (scene_seed, W, H) keys of the 64-box / 32-plane generator with the default
    camera, in parallel through the file cache; returns key -> (FP32 G-buffer, scene).
    Call it before the process touches a GPU (the workers are forked)."""
    keys = sorted(set(keys))
    if workers > 1 and len(keys) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, len(keys))) as p:
            # largest first, so the 4K renders do not trail
            list(p.imap_unordered(_render_one, sorted(keys, key=lambda k: -k[1] * k[2])))
    out = {}
    for seed, W, H in keys:
        sc = make_scene(seed, 64, 32)
        out[(seed, W, H)] = (render_gbuffer(sc, make_camera(W, H), cache=True), sc)
    return out


def as_format(gb, fp16: bool):
    """The same G-buffer with normal and radiance cast to FP16 (round to nearest even)."""
    if not fp16:
        return gb
    return {"depth": gb["depth"], "normal": gb["normal"].astype(np.float16),
            "radiance": gb["radiance"].astype(np.float16)}
