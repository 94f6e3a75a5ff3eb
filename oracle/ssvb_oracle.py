"""Plain FP64 CPU oracle of the visibility-bitmask gather (AO, indirect diffuse, ambient).

TEST INFRASTRUCTURE: imported only by the tests, the smoke check and the benchmark's
CPU-baseline leg.  It shares no code with the HIP path.

Source: O. Therrien, Y. Levesque, G. Gilet, "Screen Space Indirect Lighting with
Visibility Bitmask" (arXiv 2301.11376).  The method is a screen-space approximation,
not a fast route to a closed form, so this oracle is the algorithm itself: Algorithm 1
(AO and GI with visibility bitmasks) plus the ambient split of Section 3.2, taken step by
step in the paper's order, vectorised over pixels (every pixel is independent) and
looping over slices, sides and steps in FP64.  Integer parts (noise, slice directions,
step lattice) are exact integer arithmetic; the one floating-point operation that
decides an integer in the lattice, the step length in 1/16 pixel, is a single IEEE FP32
division, reproduced here with numpy float32.

Readings of the paper where it is silent, garbled or self-contradictory (each one is
listed again in the design notes):
  R1  hit criterion: the prose (Section 3.1 and its slice figure) sets a sector once half of
      it or more is covered; the pseudo-code uses floor/ceil.  Default ROUND sets sector k iff its
      centre lies in the sample's angular interval; PSEUDOCODE (floor start, ceil width)
      is available as an option.
  R2  the "+pi/2" inside the pseudo-code's sector count is a typo: the count spans
      theta_max - theta_min.
  R3  angles are signed, measured in the slice from the projected normal, positive toward
      the slice direction d, clamped to [-pi/2, pi/2] (the bitmask is centred on the
      projected normal, Section 3.1).
  R4  the back sample lies *behind* the front one, t farther from the camera along the
      centre pixel's view ray (s_b = s_f - t v with v pointing to the camera); only this
      makes t -> infinity equal GTAO without falloff (Section 3.1).
  R5  angles are true angles (atan2 of the slice coordinates), not cosines (Section 3.1
      converts the horizon cosines to angles).
  R6  sectors are uniform in angle (Eq. 4 and the AO update of Algorithm 1).
  R7  the AO output is visibility (1 = unoccluded), as Algorithm 1 accumulates it.
  R8  loop bounds are exclusive: N_d slices, N_s steps on *each* side (Section 4.1).
  R9  step placement: offset (j + 1 + xi) * step with xi in [0, 1) per slice (8 bits),
      shared by both sides; step = r / (N_s + 1) (Algorithm 1), at least min_step_q4/16 px.
  R10 projected radius r = radius * f_y / z_p pixels (world radius, screen aligned).
  R11 slice directions phi_i = (i + rho) pi / N_d (Algorithm 1: directions with random
      offset), quantised to pi/4096 through an integer direction table.
  R12 both cosine factors of the GI weight are clamped at 0.
  R13 off-screen, background and centre-texel samples are skipped; a background centre
      pixel outputs AO = 1, GI = 0, ambient = 0.
  R14 thickness grows linearly with depth: t_p = t0 + k z_p (Section 3.1), k = 0 default.
  R15 t = +inf is allowed and gives each side's back angle = its hemisphere edge.
  R16 a projected normal of squared length < 1e-12 in the slice gives gamma = 0.
  R17 ambient: N_a subregions of N_b / N_a sectors; direction at each subregion centre;
      ambient += (unoccluded sectors of the subregion) / N_b * L(direction) with L an L2
      real-SH probe in world space (Section 3.2; probes are named in Section 5).
  R18 GI is Algorithm 1's quantity divided by N_d, with no further normalisation.
  R19 the view-space position of step j (Algorithm 1) is the depth read from the texel containing the
      step's exact screen position, placed on that exact position's view ray (the depth
      buffer is point sampled; the sample stays in the slice plane).
  R21 the optional exponential step distribution (Section 4.3: samples denser near the
      pixel; the curve is not given) is quadratic: step j sits at ((j + 1 + xi) /
      (N_s + 1))^2 of the reach q (N_s + 1), with the same jitter xi; in integers,
      o_j = (((q a_j^2) >> 16) * floor(2^32 / (N_s + 1))) >> 32, a_j = 256 (j + 1) + xi8.
  R22 half resolution (Section 4.3: the gather runs on a quarter of the pixels, then a
      bilateral upsampler fills the image; neither is specified further): the
      gather runs on the pixels whose x and y are both even, reading the full-resolution
      G-buffer; every other pixel takes the average of its 1, 2 or 4 nearest computed
      pixels with weights bilinear x (1e-3 + exp(-((z - z_n) / (0.05 z))^2)), background
      neighbours excluded; a background pixel, or one with no computed foreground
      neighbour, outputs AO = 1, GI = 0, ambient = 0.
  R23 multi-bounce (Section 4.3: the indirect light is injected into the light buffer of
      the next frame, its intensity scaled down): next light = direct + g albedo * GI per
      pixel and channel, with a gain g in [0, 1] as the balance.
  R24 denoising (Section 4.1 and Table 2 time a denoising pass after the gather, 0.33 ms
      at full and 0.1 ms at half resolution, but do not describe it): an edge-aware
      a-trous filter.  P passes (1 to 3); pass i averages each foreground pixel's AO, GI
      and ambient over the 5 x 5 taps p + 2^i (a, b) g, a, b in -2..2 (g = 1, or 2 at half
      resolution, where the filter runs on the gathered even/even grid), with weights
      h_a h_b exp(-(n_p . (P_q - P_p) / (sigma z_p))^2) max(0, n_p . n_q)^k, h = (1, 4,
      6, 4, 1) / 16, P = z r(x, y) the view-space position and n the unit normal; the
      centre's own weight is h_0^2; taps off the image or on background are left out and
      the weights renormalised; a background pixel keeps its input.  At half resolution
      the R22 upsampler then refills the pixels with an odd coordinate.
  R25 frame sequences (Section 4.3: multi-bounce through the light buffer of the next
      frame; Section 3.1: the integral is distributed over time as well as space; Section
      4.1: one slice per pixel jittered over frames): frame n's light = direct_n + g
      albedo_n * GI_{n-1} (no feedback before frame 0), stored in the light buffer's
      precision (FP32 or FP16), and frame n draws its noise with seed s0 + n (mod 2^32).
      Temporal accumulation of the outputs (which needs reprojection for a moving camera)
      is left to the caller.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from decimal import Decimal, getcontext

import numpy as np

ROUND, PSEUDOCODE = 0, 1
NOISE_HASH, NOISE_R2, NOISE_FIXED = 0, 1, 2
NOISE_NAMES = {"hash": NOISE_HASH, "r2": NOISE_R2, "fixed": NOISE_FIXED}
STEPS_UNIFORM, STEPS_QUADRATIC = 0, 1

LUT_SIZE = 4096           # slice directions quantised to pi / 4096
LUT_ONE = 4096            # fixed-point 1.0 of the direction table
LATTICE_CAP_PX = 16383    # hard cap on the screen radius, in pixels
MASK32 = np.uint64(0xFFFFFFFF)


def _f32(v) -> float:
    """The float32 value the C ABI would carry for ``v``, as a Python float."""
    return float(np.float32(v))


@dataclass
class Camera:
    """Pinhole camera.  Pixel (x, y) has its centre at (x + 0.5, y + 0.5); the view ray
    through screen point (X, Y) is ((X - cx)/fx, -(Y - cy)/fy, -1) (view space: x right,
    y up, looking down -z).  ``view_to_world`` is a row-major 3x3 rotation."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    view_to_world: tuple = (1, 0, 0, 0, 1, 0, 0, 0, 1)


@dataclass
class Params:
    slices: int = 2               # N_d
    steps: int = 8                # N_s, per side
    sectors: int = 32             # N_b
    ambient_samples: int = 4      # N_a, divides N_b
    radius: float = 2.0           # world-space radius
    thickness: float = 0.5        # t0 (may be +inf)
    thickness_slope: float = 0.0  # k in t_p = t0 + k z_p
    max_radius_px: float = 0.0    # 0: lattice cap only
    min_step_q4: int = 16         # shortest step, 1/16 px
    step_distribution: int = 0    # STEPS_UNIFORM or STEPS_QUADRATIC (R21)
    resolution: int = 1           # 1: every pixel; 2: half resolution + upsampling (R22)
    hit_criterion: int = ROUND
    noise: int = NOISE_HASH
    seed: int = 0
    ambient_sh: tuple = field(default_factory=lambda: tuple([0.0] * 27))  # [9][3]


# ----------------------------------------------------------------------------------------
# counter-based noise (random numbers the method draws; Algorithm 1: slice directions
# turned by a random offset; Section 4.3: jitter along the sampling direction)
# ----------------------------------------------------------------------------------------

def pcg_hash(v):
    """PCG-RXS-M-XS 32-bit hash of Jarzynski & Olano, "Hash Functions for GPU Rendering"
    (JCGT 9(3), 2020), built on O'Neill's PCG output permutation."""
    v = np.asarray(v, dtype=np.uint64) & MASK32
    state = (v * np.uint64(747796405) + np.uint64(2891336453)) & MASK32
    shift = (state >> np.uint64(28)) + np.uint64(4)
    word = (((state >> shift) ^ state) * np.uint64(277803737)) & MASK32
    return ((word >> np.uint64(22)) ^ word) & MASK32


def pixel_hash(x, y, s):
    """Nested hash of a pixel and a 32-bit stream id: pcg(x + pcg(y + pcg(s)))."""
    x = np.asarray(x, dtype=np.uint64)
    y = np.asarray(y, dtype=np.uint64)
    s = np.asarray(s, dtype=np.uint64)
    return pcg_hash((x + pcg_hash((y + pcg_hash(s)) & MASK32)) & MASK32)


def r2_constants():
    """Roberts' R2 sequence in 32-bit fixed point: a1 = round(2^32/g), a2 = round(2^32/g^2)
    with g the plastic number (real root of g^3 = g + 1); a3 = round(2^32/phi) mixes the
    seed (phi the golden ratio)."""
    getcontext().prec = 60
    g = Decimal("1.3")
    for _ in range(60):
        g = g - (g ** 3 - g - 1) / (3 * g ** 2 - 1)
    phi = (1 + Decimal(5).sqrt()) / 2
    two32 = Decimal(2) ** 32
    rnd = lambda d: int(d.to_integral_value(rounding="ROUND_HALF_EVEN"))
    return rnd(two32 / g), rnd(two32 / (g * g)), rnd(two32 / phi)


def slice_noise(xs, ys, n_slices: int, noise: int, seed: int):
    """Per-pixel rotation rho16 in [0, 2^16) and per-slice jitter xi8 in [0, 256)."""
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    n = xs.shape[0]
    seed = int(seed) & 0xFFFFFFFF
    if noise == NOISE_FIXED:
        return np.zeros(n, np.int64), np.zeros((n, n_slices), np.int64)
    if noise == NOISE_HASH:
        rho16 = (pixel_hash(xs, ys, seed) >> np.uint64(16)).astype(np.int64)
    elif noise == NOISE_R2:
        a1, a2, a3 = r2_constants()
        rho32 = (xs.astype(object) * a1 + ys.astype(object) * a2 + seed * a3) % (1 << 32)
        rho16 = (np.asarray(rho32, dtype=np.int64) >> 16)
    else:
        raise ValueError("unknown noise mode")
    xi8 = np.empty((n, n_slices), np.int64)
    for i in range(n_slices):
        xi8[:, i] = (pixel_hash(xs, ys, (seed + 1 + i) & 0xFFFFFFFF) >> np.uint64(24)).astype(np.int64)
    return rho16, xi8


# ----------------------------------------------------------------------------------------
# slice directions and the step lattice
# ----------------------------------------------------------------------------------------

def direction_lut():
    """Dx[k], Dy[k] = round(4096 cos(pi k / 4096)), round(4096 sin(pi k / 4096)) (FP64)."""
    k = np.arange(LUT_SIZE, dtype=np.float64)
    phi = np.pi * k / LUT_SIZE
    dx = np.floor(LUT_ONE * np.cos(phi) + 0.5).astype(np.int64)
    dy = np.floor(LUT_ONE * np.sin(phi) + 0.5).astype(np.int64)
    return dx, dy


def step_q4(z_p, cam: Camera, prm: Params):
    """Step length in 1/16 pixel (Algorithm 1: step = r / (N_s + 1), r the projected radius).

    16 r / (N_s + 1) = C / z_p with C = 16 radius f_y / (N_s + 1), formed in FP64 and
    rounded once to FP32; the quotient is one IEEE FP32 division, floored and clamped to
    [min_step_q4, q_max], q_max = floor(16 R_cap / (N_s + 1))."""
    ns = prm.steps
    c32 = np.float32(16.0 * _f32(prm.radius) * _f32(cam.fy) / (ns + 1))
    rcap = LATTICE_CAP_PX if _f32(prm.max_radius_px) <= 0 else min(_f32(prm.max_radius_px), LATTICE_CAP_PX)
    q_min = int(prm.min_step_q4)
    q_max = max(q_min, int(math.floor(16.0 * rcap / (ns + 1))))
    with np.errstate(divide="ignore", over="ignore"):
        quot = c32 / np.asarray(z_p, dtype=np.float32)
    quot = np.minimum(quot, np.float32(q_max))
    q = np.floor(quot).astype(np.int64)
    return np.clip(q, q_min, q_max)


def step_offset_q4(q, xi8, j, ns, dist):
    """Offset of step j (0-based) from the pixel centre along the slice, 1/16 px.

    UNIFORM (Algorithm 1): (j + 1 + xi) steps of q.  QUADRATIC (Section 4.3, reading
    R21): the reach q (N_s + 1) times ((j + 1 + xi) / (N_s + 1))^2, in exact integers."""
    if dist == STEPS_UNIFORM:
        return q * (j + 1) + ((q * xi8) >> 8)
    a = (j + 1) * 256 + xi8
    t = (q * a * a) >> 16
    return (t * ((1 << 32) // (ns + 1))) >> 32


def sh_eval(coeffs, dirs):
    """L2 real spherical harmonics: sum_i c_i Y_i(d) per RGB channel.  ``coeffs`` is
    [9][3] (coefficient-major), ``dirs`` [..., 3] unit vectors in the probe's frame."""
    c = np.asarray(coeffs, dtype=np.float64).reshape(9, 3)
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    pi = math.pi
    basis = [
        np.full_like(x, 0.5 * math.sqrt(1.0 / pi)),
        math.sqrt(3.0 / (4.0 * pi)) * y,
        math.sqrt(3.0 / (4.0 * pi)) * z,
        math.sqrt(3.0 / (4.0 * pi)) * x,
        0.5 * math.sqrt(15.0 / pi) * x * y,
        0.5 * math.sqrt(15.0 / pi) * y * z,
        0.25 * math.sqrt(5.0 / pi) * (3.0 * z * z - 1.0),
        0.5 * math.sqrt(15.0 / pi) * x * z,
        0.25 * math.sqrt(15.0 / pi) * (x * x - y * y),
    ]
    out = np.zeros(x.shape + (3,))
    for i in range(9):
        out += basis[i][..., None] * c[i]
    return out


def _dot(a, b):
    return np.einsum("...k,...k->...", a, b)


def _bits(lo, hi, nb):
    """Boolean sector set [lo, hi) for integer arrays lo, hi (shape [n]) -> [n, nb]."""
    k = np.arange(nb)
    return (k[None, :] >= lo[:, None]) & (k[None, :] < hi[:, None])


# ----------------------------------------------------------------------------------------
# the method
# ----------------------------------------------------------------------------------------

def inject_bounce(direct, albedo, gi, gain):
    """Light buffer of the next frame (Section 4.3, reading R23): direct + gain * albedo *
    GI, per pixel and RGB channel, in FP64.  ``direct`` and ``albedo`` are [H, W, C >= 3]
    (FP32 or FP16, upcast exactly), ``gi`` [H, W, 3]."""
    d = np.asarray(direct)[..., :3].astype(np.float64)
    a = np.asarray(albedo)[..., :3].astype(np.float64)
    return d + float(np.float32(gain)) * a * np.asarray(gi, dtype=np.float64)


def bounce_sequence(frames, cam, prm, gain, light_dtype=np.float32, **compute_kw):
    """A sequence of frames with multi-bounce feedback and temporal jitter (reading R25).

    Frame n's light buffer is its direct light plus gain x albedo x the GI of frame n - 1
    (Section 4.3: the indirect light is injected into the light buffer the next frame
    uses; nothing before frame 0), stored as ``light_dtype``; frame n is gathered on that
    light with the noise of seed prm.seed + n, so the slices turn from frame to frame
    (Section 3.1 distributes the integral over time; the timings of Section 4.1 take one
    slice per pixel, jittered over frames).  ``frames``: a sequence of dicts with
    ``depth``, ``normal``, ``direct`` and ``albedo`` (one camera for all).  Returns one
    ``compute`` result per frame (``compute_kw`` passed on, e.g. return_masks), each with
    the frame's ``light`` added."""
    from dataclasses import replace
    out, gi = [], None
    for n, f in enumerate(frames):
        H, W = np.asarray(f["depth"]).shape
        prev = gi if gi is not None else np.zeros((H, W, 3))
        light = inject_bounce(f["direct"], f["albedo"], prev, gain).astype(light_dtype)
        r = compute(f["depth"], f["normal"], light, cam, replace(prm, seed=(prm.seed + n) % (1 << 32)), **compute_kw)
        r["light"] = light
        gi = r["gi"]
        out.append(r)
    return out


UPSAMPLE_SIGMA = 0.05    # relative depth scale of the upsampling weights (R22)
UPSAMPLE_FLOOR = 1e-3    # weight floor: depth-incompatible neighbours still blend


def bilateral_upsample(depth, ao, gi, amb):
    """Fill the pixels with an odd coordinate from the computed (even, even) pixels
    (reading R22).  ``ao`` [H, W], ``gi`` / ``amb`` [H, W, 3] hold the gather's results at
    the even pixels; returns full images (the even pixels unchanged)."""
    H, W = depth.shape
    z = np.asarray(depth, dtype=np.float32).astype(np.float64)
    fg = np.isfinite(z) & (z > 0)
    ao_o, gi_o, amb_o = ao.copy(), gi.copy(), amb.copy()
    for y in range(H):
        ny = [(y, 1.0)] if y % 2 == 0 else ([(y - 1, 0.5), (y + 1, 0.5)] if y + 1 < H else [(y - 1, 1.0)])
        for x in range(W):
            if x % 2 == 0 and y % 2 == 0:
                continue
            nx = [(x, 1.0)] if x % 2 == 0 else ([(x - 1, 0.5), (x + 1, 0.5)] if x + 1 < W else [(x - 1, 1.0)])
            sw, sao, sgi, samb = 0.0, 0.0, np.zeros(3), np.zeros(3)
            if fg[y, x]:
                for yy, by in ny:
                    for xx, bx in nx:
                        if not fg[yy, xx]:
                            continue
                        d = (z[y, x] - z[yy, xx]) / (UPSAMPLE_SIGMA * z[y, x])
                        w = by * bx * (UPSAMPLE_FLOOR + math.exp(-d * d))
                        sw += w
                        sao += w * ao[yy, xx]
                        sgi += w * gi[yy, xx]
                        samb += w * amb[yy, xx]
            if sw > 0.0:
                ao_o[y, x], gi_o[y, x], amb_o[y, x] = sao / sw, sgi / sw, samb / sw
            else:
                ao_o[y, x], gi_o[y, x], amb_o[y, x] = 1.0, 0.0, 0.0
    return ao_o, gi_o, amb_o


DENOISE_KERNEL = (1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16)  # B3 spline (R24)


def denoise(depth, normal, cam: Camera, ao, gi, amb, passes=2, normal_power=16, plane_sigma=0.05,
            resolution=1):
    """Edge-aware a-trous denoising of the gather's outputs (reading R24), in FP64.
    ``depth`` [H, W], ``normal`` [H, W, C >= 3] (FP16 upcast exactly), ``ao`` [H, W], ``gi``
    / ``amb`` [H, W, 3].  Returns (ao, gi, amb)."""
    H, W = depth.shape
    g = 2 if resolution == 2 else 1
    z = np.asarray(depth, dtype=np.float32).astype(np.float64)[::g, ::g]
    fg = np.isfinite(z) & (z > 0)
    n = np.asarray(normal)[::g, ::g, :3].astype(np.float64)
    n = n / np.linalg.norm(n, axis=-1, keepdims=True).clip(1e-300)
    gh, gw = z.shape
    ys, xs = np.meshgrid(np.arange(gh) * g, np.arange(gw) * g, indexing="ij")
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    ray = np.stack([(xs + 0.5 - cx) / fx, -(ys + 0.5 - cy) / fy, -np.ones_like(z)], axis=-1)
    pos = np.where(fg, z, 0.0)[..., None] * ray
    zp = np.where(fg, z, 1.0)    # background pixels keep their input; any scale will do
    sig = np.concatenate([np.asarray(ao, np.float64)[::g, ::g, None], np.asarray(gi, np.float64)[::g, ::g],
                          np.asarray(amb, np.float64)[::g, ::g]], axis=-1)
    inv_scale = 0.0 if math.isinf(plane_sigma) else 1.0 / float(np.float32(plane_sigma))
    for i in range(passes):
        s = 1 << i
        acc = (DENOISE_KERNEL[2] ** 2) * sig
        wsum = np.full((gh, gw), DENOISE_KERNEL[2] ** 2)
        for b in range(-2, 3):
            for a in range(-2, 3):
                if a == 0 and b == 0:
                    continue
                dy, dx = b * s, a * s
                # q = p + (dx, dy) grid cells; p ranges over the cells whose q is on the grid
                py0, py1 = max(0, -dy), min(gh, gh - dy)
                px0, px1 = max(0, -dx), min(gw, gw - dx)
                if py0 >= py1 or px0 >= px1:
                    continue
                P_p = pos[py0:py1, px0:px1]
                n_p = n[py0:py1, px0:px1]
                Q = (slice(py0 + dy, py1 + dy), slice(px0 + dx, px1 + dx))
                dist = np.sum(n_p * (pos[Q] - P_p), axis=-1) * inv_scale / zp[py0:py1, px0:px1]
                w = (DENOISE_KERNEL[a + 2] * DENOISE_KERNEL[b + 2] * np.exp(-dist * dist)
                     * np.maximum(0.0, np.sum(n_p * n[Q], axis=-1)) ** normal_power)
                w = np.where(fg[Q], w, 0.0)
                acc[py0:py1, px0:px1] += w[..., None] * sig[Q]
                wsum[py0:py1, px0:px1] += w
        sig = np.where(fg[..., None], acc / wsum[..., None], sig)
    ao_o = np.array(ao, dtype=np.float64)
    gi_o = np.array(gi, dtype=np.float64)
    amb_o = np.array(amb, dtype=np.float64)
    ao_o[::g, ::g], gi_o[::g, ::g], amb_o[::g, ::g] = sig[..., 0], sig[..., 1:4], sig[..., 4:7]
    if g == 2:
        ao_o, gi_o, amb_o = bilateral_upsample(depth, ao_o, gi_o, amb_o)
    return ao_o, gi_o, amb_o


def compute(depth, normal, radiance, cam: Camera, prm: Params, pixels=None,
            return_masks=False, return_lattice=False, return_endpoints=False,
            index_bias=None):
    """Run the visibility-bitmask gather on every pixel (or on ``pixels`` = (ys, xs)).

    depth: float32 [H, W] linear view depth (<= 0 or non-finite: background).
    normal, radiance: [H, W, C >= 3] float32 or float16 (upcast exactly to FP64).
    Returns a dict with ``ao`` [n], ``gi`` [n, 3], ``ambient`` [n, 3] (reshaped to
    [H, W, ...] when ``pixels`` is None), and optionally ``masks`` (uint32 [n, N_d] when
    N_b <= 32, else bool [n, N_d, N_b]), ``lattice`` (int [n, N_d, 2, N_s, 2]: X, Y per
    slice, side (+ then -), step) and ``endpoints`` (FP64 [n, N_d, 2, N_s, 2]: the two
    arguments whose floor (ROUND) or floor/ceil (PSEUDOCODE) give the sample's sectors;
    NaN for skipped samples).  ``index_bias`` (int, same shape as ``endpoints``) is added to
    those integers; the mismatch tracer uses it to flip a near-tie rounding.
    """
    H, W = depth.shape
    if getattr(prm, "resolution", 1) == 2:
        # half resolution (R22): the gather on the even pixels, then the upsampler
        if pixels is not None or return_masks or return_lattice or return_endpoints:
            raise ValueError("half resolution computes whole images of AO, GI and ambient only")
        from dataclasses import replace
        ye, xe = np.meshgrid(np.arange(0, H, 2), np.arange(0, W, 2), indexing="ij")
        part = compute(depth, normal, radiance, cam, replace(prm, resolution=1),
                       pixels=(ye.reshape(-1), xe.reshape(-1)))
        ao = np.ones((H, W))
        gi = np.zeros((H, W, 3))
        amb = np.zeros((H, W, 3))
        ao[ye, xe] = part["ao"].reshape(ye.shape)
        gi[ye, xe] = part["gi"].reshape(ye.shape + (3,))
        amb[ye, xe] = part["ambient"].reshape(ye.shape + (3,))
        ao, gi, amb = bilateral_upsample(depth, ao, gi, amb)
        z = np.asarray(depth, dtype=np.float32)
        return {"ao": ao, "gi": gi, "ambient": amb, "valid": np.isfinite(z) & (z > 0)}
    depth64 = np.asarray(depth, dtype=np.float32).astype(np.float64)
    nrm64 = np.asarray(normal)[..., :3].astype(np.float64)
    rad64 = np.asarray(radiance)[..., :3].astype(np.float64)
    if pixels is None:
        ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        ys, xs = ys.reshape(-1), xs.reshape(-1)
    else:
        ys, xs = (np.asarray(a, dtype=np.int64).reshape(-1) for a in pixels)
    n = ys.shape[0]
    nd, ns, nb, na = prm.slices, prm.steps, prm.sectors, prm.ambient_samples
    assert nb % na == 0
    fx, fy, cx, cy = _f32(cam.fx), _f32(cam.fy), _f32(cam.cx), _f32(cam.cy)
    Rvw = np.array([_f32(v) for v in cam.view_to_world], dtype=np.float64).reshape(3, 3)
    sh = np.array([_f32(v) for v in prm.ambient_sh], dtype=np.float64).reshape(9, 3)
    t0, tk = _f32(prm.thickness), _f32(prm.thickness_slope)

    ao = np.ones(n)
    gi = np.zeros((n, 3))
    amb = np.zeros((n, 3))
    masks = np.zeros((n, nd, nb), dtype=bool)
    lattice = np.zeros((n, nd, 2, ns, 2), dtype=np.int64) if return_lattice else None
    endpoints = np.full((n, nd, 2, ns, 2), np.nan) if return_endpoints else None

    # Algorithm 1: p, the view-space fragment position; n_p, its view-space normal
    z_p = depth64[ys, xs] if n else np.zeros(0)
    valid = np.isfinite(z_p) & (z_p > 0)
    r_p = np.stack([(xs + 0.5 - cx) / fx, -(ys + 0.5 - cy) / fy, -np.ones(n)], axis=-1)
    p = np.where(valid, z_p, 0.0)[:, None] * r_p
    v = -r_p / np.linalg.norm(r_p, axis=-1, keepdims=True)      # toward the camera
    n_p = nrm64[ys, xs] if n else np.zeros((0, 3))

    # Algorithm 1: projected radius and step size; thickness (Section 3.1)
    q = step_q4(np.where(valid, z_p, 1.0), cam, prm)
    t_p = t0 + tk * np.where(valid, z_p, 0.0) if tk != 0.0 else np.full(n, t0)

    # Algorithm 1: slice directions turned by a random offset; per-slice jitter (Section 4.3)
    rho16, xi8 = slice_noise(xs, ys, nd, prm.noise, prm.seed)
    lut_dx, lut_dy = direction_lut()

    ao_sum = np.zeros(n)
    for i in range(nd):
        k_i = (i * 65536 + rho16) // (16 * nd)
        dx_i, dy_i = lut_dx[k_i], lut_dy[k_i]
        # slice plane: spanned by v and the view-space direction of the screen line
        d3 = np.stack([dx_i / (LUT_ONE * fx), -dy_i / (LUT_ONE * fy), np.zeros(n)], axis=-1)
        e = d3 - _dot(d3, v)[:, None] * v
        e = e / np.linalg.norm(e, axis=-1, keepdims=True)
        # projected normal angle gamma, measured from v toward e (the bitmask's centre)
        n_v, n_e = _dot(n_p, v), _dot(n_p, e)
        degenerate = n_v * n_v + n_e * n_e < 1e-12
        gamma = np.where(degenerate, 0.0, np.arctan2(n_e, n_v))

        b_i = np.zeros((n, nb), dtype=bool)                    # bitmask b_i <- 0
        for side_idx, s in enumerate((1, -1)):
            for j in range(ns):
                o = step_offset_q4(q, xi8[:, i], j, ns, prm.step_distribution)  # 1/16 px
                X = ((xs << 16) + 32768 + s * o * dx_i) >> 16
                Y = ((ys << 16) + 32768 + s * o * dy_i) >> 16
                if return_lattice:
                    lattice[:, i, side_idx, j, 0] = X
                    lattice[:, i, side_idx, j, 1] = Y
                ok = valid & (X >= 0) & (X < W) & (Y >= 0) & (Y < H) & ~((X == xs) & (Y == ys))
                Xc, Yc = np.clip(X, 0, W - 1), np.clip(Y, 0, H - 1)
                z_s = depth64[Yc, Xc]
                ok &= np.isfinite(z_s) & (z_s > 0)
                z_s = np.where(ok, z_s, 1.0)
                # front sample s_f: depth of that texel on the exact step position's ray
                X_e = xs + 0.5 + s * o * dx_i / 65536.0
                Y_e = ys + 0.5 + s * o * dy_i / 65536.0
                r_e = np.stack([(X_e - cx) / fx, -(Y_e - cy) / fy, -np.ones(n)], axis=-1)
                s_f = z_s[:, None] * r_e
                delta = s_f - p
                d_e, d_v = _dot(delta, e), _dot(delta, v)
                # back sample s_b = s_f - t_p v:  (s_b - p).e = delta.e, (s_b - p).v = delta.v - t_p
                theta_f = np.arctan2(d_e, d_v) - gamma
                theta_b = np.arctan2(d_e, d_v - t_p) - gamma
                theta_f = np.clip(theta_f, -np.pi / 2, np.pi / 2)
                theta_b = np.clip(theta_b, -np.pi / 2, np.pi / 2)
                t_min, t_max = np.minimum(theta_f, theta_b), np.maximum(theta_f, theta_b)
                u_lo = (t_min + np.pi / 2) / np.pi
                u_hi = (t_max + np.pi / 2) / np.pi
                if prm.hit_criterion == ROUND:
                    arg0, arg1 = nb * u_lo + 0.5, nb * u_hi + 0.5
                    a = np.floor(arg0).astype(np.int64)
                    b = np.floor(arg1).astype(np.int64)
                else:
                    arg0, arg1 = nb * u_lo, nb * (u_hi - u_lo)
                    a = np.floor(arg0).astype(np.int64)
                    b = np.ceil(arg1).astype(np.int64)
                if index_bias is not None:
                    a = a + index_bias[:, i, side_idx, j, 0]
                    b = b + index_bias[:, i, side_idx, j, 1]
                if prm.hit_criterion != ROUND:
                    b = np.minimum(a + b, nb)                  # [a, a + width)
                if return_endpoints:
                    endpoints[:, i, side_idx, j, 0] = np.where(ok, arg0, np.nan)
                    endpoints[:, i, side_idx, j, 1] = np.where(ok, arg1, np.nan)
                b_j = _bits(a, b, nb) & ok[:, None]
                # GI from the newly covered sectors (Algorithm 1; Section 3.3)
                new = b_j & ~b_i
                cnt = new.sum(axis=1)
                contrib = cnt > 0
                if np.any(contrib):
                    l_j = delta / np.linalg.norm(delta, axis=-1, keepdims=True)
                    n_j = nrm64[Yc, Xc]
                    c_j = rad64[Yc, Xc]
                    w = (cnt / nb) * np.maximum(0.0, _dot(n_p, l_j)) * np.maximum(0.0, -_dot(n_j, l_j))
                    gi += np.where(contrib, w, 0.0)[:, None] * c_j
                b_i |= b_j
        # AO: uniform sectors (Eq. 4), accumulated as visibility
        ao_sum += 1.0 - b_i.sum(axis=1) / nb
        masks[:, i] = b_i
        # directionally occluded ambient (Section 3.2): N_a subregions, one probe
        # direction at the centre of each, weighted by its unoccluded sectors / N_b
        per = nb // na
        for k in range(na):
            psi = gamma + (-np.pi / 2 + (k + 0.5) * np.pi / na)
            a_k = np.cos(psi)[:, None] * v + np.sin(psi)[:, None] * e
            L_k = sh_eval(sh, a_k @ Rvw.T)
            free = (~b_i[:, k * per:(k + 1) * per]).sum(axis=1)
            amb += (free / nb)[:, None] * L_k

    ao = np.where(valid, ao_sum / nd, 1.0)
    gi = np.where(valid[:, None], gi / nd, 0.0)
    amb = np.where(valid[:, None], amb / nd, 0.0)
    masks &= valid[:, None, None]

    out = {"ao": ao, "gi": gi, "ambient": amb, "valid": valid}
    if return_masks:
        if nb <= 32:
            weights = (np.uint64(1) << np.arange(nb, dtype=np.uint64))
            packed = (masks.astype(np.uint64) * weights).sum(axis=-1).astype(np.uint32)
            out["masks"] = packed
        else:
            out["masks"] = masks
    if return_lattice:
        out["lattice"] = lattice
    if return_endpoints:
        out["endpoints"] = endpoints
    if pixels is None:
        for key in ("ao", "gi", "ambient", "valid", "masks", "lattice", "endpoints"):
            if key in out:
                out[key] = out[key].reshape((H, W) + out[key].shape[1:])
    return out
