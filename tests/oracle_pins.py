"""Pins of the FP64 oracle against facts fixed by the paper's model and by geometry.

Each ``pin_*`` function takes an oracle module ``O`` (the real one, or a deliberately
broken copy in the mutation test) and raises AssertionError when the oracle disagrees
with an independent source of truth: closed forms of plane geometry, the GTAO horizon
integral that the infinite-thickness limit must reproduce (Section 3.1; Eqs. 2-3), the
analytic occluded fraction of an infinite wall, a brute-force intersection of the
thick-heightfield model (brute_force.py) and algebraic invariants of Algorithm 1.
None of these re-types the oracle's own formulas.
"""
from __future__ import annotations

import math

import numpy as np

import brute_force as BF
from gbuffer_scene import crease_gbuffer, make_camera, make_scene, plane_gbuffer, render_gbuffer

INF = float("inf")


# ----------------------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------------------

def ocam(O, cam):
    return O.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.view_to_world)


def const_sh(rgb):
    """SH coefficients of a constant probe of colour ``rgb``."""
    sh = np.zeros((9, 3))
    sh[0] = np.asarray(rgb) / (0.5 * math.sqrt(1.0 / math.pi))
    return tuple(sh.reshape(-1))


def bits_of(mask32, nb=32):
    return [(int(mask32) >> k) & 1 for k in range(nb)]


def popcount32(a):
    a = np.asarray(a, dtype=np.uint64)
    return np.array([bin(int(v)).count("1") for v in a.reshape(-1)]).reshape(a.shape)


def range_mask(a, b):
    """uint32 with bits [a, b) set (0 <= a, b <= 32)."""
    if b <= a:
        return 0
    return ((1 << b) - 1) ^ ((1 << a) - 1)


def integer_step_params(O, k_px, steps, **kw):
    """FIXED noise, two axis-aligned slices and steps of exactly ``k_px`` pixels, so every
    sample sits on a texel centre on the pixel's row (slice 0) or column (slice 1)."""
    return O.Params(slices=2, steps=steps, radius=1e6, max_radius_px=float(k_px * (steps + 1)),
                    noise=O.NOISE_FIXED, **kw)


_TINY = {}


def tiny_scene():
    """A 64x48 view into a dense box scene: objects, ground and some background sky."""
    if "s" not in _TINY:
        sc = make_scene(7, 40, 20)
        cam = make_camera(64, 48, fov_y_deg=60, pitch_deg=-25)
        gb = render_gbuffer(sc, cam, cache=False)
        _TINY["s"] = (gb, cam, sc)
    return _TINY["s"]


# ----------------------------------------------------------------------------------------
# P1: an unoccluded plane facing the camera sets no bit
# ----------------------------------------------------------------------------------------

def pin_plane_fronto(O):
    cam = make_camera(41, 31, fov_y_deg=90, pitch_deg=0)
    gb = plane_gbuffer(cam, (0, 0, 1), (0, 0, -4.0))
    C = (0.3, 0.5, 0.7)
    for t in (0.1, 0.5, INF):
        prm = O.Params(slices=3, steps=6, radius=1.5, thickness=t, noise=O.NOISE_HASH, seed=11,
                       ambient_sh=const_sh(C))
        r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm, return_masks=True)
        assert np.all(r["masks"] == 0), "a fronto-parallel plane must set no sector"
        assert np.all(r["ao"] == 1.0)
        assert np.all(r["gi"] == 0.0)
        assert np.allclose(r["ambient"], np.asarray(C), rtol=1e-7, atol=0)  # SH stored as float32


def pin_plane_tilted(O):
    """Tilted plane facing the camera, samples exactly on texel centres: no bits."""
    cam = make_camera(33, 25, fov_y_deg=90, pitch_deg=0)
    n = np.array([0.35, -0.3, 1.0])
    gb = plane_gbuffer(cam, n, (0, 0, -5.0))
    for t in (0.05, 0.7, INF):
        for k in (1, 3):
            prm = integer_step_params(O, k, 5, thickness=t)
            r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm, return_masks=True)
            assert np.all(r["masks"] == 0)
            assert np.all(r["ao"] == 1.0)
            assert np.all(r["gi"] == 0.0)


def pin_plane_ambient_linear(O):
    """Centre pixel of a fronto-parallel plane under a linear SH probe: the mean of the
    subregion directions is v / (N_a sin(pi / (2 N_a))), a closed form."""
    cam = make_camera(31, 31, fov_y_deg=90, pitch_deg=0)
    gb = plane_gbuffer(cam, (0, 0, 1), (0, 0, -3.0))
    rng = np.random.default_rng(5)
    R = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    if np.linalg.det(R) < 0:
        R[:, 0] = -R[:, 0]
    cam = cam.__class__(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                        tuple(float(np.float32(v)) for v in R.reshape(-1)))
    sh = np.zeros((9, 3))
    sh[0] = [0.2, 0.1, 0.3]
    sh[1:4] = rng.uniform(-0.5, 0.5, (3, 3))
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    y00 = 0.5 * math.sqrt(1.0 / math.pi)
    Rf = np.array([float(np.float32(v)) for v in R.reshape(-1)]).reshape(3, 3)
    shf = np.array([float(np.float32(v)) for v in sh.reshape(-1)]).reshape(9, 3)
    for na in (1, 2, 4, 8):
        prm = O.Params(slices=5, steps=4, radius=1.0, thickness=0.5, noise=O.NOISE_HASH, seed=3,
                       ambient_samples=na, ambient_sh=tuple(sh.reshape(-1)))
        r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm,
                      pixels=([15], [15]))
        dbar = Rf @ np.array([0.0, 0.0, 1.0]) / (na * math.sin(math.pi / (2 * na)))
        want = shf[0] * y00 + c1 * (shf[1] * dbar[1] + shf[2] * dbar[2] + shf[3] * dbar[0])
        assert np.allclose(r["ambient"][0], want, atol=1e-12), (na, r["ambient"][0], want)


def _real_sh_scipy(l, m, dirs):
    """Real spherical harmonic (l, m) from scipy's complex ones (which carry the
    Condon-Shortley phase): sqrt(2) (-1)^m Im Y_l^|m| for m < 0, Y_l^0, sqrt(2) (-1)^m Re
    Y_l^m for m > 0.  ``dirs`` [n, 3] unit vectors."""
    from scipy.special import sph_harm_y
    theta = np.arccos(np.clip(dirs[:, 2], -1.0, 1.0))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    if m < 0:
        return math.sqrt(2.0) * (-1) ** m * np.imag(sph_harm_y(l, -m, theta, phi))
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    return math.sqrt(2.0) * (-1) ** m * np.real(sph_harm_y(l, m, theta, phi))


SH_LM = [(0, 0), (1, -1), (1, 0), (1, 1), (2, -2), (2, -1), (2, 0), (2, 1), (2, 2)]  # index l^2 + l + m


def _fibonacci_sphere(n):
    k = np.arange(n) + 0.5
    z = 1.0 - 2.0 * k / n
    r = np.sqrt(1.0 - z * z)
    ph = math.pi * (3.0 - math.sqrt(5.0)) * k
    return np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1)


def pin_sh_basis(O):
    """The ambient probe's nine basis functions are scipy's real spherical harmonics of
    degree 0-2 in the order l^2 + l + m (values at random directions), and they are
    orthonormal over the sphere (FP64 quadrature on a 20,000-point Fibonacci grid)."""
    rng = np.random.default_rng(17)
    d = rng.normal(size=(64, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    for i, (l, m) in enumerate(SH_LM):
        c = np.zeros((9, 3))
        c[i] = (1.0, -2.0, 0.5)
        got = O.sh_eval(c, d)
        want = _real_sh_scipy(l, m, d)
        for ch, s in enumerate((1.0, -2.0, 0.5)):
            assert np.allclose(got[:, ch], s * want, atol=1e-12), (i, l, m, ch)
    g = _fibonacci_sphere(20000)
    Y = np.stack([O.sh_eval(np.eye(9)[i][:, None] * np.ones((1, 3)), g)[:, 0] for i in range(9)])
    gram = Y @ Y.T * (4.0 * math.pi / g.shape[0])
    assert np.allclose(gram, np.eye(9), atol=1e-4), np.abs(gram - np.eye(9)).max()


def _sh_quadratic_form(l, m):
    """Constant c and symmetric Q with Y_lm(a) = c + a^T Q a on the unit sphere (least squares
    on scipy's values; for l <= 2 the fit is exact)."""
    rng = np.random.default_rng(3)
    d = rng.normal(size=(40, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    A = np.stack([np.ones_like(x), x, y, z, x * x, y * y, z * z, 2 * x * y, 2 * y * z, 2 * x * z], axis=1)
    sol = np.linalg.lstsq(A, _real_sh_scipy(l, m, d), rcond=None)[0]
    assert np.allclose(A @ sol, _real_sh_scipy(l, m, d), atol=1e-12)
    c, lin = sol[0], sol[1:4]
    Q = np.array([[sol[4], sol[7], sol[9]], [sol[7], sol[5], sol[8]], [sol[9], sol[8], sol[6]]])
    return c, lin, Q


def pin_plane_ambient_quadratic(O):
    """Centre pixel of a fronto-parallel plane (nothing occluded, projected normal = v),
    FIXED noise so the N_d slices lie at i pi / N_d, under probes with quadratic terms.  The
    subregion directions are a_k = cos(b_k) v + sin(b_k) e_i with b_k = -pi/2 + (k + 1/2)
    pi / N_a, so the mean over them of any function c + l.a + a^T Q a is c + mean(cos b)
    l.v + tr(Q M) with M = mean(cos^2 b) v v^T + mean(sin^2 b) mean_i(e_i e_i^T); for
    N_d >= 2 the slice tangents average to half the identity of the image plane.  The
    probe is evaluated in world space (a rotated to R a).  Tolerance: the direction table
    rounds each e_i by at most 2^-13 rad."""
    cam = make_camera(31, 31, fov_y_deg=90, pitch_deg=0)
    gb = plane_gbuffer(cam, (0, 0, 1), (0, 0, -3.0))
    rng = np.random.default_rng(23)
    R = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    if np.linalg.det(R) < 0:
        R[:, 0] = -R[:, 0]
    Rf = np.array([float(np.float32(v)) for v in R.reshape(-1)]).reshape(3, 3)
    cam = cam.__class__(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, tuple(Rf.reshape(-1)))
    forms = [_sh_quadratic_form(l, m) for (l, m) in SH_LM]
    v = np.array([0.0, 0.0, 1.0])
    probes = []
    for i in range(4, 9):  # one quadratic coefficient at a time
        sh = np.zeros((9, 3))
        sh[i] = rng.uniform(-1.0, 1.0, 3)
        probes.append(sh)
    probes.append(rng.uniform(-0.6, 0.6, (9, 3)))  # every band at once
    for nd in (2, 4):
        for na in (1, 2, 4):
            kk = np.arange(na)
            b = -0.5 * math.pi + (kk + 0.5) * math.pi / na
            mc, mc2, ms2 = np.cos(b).mean(), (np.cos(b) ** 2).mean(), (np.sin(b) ** 2).mean()
            M = mc2 * np.outer(v, v) + ms2 * 0.5 * np.diag([1.0, 1.0, 0.0])
            for sh in probes:
                shf = np.array([float(np.float32(x)) for x in sh.reshape(-1)]).reshape(9, 3)
                prm = O.Params(slices=nd, steps=4, radius=1.0, thickness=0.5, noise=O.NOISE_FIXED,
                               ambient_samples=na, ambient_sh=tuple(sh.reshape(-1)))
                r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm, pixels=([15], [15]))
                want = np.zeros(3)
                for i, (c, lin, Q) in enumerate(forms):
                    Qv = Rf.T @ Q @ Rf  # world direction = R a
                    val = c + mc * (lin @ (Rf @ v)) + np.trace(Qv @ M)
                    want += val * shf[i]
                scale = np.abs(shf).sum(axis=0)
                assert np.all(np.abs(r["ambient"][0] - want) <= 1e-3 * scale + 1e-12), \
                    (nd, na, r["ambient"][0], want)


# ----------------------------------------------------------------------------------------
# P2: infinite thickness reproduces the horizon (GTAO) integral
# ----------------------------------------------------------------------------------------

def _horizons_integer_lattice(gb, cam, k, steps, ys, xs):
    """GTAO horizon search on the two axis slices: for each pixel, slice and side, the
    maximum cosine between v and the direction to a valid sample (Jimenez et al.; the
    paper's Figure "SliceGTAO"), returned as theta relative to the projected normal,
    plus gamma.  Independent of the oracle: plain 3D geometry of texel centres."""
    depth = gb["depth"].astype(np.float64)
    nrm = gb["normal"][..., :3].astype(np.float64)
    H, W = depth.shape
    cam4 = (cam.fx, cam.fy, cam.cx, cam.cy)
    out = np.full((len(ys), 2, 2), np.nan)
    gam = np.zeros((len(ys), 2))
    for idx, (y, x) in enumerate(zip(ys, xs)):
        z_p = depth[y, x]
        for sl, (Dx, Dy) in enumerate(((4096, 0), (0, 4096))):
            p, v, e, g = BF.slice_frame(cam4, x, y, z_p, nrm[y, x], Dx, Dy)
            gam[idx, sl] = g
            for si, s in enumerate((1, -1)):
                best = -np.inf
                for j in range(steps):
                    X = x + s * k * (j + 1) * (1 if Dx else 0)
                    Y = y + s * k * (j + 1) * (1 if Dy else 0)
                    if not (0 <= X < W and 0 <= Y < H):
                        continue
                    z = depth[Y, X]
                    if not (np.isfinite(z) and z > 0):
                        continue
                    P = z * np.array([(X + 0.5 - cam.cx) / cam.fx, -(Y + 0.5 - cam.cy) / cam.fy, -1.0])
                    d = P - p
                    best = max(best, float(np.dot(d, v) / np.linalg.norm(d)))
                if best > -np.inf:
                    out[idx, sl, si] = s * math.acos(min(1.0, best)) - g
    return out, gam


def _horizon_case(O, nb):
    gb, cam, _ = tiny_scene()
    k, steps = 2, 6
    prm = integer_step_params(O, k, steps, thickness=INF, sectors=nb, ambient_samples=4)
    valid = np.argwhere(gb["depth"] > 0)
    sel = valid[:: max(1, len(valid) // 150)]
    ys, xs = sel[:, 0], sel[:, 1]
    r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm, pixels=(ys, xs),
                  return_masks=True)
    hz, gam = _horizons_integer_lattice(gb, cam, k, steps, ys, xs)
    return r, hz, gam


def pin_horizon_infinite_thickness(O):
    """t = inf: each side's mask is the sectors from its horizon to the hemisphere edge."""
    r, hz, _ = _horizon_case(O, 32)
    checked = 0
    for idx in range(hz.shape[0]):
        for sl in range(2):
            want = 0
            tie = False
            for si, s in enumerate((1, -1)):
                th = hz[idx, sl, si]
                if np.isnan(th):
                    continue
                th = min(max(th, -math.pi / 2), math.pi / 2)
                x = 32 * (th + math.pi / 2) / math.pi + 0.5
                if abs(x - round(x)) < 1e-7:
                    tie = True
                a = math.floor(x)
                want |= range_mask(a, 32) if s == 1 else range_mask(0, a)
            if tie:
                continue
            assert int(r["masks"][idx, sl]) == want, (idx, sl, hex(int(r["masks"][idx, sl])), hex(want))
            checked += 1
    assert checked > 200


def pin_horizon_uniform_integral(O):
    """t = inf: per slice, the unoccluded fraction equals the visible arc between the two
    horizons over pi (uniform sectors, Eq. 4), within one sector at N_b = 32 and 1024."""
    for nb in (32, 1024):
        r, hz, _ = _horizon_case(O, nb)
        m = r["masks"]
        for idx in range(hz.shape[0]):
            for sl in range(2):
                hi = hz[idx, sl, 0]
                lo = hz[idx, sl, 1]
                hi = math.pi / 2 if np.isnan(hi) else min(max(hi, -math.pi / 2), math.pi / 2)
                lo = -math.pi / 2 if np.isnan(lo) else min(max(lo, -math.pi / 2), math.pi / 2)
                vis = max(0.0, hi - lo) / math.pi
                if nb == 32:
                    occ = bin(int(m[idx, sl])).count("1")
                else:
                    occ = int(m[idx, sl].sum())
                assert abs((1 - occ / nb) - vis) <= 1.0 / nb + 1e-12, (nb, idx, sl, 1 - occ / nb, vis)


def _edge_u(th, delta=1e-9):
    """(u, tie) of an angle th from the projected normal: u = (th + pi/2)/pi after clamping
    to the hemisphere; an angle within delta of an edge is a tie (rounding decides on
    which side it falls)."""
    if th <= -math.pi / 2 - delta:
        return 0.0, False
    if th >= math.pi / 2 + delta:
        return 1.0, False
    if abs(th + math.pi / 2) <= delta or abs(th - math.pi / 2) <= delta:
        return None, True
    return (th + math.pi / 2) / math.pi, False


def pin_pseudocode_horizon(O):
    """PSEUDOCODE criterion (Algorithm 1: floor of the start, ceil of the width), t = inf:
    a + side sample covers [theta_f, pi/2], so it sets [floor(N_b u_f), floor(N_b u_f) +
    ceil(N_b (1 - u_f))) = [floor(N_b u_f), N_b); a - side sample covers [-pi/2, theta_f]
    and sets [0, ceil(N_b u_f)).  Per slice the mask is therefore the + side horizon's
    [floor, N_b) and the - side horizon's [0, ceil), with the horizons from the
    independent GTAO search (plain 3D geometry of texel centres)."""
    gb, cam, _ = tiny_scene()
    k, steps = 2, 6
    prm = integer_step_params(O, k, steps, thickness=INF, hit_criterion=O.PSEUDOCODE)
    valid = np.argwhere(gb["depth"] > 0)
    sel = valid[:: max(1, len(valid) // 300)]
    ys, xs = sel[:, 0], sel[:, 1]
    r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm, pixels=(ys, xs),
                  return_masks=True)
    hz, _ = _horizons_integer_lattice(gb, cam, k, steps, ys, xs)
    checked = differs_from_round = 0
    for idx in range(hz.shape[0]):
        for sl in range(2):
            want, want_round, tie = 0, 0, False
            for si, s in enumerate((1, -1)):
                th = hz[idx, sl, si]
                if np.isnan(th):
                    continue
                u, t = _edge_u(th)
                if t:
                    tie = True
                    continue
                x = 32 * u
                if abs(x - round(x)) < 1e-7 or abs(x + 0.5 - round(x + 0.5)) < 1e-7:
                    tie = True
                if s == 1:
                    want |= range_mask(math.floor(x), 32)
                    want_round |= range_mask(math.floor(x + 0.5), 32)
                else:
                    want |= range_mask(0, math.ceil(x))
                    want_round |= range_mask(0, math.floor(x + 0.5))
            if tie:
                continue
            assert int(r["masks"][idx, sl]) == want, (idx, sl, hex(int(r["masks"][idx, sl])), hex(want))
            checked += 1
            differs_from_round += want != want_round
    assert checked > 200 and differs_from_round > 100, (checked, differs_from_round)


def pin_pseudocode_wall(O):
    """PSEUDOCODE on the crease (a wall rising at alpha from a plane facing the camera).
    Centre row, t = inf: the + side covers [floor(32 u), 32) from the highest wall
    sample's elevation.  Hinge pixel, finite t (and slope): every wall sample's front
    direction is the wall's, u_f = 1 - alpha/pi; the widest interval is the nearest
    sample's, up to its back angle atan2(l cos a, l sin a - t), so the mask is
    [floor(32 u_f), floor(32 u_f) + ceil(32 (u_b - u_f))).  The samples on the plane lie
    exactly in the pixel's tangent plane, on the - side's edge, where the ceiling of a
    zero width is decided by rounding: bit 0 of slice 0 and every bit of slice 1 (all on
    the plane) are left out, except that slice 1 may hold only edge bits."""
    size, D, k, steps = 41, 4.0, 2, 6
    c = size // 2
    checked = 0
    for deg in (30.0, 37.0, 45.0, 60.0):
        alpha = math.radians(deg)
        gb, cam = _crease(alpha, size, D)
        f = float(np.float32(cam.fx))
        prm = integer_step_params(O, k, steps, thickness=INF, hit_criterion=O.PSEUDOCODE)
        xs = np.arange(c - 12, c + 1)
        ys = np.full_like(xs, c)
        r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm,
                      pixels=(ys, xs), return_masks=True)
        for idx, x in enumerate(xs):
            z_p = float(gb["depth"][c, x])
            p = np.array([z_p * (x + 0.5 - c - 0.5) / f, 0.0, -z_p])
            beta = 0.0
            for j in range(steps):
                X = x + k * (j + 1)
                if X >= size:
                    break
                z = float(gb["depth"][c, X])
                P = np.array([z * (X + 0.5 - c - 0.5) / f, 0.0, -z])
                d = P - p
                beta = max(beta, math.atan2(d[2], d[0]))
            x32 = 32 * (1 - beta / math.pi)
            if beta == 0.0 or abs(x32 - round(x32)) < 1e-6:
                continue
            want = range_mask(math.floor(x32), 32)
            got = int(r["masks"][idx, 0])
            assert got & ~1 == want & ~1, (deg, x, hex(got), hex(want))
            assert int(r["masks"][idx, 1]) & ~((1 << 31) | 1) == 0
            checked += 1
        for t0, slope in ((0.02, 0.0), (0.1, 0.0), (0.3, 0.0), (0.8, 0.0), (0.0, 0.05), (0.1, 0.1)):
            t = t0 + slope * D
            prm = integer_step_params(O, k, steps, thickness=t0, thickness_slope=slope,
                                      hit_criterion=O.PSEUDOCODE)
            r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm,
                          pixels=([c], [c]), return_masks=True)
            X = c + k
            z = float(gb["depth"][c, X])
            d = np.array([z * (X - c) / f, 0.0, D - z])
            th_b = min(math.pi / 2, math.atan2(d[0], d[2] - t))
            u_f = 1 - alpha / math.pi
            u_b = (th_b + math.pi / 2) / math.pi
            a, wd = 32 * u_f, 32 * (u_b - u_f)
            if min(abs(a - round(a)), abs(wd - round(wd))) < 1e-6:
                continue
            lo = math.floor(a)
            want = range_mask(lo, min(lo + math.ceil(wd), 32))
            got = int(r["masks"][0, 0])
            assert got & ~1 == want & ~1, (deg, t, hex(got), hex(want))
            checked += 1
    assert checked > 40, checked


def gtao_inner(h1, h2, gamma):
    """GTAO's closed-form inner integral of cos(theta - gamma) |sin theta| over the
    visible arc [h1, h2] (h1 <= 0 <= h2, angles from v), Jimenez et al. 2016, which
    the paper's Eqs. 2-3 restate."""
    return 0.25 * (-math.cos(2 * h1 - gamma) + math.cos(gamma) + 2 * h1 * math.sin(gamma)) + \
        0.25 * (-math.cos(2 * h2 - gamma) + math.cos(gamma) + 2 * h2 * math.sin(gamma))


def _cos_weight(a, b, gamma):
    """Integral over theta_v in [a, b] of cos(theta_v - gamma) |sin theta_v|."""
    def F(t):  # antiderivative of cos(t - g) sin t
        return 0.5 * (t * math.sin(gamma) - 0.5 * math.cos(2 * t - gamma))
    total = 0.0
    for lo, hi, sgn in ((a, min(b, 0.0), -1.0), (max(a, 0.0), b, 1.0)):
        if hi > lo:
            total += sgn * (F(hi) - F(lo))
    return total


def pin_gtao_cosine_closed_form(O):
    """t = inf, N_b = 1024: the cosine-weighted popcount of unoccluded sectors matches
    GTAO's analytic horizon integral within two sectors' weight."""
    nb = 1024
    r, hz, gam = _horizon_case(O, nb)
    m = r["masks"]
    # the closed form itself agrees with quadrature
    for g in (-0.7, 0.0, 0.4):
        for h1, h2 in ((-0.3 + g, 0.5 + g), (g - math.pi / 2, g + math.pi / 2)):
            if h1 <= 0 <= h2:
                assert abs(gtao_inner(h1, h2, g) - _cos_weight(h1, h2, g)) < 1e-12
    for idx in range(hz.shape[0]):
        for sl in range(2):
            g = gam[idx, sl]
            hp = hz[idx, sl, 0]
            hm = hz[idx, sl, 1]
            h2 = g + (math.pi / 2 if np.isnan(hp) else min(max(hp, -math.pi / 2), math.pi / 2))
            h1 = g + (-math.pi / 2 if np.isnan(hm) else min(max(hm, -math.pi / 2), math.pi / 2))
            if not (h1 <= 0 <= h2):
                continue
            weights = [_cos_weight(g - math.pi / 2 + kk * math.pi / nb, g - math.pi / 2 + (kk + 1) * math.pi / nb, g)
                       for kk in range(nb)]
            got = sum(w for w, bit in zip(weights, m[idx, sl]) if not bit)
            want = gtao_inner(h1, h2, g)
            assert abs(got - want) <= 2 * max(weights) + 1e-9, (idx, sl, got, want)


# ----------------------------------------------------------------------------------------
# P3: an infinite wall at a known angle
# ----------------------------------------------------------------------------------------

def _crease(alpha, size=41, D=4.0):
    cam = make_camera(size, size, fov_y_deg=90, pitch_deg=0)
    return crease_gbuffer(cam, D, alpha), cam


def pin_wall_infinite_thickness(O):
    """Centre row of a crease (floor + wall rising at alpha beyond the hinge column), t = inf:
    the + side mask starts at the elevation of the highest wall sample above the floor."""
    size, D, k, steps = 41, 4.0, 2, 6
    c = size // 2
    for deg in (30.0, 37.0, 45.0, 60.0):
        alpha = math.radians(deg)
        gb, cam = _crease(alpha, size, D)
        prm = integer_step_params(O, k, steps, thickness=INF)
        xs = np.arange(c - 12, c + 1)
        ys = np.full_like(xs, c)
        r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm,
                      pixels=(ys, xs), return_masks=True)
        f = float(np.float32(cam.fx))
        for idx, x in enumerate(xs):
            z_p = float(gb["depth"][c, x])
            p = np.array([z_p * (x + 0.5 - c - 0.5) / f, 0.0, -z_p])
            beta = 0.0
            for j in range(steps):
                X = x + k * (j + 1)
                if X >= size:
                    break
                z = float(gb["depth"][c, X])
                P = np.array([z * (X + 0.5 - c - 0.5) / f, 0.0, -z])
                d = P - p
                beta = max(beta, math.atan2(d[2], d[0]))  # elevation above the floor
            xarg = 32 * (1 - beta / math.pi) + 0.5
            if abs(xarg - round(xarg)) < 1e-6:
                continue
            want = range_mask(math.floor(xarg), 32)
            assert int(r["masks"][idx, 0]) == want, (deg, x, hex(int(r["masks"][idx, 0])), hex(want))
            assert int(r["masks"][idx, 1]) == 0
            assert abs(r["ao"][idx] - (1 - bin(want).count("1") / 32 + 1) / 2) < 1e-15
        # the hinge pixel itself: the wall direction is exactly alpha above the floor
        a = math.floor(32 * (1 - alpha / math.pi) + 0.5)
        assert int(r["masks"][-1, 0]) == range_mask(a, 32)
    # alpha = 45 degrees at the hinge: AO = (0.75 + 1) / 2 exactly
    gb, cam = _crease(math.pi / 4, size, D)
    r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam),
                  integer_step_params(O, k, steps, thickness=INF), pixels=([c], [c]))
    assert r["ao"][0] == 0.875


def pin_wall_finite_thickness(O):
    """Hinge pixel, finite t: the occluded arc runs from the wall direction to the back
    angle of the nearest wall sample, atan2(l cos a, l sin a - t) (plane geometry)."""
    size, D, k, steps = 41, 4.0, 2, 6
    c = size // 2
    for deg in (35.0, 50.0):
        alpha = math.radians(deg)
        gb, cam = _crease(alpha, size, D)
        f = float(np.float32(cam.fx))
        X = c + k
        z = float(gb["depth"][c, X])
        d = np.array([z * (X - c) / f, 0.0, D - z])      # nearest wall sample minus p
        for t0, slope in ((0.02, 0.0), (0.1, 0.0), (0.3, 0.0), (0.8, 0.0), (0.0, 0.05), (0.1, 0.1)):
            t = t0 + slope * D       # thickness grows linearly with the pixel's depth
            prm = integer_step_params(O, k, steps, thickness=t0, thickness_slope=slope)
            r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm,
                          pixels=([c], [c]), return_masks=True)
            th_b = min(math.pi / 2, math.atan2(d[0], d[2] - t))
            a = math.floor(32 * (1 - alpha / math.pi) + 0.5)
            xb = 32 * (th_b + math.pi / 2) / math.pi + 0.5
            if abs(xb - round(xb)) < 1e-6:
                continue
            b = math.floor(xb)
            assert int(r["masks"][0, 0]) == range_mask(a, b), (deg, t, hex(int(r["masks"][0, 0])), a, b)


def pin_wall_indirect(O):
    """Floor pixels facing a lit wall, t = inf: GI is the sum over wall samples, near to
    far, of (newly covered sectors / N_b) (n_p . l) (-n_w . l), with the sectors from
    each sample's elevation above the floor and l, n_w from plane geometry."""
    size, D, k, steps = 41, 4.0, 2, 6
    c = size // 2
    for deg in (40.0, 65.0):
        alpha = math.radians(deg)
        gb, cam = _crease(alpha, size, D)
        prm = integer_step_params(O, k, steps, thickness=INF)
        xs = np.arange(c - 12, c)
        ys = np.full_like(xs, c)
        r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm, pixels=(ys, xs))
        f = float(np.float32(cam.fx))
        n_p = np.array([0.0, 0.0, 1.0])
        n_w = np.array([-math.sin(alpha), 0.0, math.cos(alpha)])
        tested = 0
        for idx, x in enumerate(xs):
            z_p = float(gb["depth"][c, x])
            p = np.array([z_p * (x - c) / f, 0.0, -z_p])
            covered_from = 32
            gi = 0.0
            tie = False
            for j in range(steps):
                X = x + k * (j + 1)
                z = float(gb["depth"][c, X])
                P = np.array([z * (X - c) / f, 0.0, -z])
                d = P - p
                beta = math.atan2(d[2], d[0])
                xa = 32 * (1 - beta / math.pi) + 0.5
                tie |= abs(xa - round(xa)) < 1e-6
                a = math.floor(xa)
                if a < covered_from:
                    l = d / np.linalg.norm(d)
                    gi += (covered_from - a) / 32 * max(0.0, n_p @ l) * max(0.0, -(n_w @ l))
                    covered_from = a
            if tie:
                continue
            want = gi / 2  # two slices; the other slice and the other side see only floor
            assert np.allclose(r["gi"][idx], want, rtol=1e-6, atol=1e-9), (deg, x, r["gi"][idx], want)
            tested += want > 0
        assert tested >= 5


def wall_ao_analytic(alpha):
    """1 - (2 / pi^2) * integral_0^{pi/2} atan(tan(alpha) cos(phi)) dphi (Simpson, FP64)."""
    n = 4000
    h = (math.pi / 2) / n
    s = 0.0
    for i in range(n + 1):
        w = 1 if i in (0, n) else (4 if i % 2 else 2)
        s += w * math.atan(math.tan(alpha) * math.cos(i * h))
    return 1.0 - (2.0 / math.pi ** 2) * (s * h / 3.0)


def pin_wall_random_rotations(O):
    """Hinge pixel, 64 randomly rotated slices, t = inf: AO converges to the wall's
    analytic occluded fraction."""
    size, D = 1201, 4.0
    c = size // 2
    for deg in (45.0, 25.0):
        alpha = math.radians(deg)
        gb, cam = _crease(alpha, size, D)
        ref = wall_ao_analytic(alpha)
        for seed in (0, 1):
            prm = O.Params(slices=64, steps=4, radius=4.0, thickness=INF, noise=O.NOISE_HASH, seed=seed)
            r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm, pixels=([c], [c]))
            assert abs(r["ao"][0] - ref) < 0.01, (deg, seed, r["ao"][0], ref)


# ----------------------------------------------------------------------------------------
# P4: brute force against the thick-heightfield model
# ----------------------------------------------------------------------------------------

def _bf_pixels(gb, count, seed):
    valid = np.argwhere(gb["depth"] > 0)
    rng = np.random.default_rng(seed)
    return valid[rng.choice(len(valid), size=min(count, len(valid)), replace=False)]


def pin_bruteforce_sound(O):
    """Every sector the oracle occludes has its centre inside the model's occluded set."""
    gb, cam, _ = tiny_scene()
    cam4 = (cam.fx, cam.fy, cam.cx, cam.cy)
    lut_dx = [math.floor(4096 * math.cos(math.pi * k / 4096) + 0.5) for k in range(4096)]
    lut_dy = [math.floor(4096 * math.sin(math.pi * k / 4096) + 0.5) for k in range(4096)]
    q, steps, nd = 24, 6, 8
    sel = _bf_pixels(gb, 60, 1)
    for t in (0.3, INF):
        prm = O.Params(slices=nd, steps=steps, radius=1e6, max_radius_px=q * (steps + 1) / 16.0,
                       thickness=t, noise=O.NOISE_FIXED)
        r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm,
                      pixels=(sel[:, 0], sel[:, 1]), return_masks=True)
        nset = 0
        for idx, (y, x) in enumerate(sel):
            for i in range(nd):
                kk = (i * 65536) // (16 * nd)
                lam = (q / 16.0, q * steps / 16.0)
                ivals, _ = BF.occluded_intervals(gb["depth"].astype(np.float64), cam4, x, y,
                                                 gb["normal"][y, x, :3].astype(np.float64),
                                                 lut_dx[kk], lut_dy[kk], t, lam, lam)
                m = int(r["masks"][idx, i])
                for bit in range(32):
                    if (m >> bit) & 1:
                        nset += 1
                        centre = -math.pi / 2 + (bit + 0.5) * math.pi / 32
                        assert BF.is_occluded(ivals, centre, 1e-7), (t, y, x, i, bit)
        assert nset > 100


def pin_bruteforce_converges(O):
    """With ever denser steps over a fixed reach and N_b = 1024, each slice's occluded
    fraction converges to the model's exact occluded measure."""
    gb, cam, _ = tiny_scene()
    cam4 = (cam.fx, cam.fy, cam.cx, cam.cy)
    depth = gb["depth"].astype(np.float64)
    sel = _bf_pixels(gb, 12, 2)
    reach_q4 = 16 * 10  # 10 px
    nb, t = 1024, 0.3
    errs = {}
    for q in (16, 4, 1):
        steps = reach_q4 // q
        prm = O.Params(slices=2, steps=steps, sectors=nb, radius=1e6, min_step_q4=1,
                       max_radius_px=q * (steps + 1) / 16.0, thickness=t, noise=O.NOISE_FIXED,
                       ambient_samples=4)
        r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm,
                      pixels=(sel[:, 0], sel[:, 1]), return_masks=True)
        e = []
        for idx, (y, x) in enumerate(sel):
            for i, (Dx, Dy) in enumerate(((4096, 0), (0, 4096))):
                lam = (q / 16.0, q * steps / 16.0)
                ivals, _ = BF.occluded_intervals(depth, cam4, x, y, gb["normal"][y, x, :3].astype(np.float64),
                                                 Dx, Dy, t, lam, lam)
                exact = BF.occluded_measure(ivals) / math.pi
                got = r["masks"][idx, i].sum() / nb
                e.append(abs(got - exact))
        errs[q] = (max(e), float(np.mean(e)))
    # the residual at 1/16 px comes from the first neighbour texel at grazing angles,
    # whose angular span changes fastest within one texel; it shrinks with the step
    assert errs[1][1] <= 0.01 and errs[1][0] <= 0.04, errs
    assert errs[1][1] < errs[4][1] < errs[16][1], errs


# ----------------------------------------------------------------------------------------
# P5: invariants of Algorithm 1
# ----------------------------------------------------------------------------------------

def pin_invariants(O):
    gb, cam, sc = tiny_scene()
    oc = ocam(O, cam)
    base = dict(slices=3, steps=5, radius=1.2, noise=O.NOISE_HASH, seed=9,
                ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    runs = {}
    for t in (0.1, 0.4, INF):
        runs[t] = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, O.Params(thickness=t, **base),
                            return_masks=True)
    r = runs[0.4]
    assert np.all((r["ao"] >= 0) & (r["ao"] <= 1))
    # the mask can only grow with thickness, so AO can only fall
    m1, m2, m3 = (runs[t]["masks"].astype(np.uint64) for t in (0.1, 0.4, INF))
    assert np.all((m1 & ~m2) == 0) and np.all((m2 & ~m3) == 0)
    assert np.all(runs[0.1]["ao"] >= r["ao"]) and np.all(r["ao"] >= runs[INF]["ao"])
    # GI is linear in radiance; AO and ambient do not depend on it
    r2 = O.compute(gb["depth"], gb["normal"], 2 * gb["radiance"], oc, O.Params(thickness=0.4, **base))
    assert np.array_equal(r2["gi"], 2 * r["gi"])
    assert np.array_equal(r2["ao"], r["ao"]) and np.array_equal(r2["ambient"], r["ambient"])
    r0 = O.compute(gb["depth"], gb["normal"], 0 * gb["radiance"], oc, O.Params(thickness=0.4, **base))
    assert np.all(r0["gi"] == 0)
    # sum over steps of new sectors = final occluded sectors, and each weight <= 1
    cmax = gb["radiance"][..., :3].max()
    assert np.all(r["gi"] <= cmax * (1 - r["ao"])[..., None] + 1e-12)
    assert np.all(r["gi"] >= 0)
    # a constant probe gives ambient = colour * AO
    C = (0.25, 0.5, 1.0)
    rc = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc,
                   O.Params(thickness=0.4, **{**base, "ambient_sh": const_sh(C)}))
    fg = gb["depth"] > 0
    assert np.allclose(rc["ambient"][fg], rc["ao"][fg][:, None] * np.asarray(C), rtol=1e-7, atol=1e-12)
    # background pixels
    bg = gb["depth"] <= 0
    assert bg.any()
    assert np.all(r["ao"][bg] == 1) and np.all(r["gi"][bg] == 0) and np.all(r["ambient"][bg] == 0)
    # occlusion exists in this scene
    assert r["ao"].min() < 0.8 and (r["gi"].max() > 0)


def pin_side_symmetry(O):
    """Mirroring the scene left-right mirrors every mask: the slice at phi maps to
    pi - phi and sector k of the mirrored slice is sector N_b - 1 - k."""
    gb, cam, _ = tiny_scene()
    W = cam.width
    # a horizontally mirrored G-buffer seen through the mirrored camera (cx -> W - cx)
    gbm = {"depth": gb["depth"][:, ::-1].copy(), "normal": gb["normal"][:, ::-1].copy(),
           "radiance": gb["radiance"][:, ::-1].copy()}
    gbm["normal"][..., 0] *= -1
    camm = cam.__class__(cam.width, cam.height, cam.fx, cam.fy, float(np.float32(W - cam.cx)), cam.cy,
                         cam.view_to_world)
    prm = integer_step_params(O, 2, 5, thickness=0.5)
    r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm, return_masks=True)
    rm = O.compute(gbm["depth"], gbm["normal"], gbm["radiance"], ocam(O, camm), prm, return_masks=True)
    rev = lambda m: int(format(int(m), "032b")[::-1], 2)
    # slice 0 (phi = 0) maps onto itself with its sides swapped: sector k -> N_b - 1 - k;
    # slice 1 (phi = pi/2, a column) maps onto itself unchanged
    diff0 = diff1 = 0
    for y in range(cam.height):
        for x in range(W):
            if rev(r["masks"][y, x, 0]) != int(rm["masks"][y, W - 1 - x, 0]):
                diff0 += 1
            if int(r["masks"][y, x, 1]) != int(rm["masks"][y, W - 1 - x, 1]):
                diff1 += 1
    assert diff0 <= 2 and diff1 <= 2, (diff0, diff1)
    assert (r["masks"] != 0).mean() > 0.2


# ----------------------------------------------------------------------------------------
# lattice and noise
# ----------------------------------------------------------------------------------------

def pin_lattice_geometry(O):
    """Sample texels lie on the slice line, ordered near to far, inside the projected
    radius, one step apart, with the jitter inside one step; the two sides mirror."""
    gb, cam, _ = tiny_scene()
    f = float(np.float32(cam.fy))
    for noise in (O.NOISE_FIXED, O.NOISE_HASH, O.NOISE_R2):
        for steps, radius in ((4, 0.6), (7, 1.5)):
            prm = O.Params(slices=4, steps=steps, radius=radius, thickness=0.5, noise=noise, seed=4)
            r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm,
                          return_lattice=True)
            L = r["lattice"].astype(np.float64)          # [H, W, nd, 2, ns, 2]
            H, W = gb["depth"].shape
            ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
            ctr = np.stack([xs, ys], -1)[:, :, None, None, None, :]
            off = L - ctr                                   # texel minus centre texel
            dist = np.linalg.norm(off, axis=-1)
            z = gb["depth"].astype(np.float64)
            rpx = np.where(z > 0, radius * f / np.where(z > 0, z, 1), 0)
            step = np.maximum(rpx / (steps + 1), 1.0)
            fg = z > 0
            # inside the projected radius, or N_s + 1 shortest steps when that is longer
            # (texel snapping adds at most one pixel diagonal)
            reach = step * (steps + 1)
            assert np.all(dist[fg] <= reach[fg][:, None, None, None] + 1.5)
            # step j sits between (j + 1) and (j + 2) steps out, within snapping
            j = np.arange(steps)[None, None, None, :]
            lo = (j + 1) * step[fg][:, None, None, None] - 1.5
            hi = (j + 2) * step[fg][:, None, None, None] + 1.5
            assert np.all((dist[fg] >= lo) & (dist[fg] <= hi))
            if noise == O.NOISE_FIXED:
                hi0 = (j + 1) * step[fg][:, None, None, None] + 1.5
                assert np.all(dist[fg] <= hi0)
            # the two sides are mirror images through the pixel centre (within snapping)
            assert np.all(np.abs(off[:, :, :, 0] + off[:, :, :, 1]) <= 1.0)
            # every side runs along one straight line through the centre
            far = off[:, :, :, :, -1, :]
            u = far / np.maximum(np.linalg.norm(far, axis=-1, keepdims=True), 1e-9)
            cross = np.abs(off[..., 0] * u[..., None, 1] - off[..., 1] * u[..., None, 0])
            assert np.all(cross[fg] <= 1.5)


def pin_quadratic_steps(O):
    """Quadratic step distribution (Section 4.3; reading R21): the sampled texels lie at
    ((j + 1 + xi) / (N_s + 1))^2 of the reach from the pixel (closed form of the law
    against the lattice; xi from the pinned noise), the steps inside half the reach are
    the first floor((N_s + 1) / sqrt 2) - 1, a plane facing the camera still sets no
    sector, and every sector occluded in the box scene lies in the model's occluded set."""
    gb, cam, _ = tiny_scene()
    H, W = gb["depth"].shape
    z = gb["depth"].astype(np.float64)
    fg = z > 0
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    for noise in (O.NOISE_FIXED, O.NOISE_HASH):
        steps, nd = 9, 3
        prm = O.Params(slices=nd, steps=steps, radius=1.5, thickness=0.5, noise=noise, seed=2,
                       step_distribution=O.STEPS_QUADRATIC, min_step_q4=1)
        r = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm, return_lattice=True)
        L = r["lattice"].astype(np.float64)                      # [H, W, nd, 2, ns, 2]
        off = L - np.stack([xs, ys], -1)[:, :, None, None, None, :]
        dist = np.linalg.norm(off, axis=-1)                      # [H, W, nd, 2, ns]
        q = O.step_q4(np.where(fg, z, 1.0), ocam(O, cam), prm).astype(np.float64)
        reach = q * (steps + 1) / 16.0                            # px
        _, xi8 = O.slice_noise(xs.reshape(-1), ys.reshape(-1), nd, noise, 2)
        xi = xi8.reshape(H, W, nd).astype(np.float64) / 256.0
        j = np.arange(steps)[None, None, None, None, :]
        u = (j + 1 + xi[:, :, :, None, None]) / (steps + 1)
        expect = reach[:, :, None, None, None] * u * u
        # texel snapping moves a sample by at most half a pixel diagonal (0.707), the
        # integer evaluation of the law by less than 1/16 px, the direction table's
        # rounding (|D| = 4096 within 0.71) by 1.7e-4 of the distance
        assert np.all(np.abs(dist - expect)[fg] <= 0.8)
    # the steps inside half the reach
    ns, q = 64, 1000
    o = np.array([O.step_offset_q4(q, 0, jj, ns, O.STEPS_QUADRATIC) for jj in range(ns)])
    assert np.all(np.diff(o) > 0)
    assert int(np.sum(o <= q * (ns + 1) / 2)) == int(math.floor((ns + 1) / math.sqrt(2.0)))
    # a plane facing the camera sets nothing
    camp = make_camera(41, 31, fov_y_deg=90, pitch_deg=0)
    gbp = plane_gbuffer(camp, (0, 0, 1), (0, 0, -4.0))
    for t in (0.1, INF):
        prm = O.Params(slices=3, steps=8, radius=1.5, thickness=t, noise=O.NOISE_HASH, seed=5,
                       step_distribution=O.STEPS_QUADRATIC)
        rp = O.compute(gbp["depth"], gbp["normal"], gbp["radiance"], ocam(O, camp), prm, return_masks=True)
        assert np.all(rp["masks"] == 0) and np.all(rp["ao"] == 1.0) and np.all(rp["gi"] == 0.0)
    # brute force: the samples lie between the first and the last step, so the model's
    # occluded set over that range contains every sector the oracle sets
    cam4 = (cam.fx, cam.fy, cam.cx, cam.cy)
    lut_dx = [math.floor(4096 * math.cos(math.pi * k / 4096) + 0.5) for k in range(4096)]
    lut_dy = [math.floor(4096 * math.sin(math.pi * k / 4096) + 0.5) for k in range(4096)]
    qq, steps, nd = 40, 6, 8
    offs = [O.step_offset_q4(qq, 0, jj, steps, O.STEPS_QUADRATIC) for jj in range(steps)]
    lam = (min(offs) / 16.0, max(offs) / 16.0)
    sel = _bf_pixels(gb, 40, 3)
    nset = 0
    for t in (0.3, INF):
        prm = O.Params(slices=nd, steps=steps, radius=1e6, max_radius_px=qq * (steps + 1) / 16.0,
                       thickness=t, noise=O.NOISE_FIXED, step_distribution=O.STEPS_QUADRATIC)
        rb = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), prm,
                       pixels=(sel[:, 0], sel[:, 1]), return_masks=True)
        for idx, (y, x) in enumerate(sel):
            for i in range(nd):
                kk = (i * 65536) // (16 * nd)
                ivals, _ = BF.occluded_intervals(gb["depth"].astype(np.float64), cam4, x, y,
                                                 gb["normal"][y, x, :3].astype(np.float64),
                                                 lut_dx[kk], lut_dy[kk], t, lam, lam)
                m = int(rb["masks"][idx, i])
                for bit in range(32):
                    if (m >> bit) & 1:
                        nset += 1
                        centre = -math.pi / 2 + (bit + 0.5) * math.pi / 32
                        assert BF.is_occluded(ivals, centre, 1e-7), (t, y, x, i, bit)
    assert nset > 50


def pin_half_resolution(O):
    """Half resolution (Section 4.3; reading R22): the computed pixels equal the full
    resolution gather there; on equal depths the upsampler reproduces a linear field
    exactly (bilinear interpolation); across a depth edge a pixel takes at most the weight
    floor from the far layer; background pixels and foreground pixels with no computed
    foreground neighbour take AO = 1, GI = 0, ambient = 0; a constant probe on a plane
    gives a constant ambient."""
    gb, cam, sc = tiny_scene()
    H, W = gb["depth"].shape
    kw = dict(slices=3, steps=6, radius=1.2, thickness=0.4, noise=O.NOISE_HASH, seed=3,
              ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    full = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), O.Params(**kw))
    half = O.compute(gb["depth"], gb["normal"], gb["radiance"], ocam(O, cam), O.Params(resolution=2, **kw))
    for k in ("ao", "gi", "ambient"):
        assert np.array_equal(half[k][0::2, 0::2], full[k][0::2, 0::2])
        assert np.all(np.isfinite(half[k]))
    # linear field on equal depths (9 x 7: odd sizes exercise the last row and column)
    Hh, Wh = 7, 9
    depth = np.full((Hh, Wh), 4.0, dtype=np.float32)
    yy, xx = np.meshgrid(np.arange(Hh, dtype=np.float64), np.arange(Wh, dtype=np.float64), indexing="ij")
    lin = 0.2 + 0.03 * xx - 0.05 * yy
    vec = np.stack([lin, 2 * lin, 0.5 - lin], -1)
    ev = np.zeros((Hh, Wh), bool)
    ev[0::2, 0::2] = True
    ao0 = np.where(ev, lin, -9.0)
    gi0 = np.where(ev[..., None], vec, -9.0)
    a, g, m = O.bilateral_upsample(depth, ao0, gi0, gi0.copy())
    inner = (xx <= 2 * ((Wh - 1) // 2)) & (yy <= 2 * ((Hh - 1) // 2))   # inside the computed hull
    assert np.allclose(a[inner], lin[inner], atol=1e-12, rtol=0)
    assert np.allclose(g[inner], vec[inner], atol=1e-12, rtol=0) and np.allclose(m[inner], vec[inner], atol=1e-12)
    # depth edge: near layer (z = 2) left of column 5, far layer (z = 10) from it on
    He, We = 5, 11
    depth = np.where(np.arange(We)[None, :] < 5, 2.0, 10.0).astype(np.float32) * np.ones((He, 1), np.float32)
    val = np.where(np.arange(We)[None, :] < 5, 0.0, 1.0) * np.ones((He, 1))
    a, g, _ = O.bilateral_upsample(depth, val.copy(), np.repeat(val[..., None], 3, -1),
                                   np.repeat(val[..., None], 3, -1))
    floor = O.UPSAMPLE_FLOOR
    assert np.all(np.abs(a - val) <= floor / (1 + floor) + 1e-15)
    # background and isolated foreground pixels
    depth = np.zeros((5, 5), np.float32)
    depth[1, 1] = 3.0                     # foreground with only background computed neighbours
    depth[4, 4] = 3.0                     # computed foreground pixel, not a neighbour of (1, 1)
    a, g, m = O.bilateral_upsample(depth, np.full((5, 5), 0.25), np.full((5, 5, 3), 0.5), np.full((5, 5, 3), 0.5))
    assert a[1, 1] == 1.0 and np.all(g[1, 1] == 0.0) and np.all(m[1, 1] == 0.0)
    assert a[0, 1] == 1.0 and np.all(g[0, 1] == 0.0)          # background
    assert a[4, 4] == 0.25                                     # computed pixel unchanged
    # a camera-facing plane under a constant probe: ambient = C at every pixel
    camp = make_camera(21, 15, fov_y_deg=90, pitch_deg=0)
    gbp = plane_gbuffer(camp, (0, 0, 1), (0, 0, -4.0))
    C = (0.3, 0.5, 0.7)
    rp = O.compute(gbp["depth"], gbp["normal"], gbp["radiance"], ocam(O, camp),
                   O.Params(slices=2, steps=5, radius=1.0, noise=O.NOISE_HASH, resolution=2, ambient_sh=const_sh(C)))
    assert np.all(rp["ao"] == 1.0) and np.all(rp["gi"] == 0.0)
    assert np.allclose(rp["ambient"], np.asarray(C), rtol=1e-7, atol=0)


def _atrous_kernel(s):
    """The 5 x 5 B3-spline kernel (1, 4, 6, 4, 1)/16 squared, taps spread s cells apart."""
    h = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0
    K = np.zeros((4 * s + 1, 4 * s + 1))
    K[::s, ::s] = np.outer(h, h)
    return K


def _label_pass(sig, labels, cross, s):
    """One pass of the expected filter where a tap's weight depends only on the labels of
    the pixel and the tap: out_p = sum_l C[L_p, l] corr(sig [L = l])_p / sum_l C[L_p, l]
    corr([L = l])_p, zero-padded correlations from scipy; label -1 is background (never a
    tap, keeps its input)."""
    from scipy.ndimage import correlate
    K = _atrous_kernel(s)
    out = sig.copy()
    n_l = cross.shape[0]
    num = np.zeros((n_l,) + sig.shape)
    den = np.zeros((n_l,) + labels.shape)
    for l in range(n_l):
        m = (labels == l).astype(np.float64)
        den[l] = correlate(m, K, mode="constant", cval=0.0)
        for c in range(sig.shape[-1]):
            num[l, ..., c] = correlate(sig[..., c] * m, K, mode="constant", cval=0.0)
    for lp in range(n_l):
        sel = labels == lp
        nn = sum(cross[lp, l] * num[l] for l in range(n_l))
        dd = sum(cross[lp, l] * den[l] for l in range(n_l))
        out[sel] = nn[sel] / dd[sel][..., None]
    return out


def _denoise_expected(sig, labels, cross, passes):
    for i in range(passes):
        sig = _label_pass(sig, labels, cross, 1 << i)
    return sig


def _run_denoise(O, gb, cam, sig, **kw):
    a, g, m = O.denoise(gb["depth"], gb["normal"], ocam(O, cam), sig[..., 0], sig[..., 1:4], sig[..., 4:7], **kw)
    return np.concatenate([a[..., None], g, m], -1)


def pin_denoise(O):
    """Denoising (reading R24) against scipy's normalised correlation: on a plane every tap
    weight is the kernel's, so each pass is the zero-padded correlation with the B3
    kernel spread 2^i apart, divided by the correlation of ones (fronto-parallel and
    tilted planes, 1 to 3 passes, both resolutions); across a depth step or a normal
    crease the weight falls to exp(-d^2) or max(0, n_p . n_q)^k per side; background
    pixels are never taps and keep their input; a constant image stays constant."""
    rng = np.random.default_rng(21)
    cam = make_camera(13, 11, fov_y_deg=90, pitch_deg=0)
    H, W = 11, 13
    sig = rng.uniform(0.0, 1.0, (H, W, 7))
    one = np.zeros((1, 1)) + 1.0
    # planes: fronto-parallel and tilted (every tap on the plane: plane distance 0)
    for nrm, P0 in (((0, 0, 1), (0, 0, -4.0)), ((0, 0.6, 0.8), (0, 0, -5.0)), ((0.3, -0.3, 0.8), (0, 0, -3.0))):
        gb = plane_gbuffer(cam, nrm, P0)
        assert np.all(gb["depth"] > 0)
        for passes in (1, 2, 3):
            got = _run_denoise(O, gb, cam, sig, passes=passes)
            want = _denoise_expected(sig, np.zeros((H, W), int), one, passes)
            assert np.allclose(got, want, atol=1e-9, rtol=0), (nrm, passes)
        # half resolution: the filter on the even/even grid, then the upsampler
        got = _run_denoise(O, gb, cam, sig, passes=2, resolution=2)
        grid = _denoise_expected(sig[::2, ::2], np.zeros(((H + 1) // 2, (W + 1) // 2), int), one, 2)
        assert np.allclose(got[::2, ::2], grid, atol=1e-9, rtol=0), nrm
        full = sig.copy()
        full[::2, ::2] = grid
        a, g, m = O.bilateral_upsample(gb["depth"], full[..., 0], full[..., 1:4], full[..., 4:7])
        assert np.allclose(got, np.concatenate([a[..., None], g, m], -1), atol=1e-12, rtol=0)
    # depth steps on fronto-parallel layers: far apart (no bleed) and close (Gaussian falloff)
    xs = np.arange(W)[None, :] * np.ones((H, 1))
    lab = (xs >= 6).astype(int)
    nz = np.zeros((H, W, 3), np.float32)
    nz[..., 2] = 1.0
    for z1, z2 in ((2.0, 3.0), (4.0, 4.2)):
        depth = np.where(lab == 0, z1, z2).astype(np.float32)
        zz = (float(np.float32(z1)), float(np.float32(z2)))
        sigma = float(np.float32(0.05))
        d01 = (zz[1] - zz[0]) / (sigma * zz[0])   # plane distance of a layer-1 tap from layer 0
        d10 = (zz[1] - zz[0]) / (sigma * zz[1])
        cross = np.array([[1.0, math.exp(-d01 * d01)], [math.exp(-d10 * d10), 1.0]])
        gb = {"depth": depth, "normal": nz}
        got = _run_denoise(O, gb, cam, sig, passes=2)
        assert np.allclose(got, _denoise_expected(sig, lab, cross, 2), atol=1e-9, rtol=0), (z1, z2)
    # normal creases at constant depth with the plane term off (sigma = inf): a tap of the
    # other normal weighs max(0, n_p . n_q)^k
    depth = np.full((H, W), 4.0, np.float32)
    for n2, kpow in (((0, 0.6, 0.8), 2), ((0, 0.6, 0.8), 0), ((0, -0.6, -0.8), 2), ((1, 0, 0), 3)):
        nrm = np.where((lab == 0)[..., None], (0.0, 0.0, 1.0), n2).astype(np.float32)
        c = max(0.0, float(np.dot(np.asarray(n2, np.float32).astype(np.float64), (0, 0, 1)) /
                           np.linalg.norm(np.asarray(n2, np.float32).astype(np.float64))))
        cross = np.array([[1.0, c ** kpow], [c ** kpow, 1.0]])
        gb = {"depth": depth, "normal": nrm}
        got = _run_denoise(O, gb, cam, sig, passes=2, normal_power=kpow, plane_sigma=float("inf"))
        assert np.allclose(got, _denoise_expected(sig, lab, cross, 2), atol=1e-9, rtol=0), (n2, kpow)
    # background hole and border: background keeps its input and is never a tap
    gb = plane_gbuffer(cam, (0, 0, 1), (0, 0, -4.0))
    depth = gb["depth"].copy()
    depth[3:6, 4:9] = 0.0
    depth[0, 0] = np.inf
    bg = (depth <= 0) | ~np.isfinite(depth)
    lab = np.where(bg, -1, 0)
    for sigma in (0.05, float("inf")):   # with the plane term off only the exclusion keeps them out
        got = _run_denoise(O, dict(gb, depth=depth), cam, sig, passes=2, plane_sigma=sigma)
        assert np.array_equal(got[bg], sig[bg])
        assert np.allclose(got, _denoise_expected(sig, lab, one, 2), atol=1e-9, rtol=0), sigma
    # a constant image on a real scene stays constant
    gbs, cams, _ = tiny_scene()
    Hs, Ws = gbs["depth"].shape
    const = np.broadcast_to(np.array([0.7, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6]), (Hs, Ws, 7)).copy()
    for res in (1, 2):
        got = _run_denoise(O, gbs, cams, const, passes=3, resolution=res)
        fgs = np.isfinite(gbs["depth"]) & (gbs["depth"] > 0)
        assert np.allclose(got[fgs], const[fgs], atol=1e-12, rtol=0), res


def pin_multi_bounce(O):
    """Multi-bounce (Section 4.3; reading R23): gain 0 or zero GI leaves the direct light;
    GI is linear and non-negative in the light buffer, so feeding it back frame after
    frame on the crease (floor facing a lit wall, fixed seed) makes each pixel's GI grow
    monotonically, with positive increments that shrink (a contraction: gain x albedo
    x coupling < 1) to a fixed point."""
    cam = make_camera(48, 32, fov_y_deg=70, pitch_deg=-30)
    gb = crease_gbuffer(cam, D=3.0, alpha=math.radians(60))
    d = gb["radiance"].astype(np.float64)
    albedo = np.full(d.shape, 0.7)
    gi0 = np.ones(d.shape[:2] + (3,))
    assert np.array_equal(O.inject_bounce(d, albedo, gi0, 0.0), d[..., :3])
    assert np.array_equal(O.inject_bounce(d, albedo, 0 * gi0, 0.8), d[..., :3])
    # a black surface reflects nothing; the reflected part scales with the albedo
    assert np.array_equal(O.inject_bounce(d, 0 * albedo, gi0, 0.8), d[..., :3])
    half = O.inject_bounce(d, 0.5 * albedo, gi0, 0.8) - d[..., :3]
    assert np.allclose(O.inject_bounce(d, albedo, gi0, 0.8) - d[..., :3], 2 * half, rtol=1e-14, atol=0)
    prm = O.Params(slices=4, steps=8, radius=2.0, thickness=INF, noise=O.NOISE_FIXED)
    light = gb["radiance"]
    sums, prev = [], None
    for _ in range(6):
        r = O.compute(gb["depth"], gb["normal"], light, ocam(O, cam), prm)
        gi = r["gi"]
        if prev is not None:
            assert np.all(gi >= prev - 1e-12)       # more light never lowers GI
        prev = gi
        sums.append(gi.sum())
        light = O.inject_bounce(gb["radiance"], albedo, gi, 0.9)
    inc = np.diff(sums)
    assert sums[0] > 0 and np.all(inc > 0)
    assert np.all(inc[1:] / inc[:-1] < 1.0)
    assert inc[-1] < 1e-6 * sums[-1]


def pin_bounce_sequence(O):
    """Frame sequences (Section 4.3 multi-bounce, temporal jitter; reading R25).
    (1) Gain 0: frame n is the single-frame gather of the direct light with seed s0 + n,
    and the frames differ.  (2) The integral distributed over time: one randomly turned
    slice per frame at the hinge of a 45-degree wall, averaged over 256 frames, reaches the
    wall's analytic occluded fraction, like 64 slices in one frame.  (3) Feedback: frame
    n's light is direct + gain x albedo x GI of frame n - 1 (then rounded to the light
    buffer's FP16 when asked), and on the lit crease with FIXED noise the GI grows frame
    after frame to a fixed point (in FP16 storage once the increments fall below its
    resolution)."""
    gb, cam, sc = tiny_scene()
    oc = ocam(O, cam)
    H, W = gb["depth"].shape
    albedo = np.full((H, W, 3), 0.6, np.float32)
    frames = [dict(depth=gb["depth"], normal=gb["normal"], direct=gb["radiance"], albedo=albedo)] * 3
    prm = O.Params(slices=2, steps=6, radius=1.5, thickness=0.4, noise=O.NOISE_HASH, seed=7,
                   ambient_sh=tuple(sc.ambient_sh.reshape(-1)))
    seq = O.bounce_sequence(frames, oc, prm, 0.0)
    for n, r in enumerate(seq):
        from dataclasses import replace
        one = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, replace(prm, seed=7 + n))
        for k in ("ao", "gi", "ambient"):
            assert np.array_equal(r[k], one[k]), (n, k)
    assert not np.array_equal(seq[0]["ao"], seq[1]["ao"]), "the slices must turn from frame to frame"
    # (2) temporal distribution of the integral
    alpha = math.radians(45.0)
    cgb, ccam = _crease(alpha, 41, 4.0)
    c = 20
    ref = wall_ao_analytic(alpha)
    cframes = [dict(depth=cgb["depth"], normal=cgb["normal"], direct=cgb["radiance"],
                    albedo=np.full(cgb["radiance"].shape, 0.5, np.float32))] * 256
    for seed in (5, 1000):
        cprm = O.Params(slices=1, steps=4, radius=4.0, thickness=INF, noise=O.NOISE_HASH, seed=seed)
        ao = np.array([r["ao"][c, c] for r in O.bounce_sequence(cframes, ocam(O, ccam), cprm, 0.0)])
        assert abs(ao.mean() - ref) < 0.012, (seed, ao.mean(), ref)
        assert ao.std() > 0.01  # single frames really differ
    # (3) feedback through the light buffer
    wcam = make_camera(48, 32, fov_y_deg=70, pitch_deg=-30)
    wgb = crease_gbuffer(wcam, D=3.0, alpha=math.radians(60))
    walb = np.full(wgb["radiance"].shape, 0.7, np.float32)
    wframes = [dict(depth=wgb["depth"], normal=wgb["normal"], direct=wgb["radiance"], albedo=walb)] * 6
    wprm = O.Params(slices=4, steps=8, radius=2.0, thickness=INF, noise=O.NOISE_FIXED)
    for dt in (np.float32, np.float16):
        wseq = O.bounce_sequence(wframes, ocam(O, wcam), wprm, 0.9, light_dtype=dt)
        d = wgb["radiance"].astype(np.float64)
        assert np.array_equal(wseq[0]["light"], d.astype(dt))
        for n in range(1, 6):
            want = (d + np.float64(np.float32(0.9)) * walb.astype(np.float64) * wseq[n - 1]["gi"]).astype(dt)
            assert np.array_equal(wseq[n]["light"], want), (dt, n)
        sums = [r["gi"].sum() for r in wseq]
        inc = np.diff(sums)
        if dt == np.float32:
            assert sums[0] > 0 and np.all(inc > 0) and np.all(inc[1:] < inc[:-1]), (dt, sums)
        else:  # FP16 storage rounds the small late increments away: the fixed point comes sooner
            assert sums[0] > 0 and inc[0] > 0 and np.all(inc >= 0) and inc[-1] == 0, (dt, sums)


def pin_noise_statistics(O):
    """Rotations and jitters are uniform (chi-square) and the slices of one pixel are
    spread evenly over pi; the R2 rotation is a low-discrepancy dither."""
    H, W = 64, 64
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    for noise in (O.NOISE_HASH, O.NOISE_R2):
        rho, xi = O.slice_noise(xs.reshape(-1), ys.reshape(-1), 3, noise, 17)
        assert rho.min() >= 0 and rho.max() < 65536 and xi.min() >= 0 and xi.max() < 256
        for vals, top in ((rho, 65536), (xi[:, 1], 256)):
            hist = np.bincount((vals * 16 // top).astype(np.int64), minlength=16)
            exp = len(vals) / 16
            chi2 = ((hist - exp) ** 2 / exp).sum()
            assert chi2 < 40, (noise, chi2)
        if noise == O.NOISE_R2:
            # every 4x4 block holds rotations spread over the whole circle
            blk = rho.reshape(H // 4, 4, W // 4, 4).transpose(0, 2, 1, 3).reshape(-1, 16)
            srt = np.sort(blk, axis=1)
            gaps = np.diff(np.concatenate([srt, srt[:, :1] + 65536], axis=1), axis=1)
            assert gaps.max() <= 65536 * 0.25
    # the direction table: endpoints, symmetry, unit length
    dx, dy = O.direction_lut()
    assert (dx[0], dy[0], dx[2048], dy[2048]) == (4096, 0, 0, 4096)
    assert np.all(dx[1:] == -dx[:0:-1]) and np.all(dy[1:] == dy[:0:-1])
    assert np.all(np.abs(np.hypot(dx, dy) - 4096) <= 0.71)
    assert np.all(np.diff(dx) <= 0) and np.all(dy[:2049] == np.maximum.accumulate(dy[:2049]))
    # R2 constants: 2^32 / a1 solves g^3 = g + 1 and a2 = 2^32 / g^2
    a1, a2, a3 = O.r2_constants()
    g = 2.0 ** 32 / a1
    assert abs(g ** 3 - g - 1) < 1e-8 and abs(a2 - 2.0 ** 32 / g ** 2) < 2 and a3 == 0x9E3779B9
    # steps: the march never reaches past the projected radius
    cam = O.Camera(64, 64, 32.0, 32.0, 32.0, 32.0)
    for ns in (1, 8, 31):
        prm = O.Params(steps=ns, radius=1.7)
        z = np.geomspace(0.05, 500, 2000).astype(np.float32)
        q = O.step_q4(z, cam, prm)
        rpx = 1.7 * 32.0 / z.astype(np.float64)
        free = (q > 16) & (q < (16 * 16383) // (ns + 1))
        assert np.all(q[free] * (ns + 1) / 16.0 <= rpx[free] * (1 + 1e-6))
        assert np.all(q[free] * (ns + 1) / 16.0 >= rpx[free] - (ns + 1) / 16.0 - 1e-6)


ALL_PINS = [
    pin_plane_fronto,
    pin_plane_tilted,
    pin_plane_ambient_linear,
    pin_sh_basis,
    pin_plane_ambient_quadratic,
    pin_horizon_infinite_thickness,
    pin_horizon_uniform_integral,
    pin_gtao_cosine_closed_form,
    pin_wall_infinite_thickness,
    pin_wall_finite_thickness,
    pin_pseudocode_horizon,
    pin_pseudocode_wall,
    pin_wall_indirect,
    pin_wall_random_rotations,
    pin_bruteforce_sound,
    pin_bruteforce_converges,
    pin_invariants,
    pin_side_symmetry,
    pin_lattice_geometry,
    pin_noise_statistics,
    pin_quadratic_steps,
    pin_half_resolution,
    pin_multi_bounce,
    pin_bounce_sequence,
    pin_denoise,
]
