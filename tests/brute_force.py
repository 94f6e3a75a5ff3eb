"""Brute-force occlusion of the thick-heightfield scene model, written independently of
the oracle (it imports nothing from it).

The scene model of Section 3.1 treats every depth sample as a segment of constant
thickness t behind the visible surface.  Along one slice of one pixel, the screen line
x(lambda) = (x + 1/2, y + 1/2) + s * lambda * (Dx, Dy) / 4096 crosses a run of texels;
a texel T of depth z_T, met for lambda in [la, lb], contributes every point
z_T * ray(x(lambda)) - tau * v with lambda in [la, lb] and tau in [0, t]: a
parallelogram in the slice plane (v is the unit vector from the pixel's surface point
toward the camera).  Seen from the pixel's point p it covers the angular span of its
four corners.  This module intersects the slice with that model exactly (union of
spans) instead of marching samples, and reports the occluded set as angles relative
to the projected normal, clipped to the hemisphere [-pi/2, pi/2].
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def _ray(cam, X, Y):
    fx, fy, cx, cy = cam
    return np.array([(X - cx) / fx, -(Y - cy) / fy, -1.0])


def slice_frame(cam, x, y, z_p, n_p, Dx, Dy):
    """Return p, v, e and gamma for pixel (x, y) and the screen direction (Dx, Dy)."""
    fx, fy, _, _ = cam
    rp = _ray(cam, x + 0.5, y + 0.5)
    p = z_p * rp
    v = -rp / np.linalg.norm(rp)
    d3 = np.array([Dx / (4096.0 * fx), -Dy / (4096.0 * fy), 0.0])
    w = np.cross(v, d3)
    e = np.cross(w, v)
    e = e / np.linalg.norm(e)
    nv, ne = float(np.dot(n_p, v)), float(np.dot(n_p, e))
    gamma = 0.0 if nv * nv + ne * ne < 1e-12 else math.atan2(ne, nv)
    return p, v, e, gamma


def texel_runs(x, y, Dx, Dy, s, lam_lo, lam_hi, W, H):
    """Texels met by the screen line for lambda in [lam_lo, lam_hi] on side s.

    A point belongs to the texel floor(X), floor(Y) (point sampling).  Membership is
    decided in exact rational arithmetic; a texel met at a single point (a range end on
    a texel edge, or a corner) is returned with la == lb.  Returns (X, Y, la, lb) tuples."""
    ox, oy = Fraction(2 * x + 1, 2), Fraction(2 * y + 1, 2)
    ux, uy = Fraction(s * Dx, 4096), Fraction(s * Dy, 4096)
    lo, hi = Fraction(lam_lo), Fraction(lam_hi)
    cuts = {lo, hi}
    for u, o in ((ux, ox), (uy, oy)):
        if u == 0:
            continue
        c0, c1 = o + lo * u, o + hi * u
        for k in range(math.floor(min(c0, c1)), math.floor(max(c0, c1)) + 1):
            lam = (k - o) / u
            if lo < lam < hi:
                cuts.add(lam)
    cuts = sorted(cuts)

    def texel(lam):
        return math.floor(ox + lam * ux), math.floor(oy + lam * uy)

    pieces = []
    for idx, lam in enumerate(cuts):
        pieces.append((texel(lam), lam, lam))
        if idx + 1 < len(cuts):
            pieces.append((texel((lam + cuts[idx + 1]) / 2), lam, cuts[idx + 1]))
    runs = []
    for (X, Y), la, lb in pieces:
        if not (0 <= X < W and 0 <= Y < H) or (X == x and Y == y):
            continue
        runs.append((X, Y, float(la), float(lb)))
    return runs


def occluded_intervals(depth, cam, x, y, n_p, Dx, Dy, t, lam_range_pos, lam_range_neg):
    """Union of the model's angular spans for both sides, as sorted disjoint intervals of
    theta (relative to the projected normal), clipped to [-pi/2, pi/2]."""
    H, W = depth.shape
    z_p = float(depth[y, x])
    p, v, e, gamma = slice_frame(cam, x, y, z_p, n_p, Dx, Dy)
    ivals = []
    for s, (lo, hi) in ((1, lam_range_pos), (-1, lam_range_neg)):
        if hi < lo:
            continue
        for X, Y, la, lb in texel_runs(x, y, Dx, Dy, s, lo, hi, W, H):
            zT = float(depth[Y, X])
            if not (math.isfinite(zT) and zT > 0):
                continue
            angs = []
            for lam in (la, lb):
                P = zT * _ray(cam, x + 0.5 + s * lam * Dx / 4096.0, y + 0.5 + s * lam * Dy / 4096.0) - p
                pv, pe = float(np.dot(P, v)), float(np.dot(P, e))
                angs.append(math.atan2(pe, pv))
                if math.isinf(t):
                    angs.append(math.copysign(math.pi, pe))
                else:
                    angs.append(math.atan2(pe, pv - t))
            a0, a1 = min(angs) - gamma, max(angs) - gamma
            a0, a1 = max(a0, -math.pi / 2), min(a1, math.pi / 2)
            if a1 > a0:
                ivals.append((a0, a1))
    ivals.sort()
    merged = []
    for a0, a1 in ivals:
        if merged and a0 <= merged[-1][1]:
            merged[-1] = (merged[-1][0], max(merged[-1][1], a1))
        else:
            merged.append((a0, a1))
    return merged, gamma


def is_occluded(intervals, theta, tol=1e-9):
    return any(a0 - tol <= theta <= a1 + tol for a0, a1 in intervals)


def occluded_measure(intervals):
    return sum(a1 - a0 for a0, a1 in intervals)
