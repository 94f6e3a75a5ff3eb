"""Row-band driver of the FP64 oracle: the same ``compute`` call on disjoint row bands of
a frame, one single-threaded forked process per band.

TEST INFRASTRUCTURE: used by the tests, the smoke check and the benchmark's CPU legs
(the timed baseline and the per-output error report).  It holds none of the method's
arithmetic: every value comes from ``ssvb_oracle.compute`` on the band's pixels, so a
frame split into bands gives exactly what one call over the frame would.

Call it before the process touches a GPU: the workers are forked.
"""
from __future__ import annotations

import os
import time

import numpy as np

from . import ssvb_oracle as O

_JOB = None  # (gbuffer, camera, params, return_masks), inherited by the forked workers


def _band(rows):
    from threadpoolctl import threadpool_limits
    gb, cam, prm, masks = _JOB
    W = gb["depth"].shape[1]
    ys = np.repeat(np.arange(rows[0], rows[1]), W)
    xs = np.tile(np.arange(W), rows[1] - rows[0])
    with threadpool_limits(1):
        t0 = time.perf_counter()
        r = O.compute(gb["depth"], gb["normal"], gb["radiance"], cam, prm, pixels=(ys, xs), return_masks=masks)
        return rows, time.perf_counter() - t0, r


def split_rows(r0, r1, parts):
    """[r0, r1) cut into at most ``parts`` bands of (nearly) equal height."""
    parts = max(1, min(parts, r1 - r0))
    edges = np.linspace(r0, r1, parts + 1).round().astype(int)
    return [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]


def compute_rows(gb, cam, prm, r0, r1, workers, return_masks=False, bands=None, threads=False):
    """The oracle on rows [r0, r1) of the frame, ``bands`` bands (default: ``workers``)
    on ``workers`` forked processes, or threads of this process with ``threads`` (for a
    process that already uses a GPU, which must not fork).  Returns (result, wall seconds,
    summed per-band seconds), result holding ``ao`` [rows, W], ``gi`` and ``ambient``
    [rows, W, 3] and, with ``return_masks``, ``masks`` [rows, W, ...] as the oracle returns
    them per pixel."""
    global _JOB
    import multiprocessing as mp
    W = gb["depth"].shape[1]
    rows = split_rows(r0, r1, bands or workers)
    _JOB = (gb, cam, prm, return_masks)
    t0 = time.perf_counter()
    try:
        if workers > 1 and len(rows) > 1 and threads:
            from concurrent.futures import ThreadPoolExecutor
            from threadpoolctl import threadpool_limits
            with threadpool_limits(1), ThreadPoolExecutor(min(workers, len(rows))) as ex:
                parts = list(ex.map(_band, rows))
        elif workers > 1 and len(rows) > 1:
            with mp.get_context("fork").Pool(min(workers, len(rows))) as p:
                parts = p.map(_band, rows)
        else:
            parts = [_band(r) for r in rows]
    finally:
        _JOB = None
    wall = time.perf_counter() - t0
    parts.sort(key=lambda t: t[0][0])
    out = {}
    for key in ("ao", "gi", "ambient") + (("masks",) if return_masks else ()):
        vals = [p[2][key] for p in parts]
        cat = np.concatenate(vals, axis=0)
        out[key] = cat.reshape((r1 - r0, W) + cat.shape[1:])
    return out, wall, float(sum(p[1] for p in parts))


def host_workers(limit=16):
    """Processes for a band run: the host's CPUs, at most ``limit``."""
    return max(1, min(limit, os.cpu_count() or 1))
