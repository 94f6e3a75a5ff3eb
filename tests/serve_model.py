"""Queueing model of the request loop on one stream, for the design analysis of its round
policy (run by tests/test_serve_model_cpu.py; `python tests/serve_model.py` prints the
table).

The served stream (gbuffer_scene.request_stream: resolution uniform over 960x540 to
3840x2160, 2-8 slices, 8/16/32 steps, Poisson arrivals) is replayed against a device that
takes c0 + samples / R seconds per launch, R calibrated so that the round policy saturates
at a measured rate.  Policies:
  rounds     the library's: when the stream is idle, every waiting request (up to 64)
             forms a round: the frames of at most 8,192 tiles packed into one launch, then
             the larger frames shortest first; each part retires when it ends
  one_large  every waiting small frame packed, then only the shortest waiting large frame;
             the other large frames wait for a later round
  one_oldest the same, with the oldest waiting large frame instead of the shortest
  budget     the small frames packed, then at most `budget` seconds of large-frame work
             (shortest remaining first), the rest resumed in later rounds (a persistent
             kernel that could stop and resume inside a frame)
Latency = completion of the request's last part - arrival."""
from __future__ import annotations

import numpy as np

PACK_TILES = 8192


def tiles(r):
    return ((r["width"] + 31) // 32) * ((r["height"] + 7) // 8)


def samples(r):
    return r["width"] * r["height"] * r["slices"] * 2 * r["steps"]


def simulate(reqs, arrivals, R, c0, policy="rounds", budget=None):
    """Completion time of every request (seconds) under `policy` on one stream."""
    n = len(reqs)
    work = np.array([samples(r) / R for r in reqs])
    small = np.array([tiles(r) <= PACK_TILES for r in reqs])
    done = np.full(n, np.nan)
    t, i = 0.0, 0
    waiting, carried = [], {}  # arrived and not started; large frames left for later rounds
    while i < n or waiting or carried:
        while i < n and arrivals[i] <= t:
            waiting.append(i)
            i += 1
        if not waiting and not carried:
            t = arrivals[i]
            continue
        rnd, waiting = waiting[:64], waiting[64:]
        sm = [j for j in rnd if small[j]]
        lg = [j for j in rnd if not small[j]]
        if sm:
            t += c0 + work[sm].sum()
            done[sm] = t
        if policy == "rounds":
            for j in sorted(lg, key=lambda j: work[j]):
                t += c0 + work[j]
                done[j] = t
        elif policy in ("one_large", "one_oldest"):
            for j in lg:
                carried[j] = work[j]
            if carried:
                # dicts keep insertion order: the first key is the oldest
                j = min(carried, key=lambda j: carried[j]) if policy == "one_large" else next(iter(carried))
                t += c0 + carried.pop(j)
                done[j] = t
        elif policy == "budget":
            for j in lg:
                carried[j] = work[j]
            left = budget
            for j in sorted(carried, key=lambda j: carried[j]):
                if left <= 0:
                    break
                take = min(carried[j], left)
                t += c0 + take
                left -= take
                carried[j] -= take
                if carried[j] <= 1e-12:
                    done[j] = t
                    del carried[j]
        else:
            raise ValueError(policy)
    return done


def saturated(reqs, R, c0, n=300, **kw):
    """Frames/s with the first n requests submitted at once."""
    d = simulate(reqs[:n], np.zeros(n), R, c0, **kw)
    return n / np.nanmax(d)


def calibrate(reqs, sat_fps, c0):
    """The device rate R (samples/s) at which the round policy saturates at `sat_fps`."""
    lo, hi = 1e9, 1e13
    for _ in range(80):
        R = (lo * hi) ** 0.5
        if saturated(reqs, R, c0) > sat_fps:
            hi = R
        else:
            lo = R
    return (lo * hi) ** 0.5


def latencies(reqs, R, c0, rate_hz, policy="rounds", budget=None, discard=200):
    """Latencies (ms) after the first `discard` requests, and their resolutions."""
    gaps = np.array([r["gap"] for r in reqs])
    arr = np.cumsum(gaps) / rate_hz
    arr -= arr[0]
    lat = (simulate(reqs, arr, R, c0, policy=policy, budget=budget) - arr) * 1e3
    res = np.array([f"{r['width']}x{r['height']}" for r in reqs])
    return lat[discard:], res[discard:]


def table(sat_fps=271.6, load=0.7, c0=1e-4):
    """Rows (policy, budget_ms, saturated fraction, p50, p99, p99 per resolution)."""
    from gbuffer_scene import request_stream
    reqs = request_stream()
    R = calibrate(reqs, sat_fps, c0)
    rows = []
    for pol, b in (("rounds", None), ("one_large", None), ("one_oldest", None), ("budget", 2e-3), ("budget", 5e-3),
                   ("budget", 10e-3), ("budget", 20e-3)):
        sat = saturated(reqs, R, c0, policy=pol, budget=b)
        lat, res = latencies(reqs, R, c0, load * sat_fps, policy=pol, budget=b)
        per = {k: float(np.percentile(lat[res == k], 99)) for k in sorted(set(res), key=lambda s: int(s.split("x")[0]))}
        rows.append((pol, None if b is None else b * 1e3, sat / sat_fps, float(np.percentile(lat, 50)),
                     float(np.percentile(lat, 99)), per))
    return R, rows


if __name__ == "__main__":
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    R, rows = table()
    print(f"device rate {R / 1e9:.0f} Gsamples/s")
    for pol, b, sat, p50, p99, per in rows:
        print(f"{pol:10s} {'' if b is None else f'{b:g} ms':6s} saturated {sat:.3f}  p50 {p50:6.2f}  p99 {p99:6.2f}  "
              + "  ".join(f"{k} {v:.1f}" for k, v in per.items()))
