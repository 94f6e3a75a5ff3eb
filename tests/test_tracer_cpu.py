"""CPU tests of the mismatch tracer that holds GPU and host-build results to the oracle
(parity.compare / explain_pixel).  The "device" results here are the oracle's own, with
chosen roundings flipped through its index bias, so every case's right answer is known:
a flip of a near-tie endpoint (a floor just above an integer, a ceiling of a width that
is exactly zero, one tie among dozens in a slice) must be explained; a sector bit set far
from any tie, or an output moved by more than the tolerance, must not be."""
import numpy as np
import pytest

import oracle as O
import parity as PY


def _device_like(gb, oc, op):
    """Oracle results in the device's layout: [H, W] / [H, W, 3] outputs and packed masks."""
    H, W = gb["depth"].shape
    r = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, return_masks=True)
    m = r["masks"].reshape((H * W,) + r["masks"].shape[2:])
    out = {k: r[k].astype(np.float32) for k in ("ao", "gi", "ambient")}
    out["masks"] = PY.packed_masks(m).reshape(H, W, -1)
    return out, r


def _flipped(gb, oc, op, y, x, bias):
    r = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, pixels=([y], [x]), return_masks=True,
                  index_bias=bias[None])
    return {"ao": r["ao"][0], "gi": r["gi"][0], "ambient": r["ambient"][0], "masks": PY.packed_masks(r["masks"])[0]}


def _put(dev, y, x, res):
    for k in ("ao", "gi", "ambient", "masks"):
        dev[k][y, x] = res[k]


def _ties(gb, oc, op, y, x):
    r = O.compute(gb["depth"], gb["normal"], gb["radiance"], oc, op, pixels=([y], [x]), return_endpoints=True)
    ep = r["endpoints"][0]
    return ep, PY._near_ties(ep, op)


def _mask_changing_flip(gb, oc, op, dev, y, x, want):
    """A single near-tie flip at (y, x) that changes the pixel's masks and satisfies
    ``want(endpoint value, position)``; None if there is none."""
    ep, near = _ties(gb, oc, op, y, x)
    for pos, d in near:
        if not want(ep[pos], pos):
            continue
        bias = np.zeros(ep.shape, np.int64)
        bias[pos] = d
        res = _flipped(gb, oc, op, y, x, bias)
        if not np.array_equal(res["masks"], dev["masks"][y, x]):
            return res
    return None


@pytest.fixture(scope="module")
def edge_frame():
    """A frame of axis-aligned planes under PSEUDOCODE where rows of samples lie exactly in
    a pixel's tangent plane (the seeded random case 26 of the host-build tests)."""
    gb, cam, kw = PY.random_case(np.random.default_rng(1026))
    _, oc = PY.cams(cam)
    _, op = PY.params(**kw)
    assert op.hit_criterion == O.PSEUDOCODE
    dev, _ = _device_like(gb, oc, op)
    return gb, oc, op, dev


def test_exact_zero_width_ceiling_is_explained(edge_frame):
    gb, oc, op, dev0 = edge_frame
    H, W = gb["depth"].shape
    done = 0
    for y in range(H):
        for x in range(W):
            dev = {k: v.copy() for k, v in dev0.items()}
            res = _mask_changing_flip(gb, oc, op, dev, y, x, lambda v, pos: pos[-1] == 1 and v == 0.0)
            if res is None:
                continue
            _put(dev, y, x, res)
            rep = {}
            PY.compare(dev, {k: v for k, v in _device_like(gb, oc, op)[1].items()}, gb, oc, op, report=rep,
                       agreement=0.0)
            assert rep["mismatched_pixels"] >= 1 and rep["explained"] == rep["mismatched_pixels"]
            done += 1
            if done == 3:
                return
    pytest.fail("no pixel with a zero width at a tie")


def test_one_of_many_ties_is_explained(edge_frame):
    """A pixel with more than 10 near ties takes the per-slice search."""
    gb, oc, op, dev0 = edge_frame
    H, W = gb["depth"].shape
    for y in range(H):
        for x in range(W):
            ep, near = _ties(gb, oc, op, y, x)
            if len(near) <= 10:
                continue
            dev = {k: v.copy() for k, v in dev0.items()}
            # flip the last tie in march order that changes the masks
            for pos, d in reversed(near):
                bias = np.zeros(ep.shape, np.int64)
                bias[pos] = d
                res = _flipped(gb, oc, op, y, x, bias)
                if not np.array_equal(res["masks"], dev["masks"][y, x]):
                    break
            else:
                continue
            _put(dev, y, x, res)
            assert PY.explain_pixel(dev, gb, oc, op, y, x, PY.TOL_FP32)
            return
    pytest.fail("no pixel with more than 10 near ties whose flip changes its masks")


def test_bit_far_from_any_tie_is_not_explained(edge_frame):
    gb, oc, op, dev0 = edge_frame
    H, W = gb["depth"].shape
    nb = op.sectors
    for y in range(H):
        for x in range(W):
            ep, near = _ties(gb, oc, op, y, x)
            if not near or not np.isfinite(ep).any():
                continue
            # a sector of slice 0 at least 3 sectors from every finite endpoint's boundaries
            e = ep[0][np.isfinite(ep[0])]
            cand = [k for k in range(nb) if np.all(np.abs(e - k) > 3) and np.all(np.abs(e - (k + 1)) > 3)]
            if not cand:
                continue
            dev = {k: v.copy() for k, v in dev0.items()}
            k = cand[len(cand) // 2]
            dev["masks"][y, x, k // 32] ^= np.uint32(1 << (k % 32))
            assert not PY.explain_pixel(dev, gb, oc, op, y, x, PY.TOL_FP32)
            return
    pytest.fail("no pixel to plant a bit in")


def test_output_beyond_tolerance_is_not_explained(edge_frame):
    gb, oc, op, dev0 = edge_frame
    H, W = gb["depth"].shape
    for y in range(H):
        for x in range(W):
            dev = {k: v.copy() for k, v in dev0.items()}
            res = _mask_changing_flip(gb, oc, op, dev, y, x, lambda v, pos: True)
            if res is None:
                continue
            res["ao"] = res["ao"] + 2 * PY.TOL_FP32
            _put(dev, y, x, res)
            assert not PY.explain_pixel(dev, gb, oc, op, y, x, PY.TOL_FP32)
            ref = _device_like(gb, oc, op)[1]
            with pytest.raises(AssertionError, match="unexplained"):
                PY.compare(dev, ref, gb, oc, op, agreement=0.0)
            return
    pytest.fail("no pixel with a near tie")


def test_floor_flip_direction():
    """Away from an integer a flip crosses to the nearest one; on it, floors drop and
    ceilings rise; a sector start clamped to 0 has no flip."""
    assert PY._flip(2.9999999, False) == 1 and PY._flip(3.0000001, False) == -1
    assert PY._flip(3.0, False) == -1 and PY._flip(3.0, True) == 1
    assert PY._flip(0.0, True) == 1
    op = O.Params(hit_criterion=O.PSEUDOCODE)
    ep = np.full((1, 2, 1, 2), np.nan)
    ep[0, 0, 0] = (0.0, 0.0)
    ep[0, 1, 0] = (5.0, 2.0)
    near = dict(PY._near_ties(ep, op))
    assert (0, 0, 0, 0) not in near and near[(0, 0, 0, 1)] == 1
    assert near[(0, 1, 0, 0)] == -1 and near[(0, 1, 0, 1)] == 1
