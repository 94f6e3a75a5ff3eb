"""Regression: the oracle's noise, direction table and step lengths match the stored
vectors (written by tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np

import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "noise_lattice_vectors.json")


def test_golden_vectors():
    g = json.load(open(GOLDEN))
    for k, v in g["pcg_hash"].items():
        assert int(O.pcg_hash(int(k))) == v
    xs = np.array([0, 1, 2, 17, 255, 1919, 3839, 16383])
    ys = np.array([0, 5, 1079, 3, 2159, 77, 1, 16383])
    assert [int(h) for h in O.pixel_hash(xs, ys, 7)] == g["pixel_hash_seed7"]
    for name, mode in (("hash", O.NOISE_HASH), ("r2", O.NOISE_R2)):
        rho, xi = O.slice_noise(xs, ys, 4, mode, 123)
        assert rho.tolist() == g[f"rho16_{name}_seed123"]
        assert xi.tolist() == g[f"xi8_{name}_seed123_nd4"]
    assert list(O.r2_constants()) == g["r2_constants"]
    dx, dy = O.direction_lut()
    for k, (a, b) in g["lut"].items():
        assert (dx[int(k)], dy[int(k)]) == (a, b)
    assert [int(dx.sum()), int(dy.sum()), int((dx * np.arange(4096)).sum())] == g["lut_sum"]


def test_direction_table_not_near_ties():
    # 4096 cos(pi k / 4096) is never within 1e-6 of a half integer unless it is an
    # integer, so any correctly rounded FP64 cosine builds the same table
    k = np.arange(4096)
    for f in (np.cos, np.sin):
        v = 4096 * f(np.pi * k / 4096)
        frac = np.abs(v - np.floor(v) - 0.5)
        ok = (frac > 1e-6) | (np.abs(v - np.round(v)) < 1e-9)
        assert np.all(ok)
