"""Write the regression vectors in this folder.  Calls only the oracle.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    xs = np.array([0, 1, 2, 17, 255, 1919, 3839, 16383])
    ys = np.array([0, 5, 1079, 3, 2159, 77, 1, 16383])
    out = {"comment": "PCG hash (Jarzynski and Olano 2020), nested pixel hash, R2 rotation, "
                      "per-slice jitter, direction table entries and FP32 step lengths, as the "
                      "oracle computes them.",
           "pcg_hash": {str(v): int(O.pcg_hash(v)) for v in (0, 1, 2, 0xFFFFFFFF, 0x9E3779B9, 12345)}}
    out["pixel_hash_seed7"] = [int(h) for h in O.pixel_hash(xs, ys, 7)]
    for name, mode in (("hash", O.NOISE_HASH), ("r2", O.NOISE_R2)):
        rho, xi = O.slice_noise(xs, ys, 4, mode, 123)
        out[f"rho16_{name}_seed123"] = rho.tolist()
        out[f"xi8_{name}_seed123_nd4"] = xi.tolist()
    out["r2_constants"] = list(O.r2_constants())
    dx, dy = O.direction_lut()
    ks = [0, 1, 2, 100, 1023, 1024, 1025, 2047, 2048, 2049, 3000, 4095]
    out["lut"] = {str(k): [int(dx[k]), int(dy[k])] for k in ks}
    out["lut_sum"] = [int(dx.sum()), int(dy.sum()), int((dx * np.arange(4096)).sum())]
    cam = O.Camera(1920, 1080, 540.0, 540.0, 960.0, 540.0)
    z = np.array([0.1, 1.0, 1.1361724, 3.3333333, 12.918648, 1e-3, 1e6], dtype=np.float32)
    out["step_q4_r3_ns16"] = O.step_q4(z, cam, O.Params(steps=16, radius=3.0)).tolist()
    out["step_q4_r8_ns32"] = O.step_q4(z, cam, O.Params(steps=32, radius=8.0)).tolist()
    with open(os.path.join(HERE, "noise_lattice_vectors.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
