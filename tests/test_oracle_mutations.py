"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that the pins
catch every one: a dropped term, a wrong sign, index or operand must fail some pin.

Two natural mutants are left out because they are equivalent, not wrong: widening the
hemisphere clamp, and dropping the clamp of n_p . l at zero.  Sectors outside
[0, N_b) do not exist, so an out-of-hemisphere endpoint sets nothing either way, and a
sample with n_p . l < 0 lies below the tangent plane, where it can cover no sector."""
import os
import sys
import types

import pytest

import oracle_pins as P

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "oracle", "ssvb_oracle.py")

MUTATIONS = {
    "back sample toward the camera": ("d_v - t_p", "d_v + t_p"),
    "front angle ignores the projected normal": ("theta_f = np.arctan2(d_e, d_v) - gamma",
                                                 "theta_f = np.arctan2(d_e, d_v)"),
    "floor instead of round criterion": ("nb * u_lo + 0.5, nb * u_hi + 0.5", "nb * u_lo, nb * u_hi"),
    "sample normal factor sign": ("np.maximum(0.0, -_dot(n_j, l_j))", "np.maximum(0.0, _dot(n_j, l_j))"),
    "GI counts all covered sectors": ("new = b_j & ~b_i", "new = b_j"),
    "ambient weight over the subregion": ("free / nb", "free / per"),
    "first step at zero offset": ("return q * (j + 1) +", "return q * j +"),
    "exact position ignores the side": ("X_e = xs + 0.5 + s * o * dx_i / 65536.0",
                                        "X_e = xs + 0.5 + o * dx_i / 65536.0"),
    "slice tangent sign": ("e = d3 - _dot(d3, v)[:, None] * v", "e = d3 + _dot(d3, v)[:, None] * v"),
    "AO as occlusion": ("ao_sum += 1.0 - b_i.sum(axis=1) / nb", "ao_sum += b_i.sum(axis=1) / nb"),
    "transposed view-to-world": ("a_k @ Rvw.T", "a_k @ Rvw"),
    "image y not flipped": ("-(Y_e - cy) / fy", "(Y_e - cy) / fy"),
    "hemisphere clamp too tight": ("theta_f = np.clip(theta_f, -np.pi / 2, np.pi / 2)",
                                   "theta_f = np.clip(theta_f, -np.pi / 2.2, np.pi / 2.2)"),
    "ambient direction at subregion edge": ("(k + 0.5) * np.pi / na", "k * np.pi / na"),
    "view vector away from camera": ("v = -r_p / np.linalg.norm", "v = r_p / np.linalg.norm"),
    "gamma operands swapped": ("np.arctan2(n_e, n_v)", "np.arctan2(n_v, n_e)"),
    "GI weight ignores new-sector count": ("(cnt / nb) *", "(1.0 / nb) *"),
    "centre normal factor dropped": ("np.maximum(0.0, _dot(n_p, l_j))", "1.0"),
    "mask not accumulated": ("b_i |= b_j", "b_i = b_i | (b_j & False)"),
    "slices cover half a turn": ("(i * 65536 + rho16) // (16 * nd)", "(i * 65536 + rho16) // (32 * nd)"),
    "direction table sine": ("dy = np.floor(LUT_ONE * np.sin(phi) + 0.5)", "dy = np.floor(LUT_ONE * np.cos(phi) + 0.5)"),
    "projected radius halved": ("16.0 * _f32(prm.radius)", "8.0 * _f32(prm.radius)"),
    "lattice drops the half pixel": ("X = ((xs << 16) + 32768 + s * o * dx_i) >> 16",
                                     "X = ((xs << 16) + s * o * dx_i) >> 16"),
    "thickness slope sign": ("t0 + tk *", "t0 - tk *"),
    "ambient counts occluded sectors": ("(~b_i[:, k * per:(k + 1) * per])", "(b_i[:, k * per:(k + 1) * per])"),
    "GI reads the centre radiance": ("c_j = rad64[Yc, Xc]", "c_j = rad64[ys, xs]"),
    "GI light direction reversed": ("l_j = delta / np.linalg.norm", "l_j = -delta / np.linalg.norm"),
    "front/back not ordered": ("t_min, t_max = np.minimum(theta_f, theta_b), np.maximum(theta_f, theta_b)",
                               "t_min, t_max = theta_f, theta_b"),
    "jitter too large": ("((q * xi8) >> 8)", "((q * xi8) >> 5)"),
    "quadratic steps linear in j": ("t = (q * a * a) >> 16", "t = (q * a * 256) >> 16"),
    "quadratic reach over N_s": ("((1 << 32) // (ns + 1))", "((1 << 32) // ns)"),
    "quadratic steps ignore the jitter": ("a = (j + 1) * 256 + xi8", "a = (j + 1) * 256"),
    "upsampling ignores depth": ("(UPSAMPLE_FLOOR + math.exp(-d * d))", "(UPSAMPLE_FLOOR + 1.0)"),
    "upsampling not normalised": ("sao / sw, sgi / sw, samb / sw", "sao, sgi, samb"),
    "upsampling takes the far neighbour twice": ("[(y - 1, 0.5), (y + 1, 0.5)]", "[(y + 1, 0.5), (y + 1, 0.5)]"),
    "half resolution samples odd pixels": ("np.arange(0, H, 2), np.arange(0, W, 2)", "np.arange(1, H, 2), np.arange(1, W, 2)"),
    "bounce ignores the albedo": ("return d + float(np.float32(gain)) * a * np.asarray", "return d + float(np.float32(gain)) * np.asarray"),
    "bounce replaces the direct light": ("return d + float(np.float32(gain))", "return 0 * d + float(np.float32(gain))"),
    "background samples kept": ("ok &= np.isfinite(z_s) & (z_s > 0)", "ok &= np.isfinite(z_s)"),
    "step floor not clamped": ("return np.clip(q, q_min, q_max)", "return np.clip(q, 1, q_max)"),
    "denoise kernel not the B3 spline": ("(1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16)",
                                         "(1.0 / 9, 2.0 / 9, 3.0 / 9, 2.0 / 9, 1.0 / 9)"),
    "a-trous spacing not doubled": ("s = 1 << i", "s = 1 + i"),
    "denoise weight from the depth difference": ("np.sum(n_p * (pos[Q] - P_p), axis=-1) * inv_scale",
                                                 "(z[Q] - z[py0:py1, px0:px1]) * inv_scale"),
    "plane distance not relative to depth": ("* inv_scale / zp[py0:py1, px0:px1]", "* inv_scale"),
    "plane falloff not Gaussian": ("np.exp(-dist * dist)", "np.exp(-np.abs(dist))"),
    "normal weight not clamped": ("np.maximum(0.0, np.sum(n_p * n[Q], axis=-1)) ** normal_power",
                                  "np.sum(n_p * n[Q], axis=-1) ** normal_power"),
    "denoise keeps background taps": ("w = np.where(fg[Q], w, 0.0)", "w = np.where(True, w, 0.0)"),
    "denoise centre weight one": ("wsum = np.full((gh, gw), DENOISE_KERNEL[2] ** 2)", "wsum = np.full((gh, gw), 1.0)"),
    "denoise grid positions at half resolution": ("np.arange(gh) * g, np.arange(gw) * g",
                                                  "np.arange(gh), np.arange(gw)"),
    "denoise tap taken from the pixel": ("acc[py0:py1, px0:px1] += w[..., None] * sig[Q]",
                                         "acc[py0:py1, px0:px1] += w[..., None] * sig[py0:py1, px0:px1]"),
    "SH xy constant halved": ("0.5 * math.sqrt(15.0 / pi) * x * y", "0.25 * math.sqrt(15.0 / pi) * x * y"),
    "SH yz and xz swapped": ("0.5 * math.sqrt(15.0 / pi) * y * z,\n        0.25 * math.sqrt(5.0 / pi) * (3.0 * z * z - 1.0),\n"
                             "        0.5 * math.sqrt(15.0 / pi) * x * z,",
                             "0.5 * math.sqrt(15.0 / pi) * x * z,\n        0.25 * math.sqrt(5.0 / pi) * (3.0 * z * z - 1.0),\n"
                             "        0.5 * math.sqrt(15.0 / pi) * y * z,"),
    "SH x^2 - y^2 read as x^2 - z^2": ("(x * x - y * y)", "(x * x - z * z)"),
    "SH zonal constant doubled": ("0.25 * math.sqrt(5.0 / pi) * (3.0 * z * z - 1.0)",
                                  "0.5 * math.sqrt(5.0 / pi) * (3.0 * z * z - 1.0)"),
    "SH zonal without the constant": ("(3.0 * z * z - 1.0)", "(3.0 * z * z)"),
    "SH x^2 - y^2 constant": ("0.25 * math.sqrt(15.0 / pi) * (x * x - y * y)", "0.5 * math.sqrt(15.0 / pi) * (x * x - y * y)"),
    "sequence seed not advanced": ("seed=(prm.seed + n) % (1 << 32)", "seed=prm.seed"),
    "sequence feeds back the light": ("        gi = r[\"gi\"]\n        out.append(r)", "        gi = light\n        out.append(r)"),
    "sequence ignores the gain": ("light = inject_bounce(f[\"direct\"], f[\"albedo\"], prev, gain)",
                                  "light = inject_bounce(f[\"direct\"], f[\"albedo\"], prev, 1.0)"),
    "sequence light kept in FP64": (".astype(light_dtype)", ""),
    "denoise background overwritten": ("sig = np.where(fg[..., None], acc / wsum[..., None], sig)",
                                       "sig = acc / wsum[..., None]"),
    "pseudocode width floored": ("b = np.ceil(arg1).astype(np.int64)", "b = np.floor(arg1).astype(np.int64)"),
    "pseudocode start rounded": ("arg0, arg1 = nb * u_lo, nb * (u_hi - u_lo)",
                                 "arg0, arg1 = nb * u_lo + 0.5, nb * (u_hi - u_lo)"),
    "pseudocode width read as the end": ("b = np.minimum(a + b, nb)", "b = np.minimum(b, nb)"),
    "pseudocode width from the upper angle": ("arg0, arg1 = nb * u_lo, nb * (u_hi - u_lo)",
                                              "arg0, arg1 = nb * u_lo, nb * u_hi"),
}


def _mutant(name, old, new):
    src = open(ORACLE_SRC).read()
    assert src.count(old) >= 1, f"mutation '{name}' does not apply"
    modname = "oracle_mutant_" + str(abs(hash(name)))
    mod = types.ModuleType(modname)
    sys.modules[modname] = mod  # dataclasses look their module up here
    exec(compile(src.replace(old, new), ORACLE_SRC + f" [{name}]", "exec"), mod.__dict__)
    return mod


# the pin most likely to catch a mutant of this kind runs first (only the run time
# depends on the order: a mutant passes this test if any pin fails on it)
FIRST = [("denoise", "pin_denoise"), ("a-trous", "pin_denoise"), ("plane distance", "pin_denoise"),
         ("plane falloff", "pin_denoise"), ("normal weight", "pin_denoise"), ("sequence", "pin_bounce_sequence"),
         ("SH ", "pin_sh_basis"), ("bounce", "pin_multi_bounce"), ("upsampling", "pin_half_resolution"),
         ("half resolution", "pin_half_resolution"), ("quadratic", "pin_quadratic_steps"),
         ("pseudocode", "pin_pseudocode_horizon")]


def pin_order(name):
    first = [pin for key, pin in FIRST if key in name]
    return sorted(P.ALL_PINS, key=lambda f: 0 if f.__name__ in first else 1)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name):
    old, new = MUTATIONS[name]
    O = _mutant(name, old, new)
    for pin in pin_order(name):
        try:
            pin(O)
        except Exception:
            return
    pytest.fail(f"no pin caught the planted mistake: {name}")
