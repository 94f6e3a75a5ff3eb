"""CPU checks of the C ABI: the library loads, exports every symbol include/ssvb.h
declares, and its host-side validation accepts and rejects what the header says.
No compute call is made (there is no GPU here)."""
import ctypes
import math
import os
import re

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_2301_11376_amd import binding, build_lib
    if not os.path.exists(binding.LIB_PATH):
        build_lib.build()
    binding.lib()
    return binding


def header_functions():
    src = open(os.path.join(ROOT, "include", "ssvb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ssvb_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(B):
    names = header_functions()
    assert len(names) >= 10
    lib = B.lib()
    for n in names:
        assert hasattr(lib, n), f"{n} declared in ssvb.h but not exported"
    assert sorted(B.EXPORTED) == names


def test_status_strings(B):
    for code, name in B.STATUS.items():
        assert B.lib().ssvb_status_string(code).decode() == name


def test_default_params(B):
    p = B.default_params()
    assert (p.slices, p.steps, p.sectors, p.ambient_samples, p.min_step_q4) == (4, 16, 32, 4, 16)
    assert (p.radius, p.thickness, p.hit_criterion, p.noise, p.step_distribution, p.resolution) == (1.0, 0.5, 0, 0, 0, 1)
    d = B.Params()
    assert (d.slices, d.steps, d.sectors, d.ambient_samples, d.min_step_q4) == (4, 16, 32, 4, 16)


def test_noise_constants_match_oracle(B):
    # independent derivations of Roberts' R2 constants (C++ long double vs Python Decimal)
    assert B.noise_constants() == list(O.r2_constants())


FAKE = 0x100000  # validation only inspects pointers for NULL and alignment


def frame(B, W=64, H=48, **over):
    d = B.ssvb_image(FAKE, 0, B.F32, 1)
    n = B.ssvb_image(FAKE, 0, B.F32, 3)
    r = B.ssvb_image(FAKE, 0, B.F16, 4)
    c = B.Camera(W, H, 40.0, 40.0, W / 2, H / 2).to_c()
    p = B.Params(slices=2, steps=8).to_c()
    o = B.ssvb_outputs(FAKE, FAKE, FAKE, None, 0, 0, 0, 0)
    parts = dict(d=d, n=n, r=r, c=c, p=p, o=o)
    for k, fn in over.items():
        fn(parts[k])
    return parts


def status(B, parts):
    return B.validate(parts["d"], parts["n"], parts["r"], parts["c"], parts["p"], parts["o"])


def setter(attr, value):
    def fn(obj):
        setattr(obj, attr, value)
    return fn


def test_validate_accepts_good_frames(B):
    assert status(B, frame(B)) == 0
    assert status(B, frame(B, p=setter("thickness", math.inf))) == 0
    assert status(B, frame(B, p=setter("step_distribution", 1))) == 0
    assert status(B, frame(B, p=setter("resolution", 2))) == 0
    assert status(B, frame(B, W=16384, H=1)) == 0
    assert status(B, frame(B, W=0, H=0, d=setter("ptr", None), n=setter("ptr", None),
                           o=setter("ao", None))) == 0
    assert status(B, frame(B, d=setter("pitch_bytes", 64 * 4 + 256))) == 0
    assert status(B, frame(B, o=setter("masks", FAKE))) == 0


BAD = {
    "null depth": dict(d=setter("ptr", None)),
    "misaligned normal": dict(n=setter("ptr", FAKE + 2)),
    "depth pitch too small": dict(d=setter("pitch_bytes", 4 * 63)),
    "pitch not a multiple": dict(n=setter("pitch_bytes", 64 * 12 + 2)),
    "depth as F16": dict(d=setter("dtype", 1)),
    "two channels": dict(n=setter("channels", 2)),
    "unknown dtype": dict(r=setter("dtype", 9)),
    "zero slices": dict(p=setter("slices", 0)),
    "too many slices": dict(p=setter("slices", 65)),
    "too many steps": dict(p=setter("steps", 1025)),
    "zero sectors": dict(p=setter("sectors", 0)),
    "ambient 3": dict(p=setter("ambient_samples", 3)),
    "nan radius": dict(p=setter("radius", math.nan)),
    "negative radius": dict(p=setter("radius", -1.0)),
    "negative thickness": dict(p=setter("thickness", -0.1)),
    "nan thickness": dict(p=setter("thickness", math.nan)),
    "inf slope": dict(p=setter("thickness_slope", math.inf)),
    "min step 0": dict(p=setter("min_step_q4", 0)),
    "min step 17": dict(p=setter("min_step_q4", 17)),
    "criterion 2": dict(p=setter("hit_criterion", 2)),
    "step distribution 2": dict(p=setter("step_distribution", 2)),
    "resolution 3": dict(p=setter("resolution", 3)),
    "resolution 0": dict(p=setter("resolution", 0)),
    "noise 5": dict(p=setter("noise", 5)),
    "wide image": dict(c=setter("width", 16385)),
    "zero focal": dict(c=setter("fx", 0.0)),
    "null ao": dict(o=setter("ao", None)),
    "gi pitch too small": dict(o=setter("gi_pitch_bytes", 64 * 12 - 4)),
}


@pytest.mark.parametrize("case", sorted(BAD))
def test_validate_rejects(B, case):
    assert status(B, frame(B, **BAD[case])) == 1, case
    assert B.lib().ssvb_last_error().decode() != ""


def test_validate_half_resolution_without_masks(B):
    def half(p):
        p.resolution = 2
    assert status(B, frame(B, p=half, o=setter("masks", FAKE))) == 1


def test_validate_unsupported_sectors(B):
    assert status(B, frame(B, p=setter("sectors", 64))) == 2
    assert status(B, frame(B, p=setter("sectors", 128))) == 0


def test_validate_sectors128_layouts(B):
    def s128(p):
        p.sectors = 128
    # masks: N_d x 4 words per pixel
    assert status(B, frame(B, p=s128, o=setter("masks", FAKE))) == 0
    def short_pitch(o):
        o.masks = FAKE
        o.masks_pitch_bytes = 64 * 2 * 4  # one word per slice: too short for 128 sectors
    assert status(B, frame(B, p=s128, o=short_pitch)) == 1
    def amb(p):
        p.sectors = 128
        p.ambient_samples = 64           # more than 32 subregions
    assert status(B, frame(B, p=amb)) == 1


def test_validate_nan_probe(B):
    def bad_sh(p):
        p.ambient_sh[4] = math.nan
    assert status(B, frame(B, p=bad_sh)) == 1


def test_create_without_gpu_fails_cleanly(B):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert B.lib().ssvb_create(0, ctypes.byref(h)) != 0
    assert not h.value


def test_sequence_null_handles(B):
    """The frame-sequence entry points refuse missing handles before touching a device."""
    L = B.lib()
    h = ctypes.c_void_p()
    assert L.ssvb_sequence_create(None, 16, 16, 0, ctypes.byref(h)) == 1 and not h.value
    assert L.ssvb_sequence_create(None, 16, 16, 0, None) == 1
    assert L.ssvb_sequence_step(None, None, None, None, None, None, None, 0.5, None, None) == 1
    assert L.ssvb_sequence_reset(None) == 1
    v = ctypes.c_int64(-1)
    assert L.ssvb_sequence_frame(None, ctypes.byref(v)) == 1 and v.value == -1
    assert L.ssvb_sequence_copy_light(None, None, 0, None) == 1
    assert L.ssvb_sequence_destroy(None) == 0


def test_slice_order_null_context(B):
    """ssvb_set_slice_order refuses a missing context, whatever the chunk."""
    L = B.lib()
    for chunk in (0, 1, 65536, -1, 65537):
        assert L.ssvb_set_slice_order(None, chunk) == 1
    assert "context" in B.lib().ssvb_last_error().decode().lower()


def test_validate_depth_span_limit(B):
    # images are addressed with 32-bit byte offsets
    assert status(B, frame(B, W=16384, H=16384, d=setter("pitch_bytes", 65536))) == 0
    assert status(B, frame(B, W=16384, H=16384, d=setter("pitch_bytes", 4 * 65536))) == 0
    assert status(B, frame(B, W=16384, H=16384, d=setter("pitch_bytes", 4 * 65536 + 64))) == 1
    # 16384 x 16384 x 4 channels x FP32 is exactly 4 GiB; one more row of pitch is not
    assert status(B, frame(B, W=16384, H=16384, n=setter("channels", 4))) == 0
    assert status(B, frame(B, W=16384, H=16384, n=setter("channels", 4),
                           d=setter("pitch_bytes", 0))) == 0
    assert status(B, frame(B, W=16384, H=16384, n=setter("pitch_bytes", 16384 * 16 + 16))) == 1


def test_binding_checks_tensors_against_the_camera(B):
    """The C ABI takes bare pointers and pitches: the binding refuses tensors that the
    library would read or write out of bounds (host tensors here, as the server takes)."""
    import torch
    chk = B.check_tensor
    H, W = 6, 10
    ok3 = torch.zeros((H, W, 3))
    chk(ok3, "n", H, W, (3, 4), "image", allow_host=True)
    chk(torch.zeros((H, W + 7, 4))[:, :W], "n", H, W, (3, 4), "image", allow_host=True)   # pitched view
    chk(torch.zeros((H, W), dtype=torch.float16)[:, :W], "d", H, W, None, "image", allow_host=True)
    chk(torch.zeros((0, 0)), "d", 0, 0, None, "f32", allow_host=True)
    bad = [
        (torch.zeros((H - 1, W, 3)), (3, 4), "image"),                 # fewer rows than the camera
        (torch.zeros((H, W + 1, 3)), (3, 4), "image"),                 # wider than the camera
        (torch.zeros((H, W, 2)), (3, 4), "image"),                     # channel count
        (torch.zeros((H, W, 3), dtype=torch.float64), (3, 4), "image"),
        (torch.zeros((1, W, 3)).expand(H, W, 3), (3, 4), "image"),     # every row the same memory
        (torch.zeros((H, 2 * W, 3))[:, ::2], (3, 4), "image"),         # pixels not contiguous
        (torch.zeros((H, W, 3)).permute(1, 0, 2).contiguous().permute(1, 0, 2), (3, 4), "image"),
        (torch.zeros((H, W)), None, "i32"),                            # masks are int32
    ]
    for t, ch, kind in bad:
        with pytest.raises(ValueError):
            chk(t, "x", H, W, ch, kind, allow_host=True)
    with pytest.raises(ValueError):                                    # device tensors only
        chk(ok3, "n", H, W, (3, 4), "image")
    out = {"ao": torch.zeros((H, W)), "gi": torch.zeros((H, W, 3)), "ambient": torch.zeros((H, W, 3))}
    B.check_outputs(out, H, W, allow_host=True)
    B.check_outputs(dict(out, masks=torch.zeros((H, W, 4), dtype=torch.int32)), H, W, allow_host=True, masks_words=4)
    for k, t in (("ao", torch.zeros((H, W, 1))), ("gi", torch.zeros((H, W, 4))), ("ambient", torch.zeros((H, W - 1, 3))),
                 ("masks", torch.zeros((H, W, 3), dtype=torch.int32))):
        with pytest.raises(ValueError):
            B.check_outputs(dict(out, **{k: t}), H, W, allow_host=True, masks_words=4)
