"""ctypes binding of libssvb.so (the C ABI in include/ssvb.h).

Argument marshalling only: every step of the gather runs in the HIP library.  Torch
tensors supply device memory and the stream; nothing here computes on the data.  The
library must have been built (``paper_2301_11376_amd.build_lib.build()``); loading
fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

PKG = os.path.dirname(os.path.abspath(__file__))
# SSVB_LIBRARY may name another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("SSVB_LIBRARY") or os.path.join(PKG, "libssvb.so")

SSVB_OK = 0
STATUS = {0: "SSVB_OK", 1: "SSVB_ERR_INVALID_ARG", 2: "SSVB_ERR_UNSUPPORTED", 3: "SSVB_ERR_OUT_OF_MEMORY",
          4: "SSVB_ERR_DEVICE", 5: "SSVB_ERR_BUSY", 6: "SSVB_ERR_TIMEOUT", 7: "SSVB_ERR_NOT_FOUND"}
F32, F16 = 0, 1
HIT_ROUND, HIT_PSEUDOCODE = 0, 1
NOISE_HASH, NOISE_R2, NOISE_FIXED = 0, 1, 2
NOISE_NAMES = {"hash": NOISE_HASH, "r2": NOISE_R2, "fixed": NOISE_FIXED}
STEPS_UNIFORM, STEPS_QUADRATIC = 0, 1

# every symbol include/ssvb.h declares
EXPORTED = [
    "ssvb_status_string", "ssvb_last_error", "ssvb_default_params", "ssvb_create", "ssvb_destroy",
    "ssvb_validate", "ssvb_compute", "ssvb_compute_batch", "ssvb_set_launch", "ssvb_get_launch",
    "ssvb_set_slice_order",
    "ssvb_autotune", "ssvb_debug_lattice", "ssvb_debug_endpoints", "ssvb_debug_direction_table",
    "ssvb_debug_noise_constants", "ssvb_server_create", "ssvb_server_submit", "ssvb_server_poll",
    "ssvb_server_wait", "ssvb_server_release", "ssvb_server_stats", "ssvb_server_destroy", "ssvb_inject_bounce",
    "ssvb_default_denoise_params", "ssvb_denoise", "ssvb_sequence_create", "ssvb_sequence_step",
    "ssvb_sequence_reset", "ssvb_sequence_frame", "ssvb_sequence_copy_light", "ssvb_sequence_destroy",
]


class ssvb_image(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("pitch_bytes", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("channels", ctypes.c_int32)]


class ssvb_camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("view_to_world", ctypes.c_float * 9)]


class ssvb_params(ctypes.Structure):
    _fields_ = [("slices", ctypes.c_int32), ("steps", ctypes.c_int32), ("sectors", ctypes.c_int32),
                ("ambient_samples", ctypes.c_int32), ("radius", ctypes.c_float), ("thickness", ctypes.c_float),
                ("thickness_slope", ctypes.c_float), ("max_radius_px", ctypes.c_float),
                ("min_step_q4", ctypes.c_int32), ("step_distribution", ctypes.c_int32),
                ("resolution", ctypes.c_int32), ("hit_criterion", ctypes.c_int32), ("noise", ctypes.c_int32),
                ("seed", ctypes.c_uint32), ("ambient_sh", ctypes.c_float * 27)]


class ssvb_outputs(ctypes.Structure):
    _fields_ = [("ao", ctypes.c_void_p), ("gi", ctypes.c_void_p), ("ambient", ctypes.c_void_p),
                ("masks", ctypes.c_void_p), ("ao_pitch_bytes", ctypes.c_int64), ("gi_pitch_bytes", ctypes.c_int64),
                ("ambient_pitch_bytes", ctypes.c_int64), ("masks_pitch_bytes", ctypes.c_int64)]


class ssvb_frame(ctypes.Structure):
    _fields_ = [("depth", ssvb_image), ("normal", ssvb_image), ("radiance", ssvb_image), ("camera", ssvb_camera),
                ("params", ssvb_params), ("out", ssvb_outputs)]


class ssvb_denoise_params(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("normal_power", ctypes.c_int32), ("plane_sigma", ctypes.c_float),
                ("resolution", ctypes.c_int32)]


class ssvb_launch(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("strip", ctypes.c_int32),
                ("lanes_per_pixel", ctypes.c_int32)]

    def as_tuple(self):
        return (self.tile_w, self.tile_h, self.strip, self.lanes_per_pixel)


class ssvb_server_counters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("rounds", ctypes.c_uint64), ("frames_in_rounds", ctypes.c_uint64),
                ("admitted_while_running", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("arena_in_use", ctypes.c_uint64), ("arena_peak", ctypes.c_uint64), ("queued", ctypes.c_int32),
                ("resident", ctypes.c_int32), ("running_rounds", ctypes.c_int32),
                ("max_running_rounds", ctypes.c_int32), ("max_round_frames", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_LIB = None


def lib() -> ctypes.CDLL:
    """Load libssvb.so and declare its signatures.  Raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    P, I, V = ctypes.POINTER, ctypes.c_int32, ctypes.c_void_p
    L.ssvb_status_string.restype = ctypes.c_char_p
    L.ssvb_status_string.argtypes = [I]
    L.ssvb_last_error.restype = ctypes.c_char_p
    L.ssvb_last_error.argtypes = []
    L.ssvb_default_params.restype = None
    L.ssvb_default_params.argtypes = [P(ssvb_params)]
    L.ssvb_create.restype = I
    L.ssvb_create.argtypes = [I, P(V)]
    L.ssvb_destroy.restype = I
    L.ssvb_destroy.argtypes = [V]
    L.ssvb_validate.restype = I
    L.ssvb_validate.argtypes = [P(ssvb_image), P(ssvb_image), P(ssvb_image), P(ssvb_camera), P(ssvb_params),
                                P(ssvb_outputs)]
    L.ssvb_compute.restype = I
    L.ssvb_compute.argtypes = [V, P(ssvb_image), P(ssvb_image), P(ssvb_image), P(ssvb_camera), P(ssvb_params),
                               P(ssvb_outputs), V]
    L.ssvb_compute_batch.restype = I
    L.ssvb_compute_batch.argtypes = [V, P(ssvb_frame), I, V]
    L.ssvb_set_launch.restype = I
    L.ssvb_set_launch.argtypes = [V, P(ssvb_launch)]
    L.ssvb_set_slice_order.restype = I
    L.ssvb_set_slice_order.argtypes = [V, ctypes.c_int32]
    L.ssvb_get_launch.restype = I
    L.ssvb_get_launch.argtypes = [V, P(ssvb_camera), P(ssvb_params), I, P(ssvb_launch)]
    L.ssvb_autotune.restype = I
    L.ssvb_autotune.argtypes = [V, P(ssvb_frame), V, P(ssvb_launch), P(ctypes.c_float)]
    L.ssvb_debug_lattice.restype = I
    L.ssvb_debug_lattice.argtypes = [V, P(ssvb_image), P(ssvb_camera), P(ssvb_params), V, V]
    L.ssvb_debug_endpoints.restype = I
    L.ssvb_debug_endpoints.argtypes = [V, P(ssvb_image), P(ssvb_image), P(ssvb_camera), P(ssvb_params), V, V]
    L.ssvb_debug_direction_table.restype = I
    L.ssvb_debug_direction_table.argtypes = [V, P(ctypes.c_int32)]
    L.ssvb_debug_noise_constants.restype = None
    L.ssvb_debug_noise_constants.argtypes = [P(ctypes.c_uint32)]
    L.ssvb_inject_bounce.restype = I
    L.ssvb_inject_bounce.argtypes = [V, I, I, P(ssvb_image), P(ssvb_image), V, ctypes.c_int64, ctypes.c_float,
                                     P(ssvb_image), V]
    L.ssvb_default_denoise_params.restype = None
    L.ssvb_default_denoise_params.argtypes = [P(ssvb_denoise_params)]
    L.ssvb_denoise.restype = I
    L.ssvb_denoise.argtypes = [V, P(ssvb_image), P(ssvb_image), P(ssvb_camera), P(ssvb_outputs), P(ssvb_outputs),
                               P(ssvb_outputs), P(ssvb_denoise_params), V]
    L.ssvb_sequence_create.restype = I
    L.ssvb_sequence_create.argtypes = [V, I, I, I, P(V)]
    L.ssvb_sequence_step.restype = I
    L.ssvb_sequence_step.argtypes = [V, P(ssvb_image), P(ssvb_image), P(ssvb_image), P(ssvb_image), P(ssvb_camera),
                                     P(ssvb_params), ctypes.c_float, P(ssvb_outputs), V]
    L.ssvb_sequence_reset.restype = I
    L.ssvb_sequence_reset.argtypes = [V]
    L.ssvb_sequence_frame.restype = I
    L.ssvb_sequence_frame.argtypes = [V, P(ctypes.c_int64)]
    L.ssvb_sequence_copy_light.restype = I
    L.ssvb_sequence_copy_light.argtypes = [V, V, ctypes.c_int64, V]
    L.ssvb_sequence_destroy.restype = I
    L.ssvb_sequence_destroy.argtypes = [V]
    U64, D = ctypes.c_uint64, ctypes.c_double
    L.ssvb_server_create.restype = I
    L.ssvb_server_create.argtypes = [V, U64, I, P(V)]
    L.ssvb_server_submit.restype = I
    L.ssvb_server_submit.argtypes = [V, P(ssvb_frame), V, P(U64)]
    L.ssvb_server_poll.restype = I
    L.ssvb_server_poll.argtypes = [V, U64, P(I), P(D)]
    L.ssvb_server_wait.restype = I
    L.ssvb_server_wait.argtypes = [V, U64, D, P(D)]
    L.ssvb_server_release.restype = I
    L.ssvb_server_release.argtypes = [V, U64]
    L.ssvb_server_stats.restype = I
    L.ssvb_server_stats.argtypes = [V, P(ssvb_server_counters)]
    L.ssvb_server_destroy.restype = I
    L.ssvb_server_destroy.argtypes = [V]
    _LIB = L
    return L


class SSVBError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = lib().ssvb_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")


def check(status: int, where: str) -> None:
    if status != SSVB_OK:
        raise SSVBError(status, where)


# ---------------------------------------------------------------------------------------
# plain-Python descriptions of a camera and of the sampling parameters
# ---------------------------------------------------------------------------------------

@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    view_to_world: tuple = (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0)

    def to_c(self) -> ssvb_camera:
        c = ssvb_camera(self.width, self.height, self.fx, self.fy, self.cx, self.cy)
        for i, v in enumerate(self.view_to_world):
            c.view_to_world[i] = v
        return c


@dataclass
class Params:
    slices: int = 4
    steps: int = 16
    sectors: int = 32
    ambient_samples: int = 4
    radius: float = 1.0
    thickness: float = 0.5
    thickness_slope: float = 0.0
    max_radius_px: float = 0.0
    min_step_q4: int = 16
    step_distribution: int = STEPS_UNIFORM
    resolution: int = 1
    hit_criterion: int = HIT_ROUND
    noise: int = NOISE_HASH
    seed: int = 0
    ambient_sh: tuple = field(default_factory=lambda: tuple([0.0] * 27))

    def to_c(self) -> ssvb_params:
        p = ssvb_params(self.slices, self.steps, self.sectors, self.ambient_samples, self.radius, self.thickness,
                        self.thickness_slope, self.max_radius_px, self.min_step_q4, self.step_distribution,
                        self.resolution, self.hit_criterion, self.noise, self.seed & 0xFFFFFFFF)
        for i, v in enumerate(self.ambient_sh):
            p.ambient_sh[i] = v
        return p


def image_of(t, channels_expected=None) -> ssvb_image:
    """Describe a torch tensor [H, W] (depth) or [H, W, C] (normal / radiance)."""
    import torch
    if t is None:
        return ssvb_image(None, 0, F32, 3)
    if t.dim() == 2:
        ch = 1
        if t.stride(1) != 1:
            raise ValueError("image rows must be contiguous")
    elif t.dim() == 3:
        ch = t.shape[2]
        if t.stride(2) != 1 or t.stride(1) != ch:
            raise ValueError("image pixels must be contiguous HWC")
    else:
        raise ValueError("images are [H, W] or [H, W, C]")
    if t.dtype == torch.float32:
        dt, es = F32, 4
    elif t.dtype == torch.float16:
        dt, es = F16, 2
    else:
        raise ValueError(f"unsupported dtype {t.dtype}")
    return ssvb_image(t.data_ptr(), t.stride(0) * es, dt, ch)


def check_tensor(t, name, H, W, channels=None, kind="image", device=None, allow_host=False):
    """Check that tensor ``t`` can hold what the library reads or writes through its
    pointer for an H x W frame: the C ABI takes bare pointers and pitches, so a tensor
    smaller than the camera says (or with overlapping rows) would be read or written out
    of bounds on the device.  ``channels``: None for [H, W], else the allowed C of
    [H, W, C].  ``kind``: "image" (FP32 or FP16), "f32" or "i32"."""
    import torch
    if t is None:
        raise ValueError(f"{name}: missing")
    if channels is None:
        if t.dim() != 2:
            raise ValueError(f"{name}: expected [H, W], got shape {tuple(t.shape)}")
        C = 1
    else:
        if t.dim() != 3 or t.shape[2] not in channels:
            raise ValueError(f"{name}: expected [H, W, C] with C in {tuple(channels)}, got shape {tuple(t.shape)}")
        C = t.shape[2]
    if tuple(t.shape[:2]) != (H, W):
        raise ValueError(f"{name}: shape {tuple(t.shape)} does not match the {W}x{H} camera")
    allowed = {"image": (torch.float32, torch.float16), "f32": (torch.float32,), "i32": (torch.int32,)}[kind]
    if t.dtype not in allowed:
        raise ValueError(f"{name}: dtype {t.dtype} (need one of {allowed})")
    if t.is_cuda:
        if device is not None and t.device.index != device:
            raise ValueError(f"{name}: on {t.device}, the context is on cuda:{device}")
    elif not allow_host:
        raise ValueError(f"{name}: must be a device tensor")
    if H * W > 0:
        if (C > 1 and (t.stride(2) != 1 or t.stride(1) != C)) or (C == 1 and t.stride(1) != 1):
            raise ValueError(f"{name}: pixels must be contiguous")
        if H > 1 and t.stride(0) < W * C:
            raise ValueError(f"{name}: rows overlap (row stride {t.stride(0)} < {W * C})")


def check_outputs(out, H, W, device=None, allow_host=False, masks_words=None):
    check_tensor(out.get("ao"), "ao", H, W, None, "f32", device, allow_host)
    check_tensor(out.get("gi"), "gi", H, W, (3,), "f32", device, allow_host)
    check_tensor(out.get("ambient"), "ambient", H, W, (3,), "f32", device, allow_host)
    if out.get("masks") is not None:
        check_tensor(out["masks"], "masks", H, W, (masks_words,), "i32", device, allow_host)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class FrameArray:
    """Frames already marshalled for the C ABI (see Context.frames)."""

    def __init__(self, arr, n):
        self.arr, self.n = arr, n


class Context:
    """An ssvb_ctx on one device (torch's current device by default)."""

    def __init__(self, device: int | None = None):
        import torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        check(lib().ssvb_create(self.device, ctypes.byref(h)), "ssvb_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().ssvb_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def compute(self, depth, normal, radiance, camera: Camera, params: Params, out=None, masks=False, stream=None):
        """Run ssvb_compute on torch device tensors; returns dict(ao, gi, ambient[, masks])."""
        import torch
        H, W = camera.height, camera.width
        self._check_inputs(depth, normal, radiance, H, W)
        dev = depth.device
        if out is None:
            out = {"ao": torch.empty((H, W), dtype=torch.float32, device=dev),
                   "gi": torch.empty((H, W, 3), dtype=torch.float32, device=dev),
                   "ambient": torch.empty((H, W, 3), dtype=torch.float32, device=dev)}
            if masks:
                out["masks"] = torch.empty((H, W, params.slices * (params.sectors // 32)), dtype=torch.int32,
                                           device=dev)
        check_outputs(out, H, W, self.device, masks_words=params.slices * (params.sectors // 32))
        o = ssvb_outputs(out["ao"].data_ptr(), out["gi"].data_ptr(), out["ambient"].data_ptr(),
                         out["masks"].data_ptr() if out.get("masks") is not None else None,
                         out["ao"].stride(0) * 4, out["gi"].stride(0) * 4, out["ambient"].stride(0) * 4,
                         out["masks"].stride(0) * 4 if out.get("masks") is not None else 0)
        d, n, r = image_of(depth), image_of(normal), image_of(radiance)
        c, p = camera.to_c(), params.to_c()
        check(lib().ssvb_compute(self.handle, ctypes.byref(d), ctypes.byref(n), ctypes.byref(r), ctypes.byref(c),
                                 ctypes.byref(p), ctypes.byref(o), _stream_ptr(stream)), "ssvb_compute")
        return out

    def _check_inputs(self, depth, normal, radiance, H, W, allow_host=False):
        check_tensor(depth, "depth", H, W, None, "f32", self.device, allow_host)
        check_tensor(normal, "normal", H, W, (3, 4), "image", self.device, allow_host)
        check_tensor(radiance, "radiance", H, W, (3, 4), "image", self.device, allow_host)

    @staticmethod
    def alloc_outputs(H, W, slices, device, masks=False, sectors=32):
        """Output tensors; masks (if asked) hold N_d x N_b / 32 words per pixel."""
        import torch
        out = {"ao": torch.empty((H, W), dtype=torch.float32, device=device),
               "gi": torch.empty((H, W, 3), dtype=torch.float32, device=device),
               "ambient": torch.empty((H, W, 3), dtype=torch.float32, device=device)}
        if masks:
            out["masks"] = torch.empty((H, W, slices * (sectors // 32)), dtype=torch.int32, device=device)
        return out

    @staticmethod
    def outputs_of(out) -> ssvb_outputs:
        m = out.get("masks")
        return ssvb_outputs(out["ao"].data_ptr(), out["gi"].data_ptr(), out["ambient"].data_ptr(),
                            m.data_ptr() if m is not None else None, out["ao"].stride(0) * 4,
                            out["gi"].stride(0) * 4, out["ambient"].stride(0) * 4,
                            m.stride(0) * 4 if m is not None else 0)

    def frame(self, depth, normal, radiance, camera: Camera, params: Params, out, allow_host=False) -> ssvb_frame:
        H, W = camera.height, camera.width
        self._check_inputs(depth, normal, radiance, H, W, allow_host)
        check_outputs(out, H, W, self.device, allow_host, masks_words=params.slices * (params.sectors // 32))
        return ssvb_frame(image_of(depth), image_of(normal), image_of(radiance), camera.to_c(), params.to_c(),
                          self.outputs_of(out))

    def frames(self, items):
        """Marshal (depth, normal, radiance, camera, params, out) tuples once into an
        ssvb_frame array, for repeated compute_batch / compute_each calls."""
        arr = (ssvb_frame * max(len(items), 1))()
        for i, it in enumerate(items):
            arr[i] = self.frame(*it)
        return FrameArray(arr, len(items))

    def compute_batch(self, items, stream=None):
        """items: list of (depth, normal, radiance, camera, params, out) with torch device
        tensors, or a FrameArray from frames(); runs ssvb_compute_batch (one graph replay
        per 64 frames)."""
        fa = items if isinstance(items, FrameArray) else self.frames(items)
        check(lib().ssvb_compute_batch(self.handle, fa.arr, fa.n, _stream_ptr(stream)), "ssvb_compute_batch")

    def compute_each(self, fa, stream=None):
        """One ssvb_compute call per frame of a FrameArray, back to back on one stream."""
        L, s, h = lib(), _stream_ptr(stream), self.handle
        for i in range(fa.n):
            F = fa.arr[i]
            check(L.ssvb_compute(h, ctypes.byref(F.depth), ctypes.byref(F.normal), ctypes.byref(F.radiance),
                                 ctypes.byref(F.camera), ctypes.byref(F.params), ctypes.byref(F.out), s),
                  "ssvb_compute")

    def inject_bounce(self, direct, albedo, gi, gain, out=None, stream=None):
        """Light buffer for the next frame: direct + gain * albedo * gi (multi-bounce).
        ``out`` defaults to a new tensor shaped and typed like ``direct``."""
        import torch
        H, W = direct.shape[:2]
        if out is None:
            out = torch.empty_like(direct)
        check_tensor(direct, "direct", H, W, (3, 4), "image", self.device)
        check_tensor(albedo, "albedo", H, W, (3, 4), "image", self.device)
        check_tensor(gi, "gi", H, W, (3,), "f32", self.device)
        check_tensor(out, "out", H, W, (3, 4), "image", self.device)  # the library checks C against direct
        d, a, o = image_of(direct), image_of(albedo), image_of(out)
        check(lib().ssvb_inject_bounce(self.handle, W, H, ctypes.byref(d), ctypes.byref(a), gi.data_ptr(),
                                       gi.stride(0) * 4, float(gain), ctypes.byref(o), _stream_ptr(stream)),
              "ssvb_inject_bounce")
        return out

    def denoise(self, depth, normal, camera: Camera, src, passes=2, normal_power=16, plane_sigma=0.05,
                resolution=1, out=None, tmp=None, stream=None):
        """Edge-aware a-trous denoising of ``src`` (dict ao, gi, ambient as ``compute``
        returns it); returns ``out`` (new tensors by default).  ``tmp`` holds the
        intermediate passes (allocated when needed and not given)."""
        import torch

        def like(s):
            return {k: torch.empty_like(s[k]) for k in ("ao", "gi", "ambient")}

        H, W = camera.height, camera.width
        check_tensor(depth, "depth", H, W, None, "f32", self.device)
        check_tensor(normal, "normal", H, W, (3, 4), "image", self.device)
        check_outputs({k: src.get(k) for k in ("ao", "gi", "ambient")}, H, W, self.device)
        if out is None:
            out = like(src)
        if tmp is None and passes > 1:
            tmp = like(src)
        check_outputs(out, H, W, self.device)
        if tmp is not None:
            check_outputs(tmp, H, W, self.device)
        P = ssvb_denoise_params(int(passes), int(normal_power), float(plane_sigma), int(resolution))
        d, n, c = image_of(depth), image_of(normal), camera.to_c()
        three = ("ao", "gi", "ambient")  # slice masks (if `src` holds them) are not filtered
        i, o = self.outputs_of({k: src[k] for k in three}), self.outputs_of({k: out[k] for k in three})
        t = self.outputs_of({k: tmp[k] for k in three}) if tmp is not None else None
        check(lib().ssvb_denoise(self.handle, ctypes.byref(d), ctypes.byref(n), ctypes.byref(c), ctypes.byref(i),
                                 ctypes.byref(t) if t is not None else None, ctypes.byref(o), ctypes.byref(P),
                                 _stream_ptr(stream)), "ssvb_denoise")
        return out

    def set_launch(self, shape=None):
        """Force a launch shape (tile_w, tile_h, strip, lanes_per_pixel); None: automatic."""
        if shape is None:
            check(lib().ssvb_set_launch(self.handle, None), "ssvb_set_launch")
        else:
            L = ssvb_launch(*shape)
            check(lib().ssvb_set_launch(self.handle, ctypes.byref(L)), "ssvb_set_launch")

    def set_slice_order(self, chunk_tiles: int = 0):
        """Slice-major work order of later compute calls and sequence steps in chunks of
        `chunk_tiles` tiles (0: each workgroup runs every slice of its tile)."""
        check(lib().ssvb_set_slice_order(self.handle, int(chunk_tiles)), "ssvb_set_slice_order")

    def get_launch(self, camera: Camera, params: Params, fp16_mask=0):
        L = ssvb_launch()
        check(lib().ssvb_get_launch(self.handle, ctypes.byref(camera.to_c()), ctypes.byref(params.to_c()),
                                    fp16_mask, ctypes.byref(L)), "ssvb_get_launch")
        return L.as_tuple()

    def autotune(self, depth, normal, radiance, camera: Camera, params: Params, out, stream=None):
        """Time candidate launch shapes on this frame; returns (shape tuple, ms)."""
        F = self.frame(depth, normal, radiance, camera, params, out)
        L = ssvb_launch()
        ms = ctypes.c_float()
        check(lib().ssvb_autotune(self.handle, ctypes.byref(F), _stream_ptr(stream), ctypes.byref(L),
                                  ctypes.byref(ms)), "ssvb_autotune")
        return L.as_tuple(), ms.value

    def debug_lattice(self, depth, camera: Camera, params: Params, stream=None):
        import torch
        H, W = camera.height, camera.width
        check_tensor(depth, "depth", H, W, None, "f32", self.device)
        xy = torch.empty((H, W, params.slices, 2, params.steps, 2), dtype=torch.int32, device=depth.device)
        d, c, p = image_of(depth), camera.to_c(), params.to_c()
        check(lib().ssvb_debug_lattice(self.handle, ctypes.byref(d), ctypes.byref(c), ctypes.byref(p),
                                       ctypes.c_void_p(xy.data_ptr()), _stream_ptr(stream)), "ssvb_debug_lattice")
        return xy

    def debug_endpoints(self, depth, normal, camera: Camera, params: Params, stream=None):
        import torch
        H, W = camera.height, camera.width
        check_tensor(depth, "depth", H, W, None, "f32", self.device)
        check_tensor(normal, "normal", H, W, (3, 4), "image", self.device)
        ep = torch.empty((H, W, params.slices, 2, params.steps, 2), dtype=torch.float32, device=depth.device)
        d, n, c, p = image_of(depth), image_of(normal), camera.to_c(), params.to_c()
        check(lib().ssvb_debug_endpoints(self.handle, ctypes.byref(d), ctypes.byref(n), ctypes.byref(c),
                                         ctypes.byref(p), ctypes.c_void_p(ep.data_ptr()), _stream_ptr(stream)),
              "ssvb_debug_endpoints")
        return ep

    def direction_table(self):
        buf = (ctypes.c_int32 * 8192)()
        check(lib().ssvb_debug_direction_table(self.handle, buf), "ssvb_debug_direction_table")
        return [(buf[2 * k], buf[2 * k + 1]) for k in range(4096)]


class Sequence:
    """An ssvb_sequence: frames of one size with multi-bounce feedback through a light
    buffer the sequence owns, and the noise seed advanced per frame (temporal jitter)."""

    def __init__(self, ctx: Context, width: int, height: int, light_dtype: str = "f32"):
        h = ctypes.c_void_p()
        dt = {"f32": F32, "f16": F16}[light_dtype]
        check(lib().ssvb_sequence_create(ctx.handle, int(width), int(height), dt, ctypes.byref(h)),
              "ssvb_sequence_create")
        self.handle = h
        self.ctx = ctx
        self.width, self.height, self.light_dtype = int(width), int(height), light_dtype

    def step(self, depth, normal, direct, albedo, camera: Camera, params: Params, gain: float, out=None,
             masks=False, stream=None):
        """Frame n of the sequence: light = direct + gain * albedo * GI of frame n - 1, then
        the gather on that light with seed params.seed + n; returns the outputs dict."""
        H, W = camera.height, camera.width
        ctx = self.ctx
        check_tensor(depth, "depth", H, W, None, "f32", ctx.device)
        check_tensor(normal, "normal", H, W, (3, 4), "image", ctx.device)
        check_tensor(direct, "direct", H, W, (3, 4), "image", ctx.device)
        check_tensor(albedo, "albedo", H, W, (3, 4), "image", ctx.device)
        if out is None:
            out = Context.alloc_outputs(H, W, params.slices, depth.device, masks=masks, sectors=params.sectors)
        check_outputs(out, H, W, ctx.device, masks_words=params.slices * (params.sectors // 32))
        o = Context.outputs_of(out)
        d, n, dl, al = image_of(depth), image_of(normal), image_of(direct), image_of(albedo)
        c, p = camera.to_c(), params.to_c()
        check(lib().ssvb_sequence_step(self.handle, ctypes.byref(d), ctypes.byref(n), ctypes.byref(dl),
                                       ctypes.byref(al), ctypes.byref(c), ctypes.byref(p), float(gain),
                                       ctypes.byref(o), _stream_ptr(stream)), "ssvb_sequence_step")
        return out

    def reset(self):
        check(lib().ssvb_sequence_reset(self.handle), "ssvb_sequence_reset")

    @property
    def frame(self) -> int:
        v = ctypes.c_int64()
        check(lib().ssvb_sequence_frame(self.handle, ctypes.byref(v)), "ssvb_sequence_frame")
        return v.value

    def light(self, stream=None):
        """A copy of the light buffer of the last step ([H, W, 3] tensor of the light type)."""
        import torch
        t = torch.empty((self.height, self.width, 3),
                        dtype=torch.float16 if self.light_dtype == "f16" else torch.float32,
                        device=f"cuda:{self.ctx.device}")
        check(lib().ssvb_sequence_copy_light(self.handle, ctypes.c_void_p(t.data_ptr()), 0, _stream_ptr(stream)),
              "ssvb_sequence_copy_light")
        return t

    def close(self):
        if getattr(self, "handle", None):
            st = lib().ssvb_sequence_destroy(self.handle)
            self.handle = None
            check(st, "ssvb_sequence_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """An ssvb_server: admission by HBM footprint and continuous batching on `streams`
    compute streams.  Tensors handed to submit (device, or pinned host) must stay alive
    until the request has finished; this wrapper keeps a reference to them meanwhile."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, streams: int = 1):
        h = ctypes.c_void_p()
        check(lib().ssvb_server_create(ctx.handle, int(hbm_budget_bytes), int(streams), ctypes.byref(h)),
              "ssvb_server_create")
        self.handle = h
        self.ctx = ctx
        self._held = {}

    def submit(self, depth, normal, radiance, camera: Camera, params: Params, out, stream=None) -> int:
        """Queue a frame; the server orders its work after everything enqueued on `stream`
        (default: the current torch stream of the context's device) before this call."""
        F = self.ctx.frame(depth, normal, radiance, camera, params, out, allow_host=True)
        t = ctypes.c_uint64()
        check(lib().ssvb_server_submit(self.handle, ctypes.byref(F), _stream_ptr(stream), ctypes.byref(t)),
              "ssvb_server_submit")
        self._held[t.value] = (depth, normal, radiance, out)
        return t.value

    def poll(self, ticket: int):
        """(done, latency_ms or None)."""
        done, lat = ctypes.c_int32(), ctypes.c_double()
        check(lib().ssvb_server_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(lat)), "ssvb_server_poll")
        return bool(done.value), (lat.value if done.value else None)

    def wait(self, ticket: int, timeout_ms: float = -1.0) -> float:
        """Block until the request finishes; returns its latency in ms."""
        lat = ctypes.c_double()
        check(lib().ssvb_server_wait(self.handle, ticket, float(timeout_ms), ctypes.byref(lat)), "ssvb_server_wait")
        return lat.value

    def release(self, ticket: int) -> None:
        check(lib().ssvb_server_release(self.handle, ticket), "ssvb_server_release")
        self._held.pop(ticket, None)

    def stats(self) -> dict:
        c = ssvb_server_counters()
        check(lib().ssvb_server_stats(self.handle, ctypes.byref(c)), "ssvb_server_stats")
        return c.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            st = lib().ssvb_server_destroy(self.handle)
            self.handle = None
            self._held.clear()
            check(st, "ssvb_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_params() -> ssvb_params:
    p = ssvb_params()
    lib().ssvb_default_params(ctypes.byref(p))
    return p


def validate(depth: ssvb_image, normal: ssvb_image, radiance: ssvb_image, camera: ssvb_camera, params: ssvb_params,
             out: ssvb_outputs) -> int:
    """Host-only argument check (no device, no context); returns the status code."""
    return lib().ssvb_validate(ctypes.byref(depth), ctypes.byref(normal), ctypes.byref(radiance),
                               ctypes.byref(camera), ctypes.byref(params), ctypes.byref(out))


def noise_constants():
    buf = (ctypes.c_uint32 * 3)()
    lib().ssvb_debug_noise_constants(buf)
    return list(buf)
