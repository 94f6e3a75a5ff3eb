"""FP64 CPU oracle for the screen-space visibility-bitmask gather.

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path (the HIP
library and its Python binding) never imports, links or calls it, and the oracle shares
no code, table or constant generator with that path.
"""
from .ssvb_oracle import (  # noqa: F401
    Camera,
    Params,
    ROUND,
    PSEUDOCODE,
    NOISE_HASH,
    NOISE_R2,
    NOISE_FIXED,
    NOISE_NAMES,
    STEPS_UNIFORM,
    STEPS_QUADRATIC,
    pcg_hash,
    pixel_hash,
    r2_constants,
    direction_lut,
    slice_noise,
    step_q4,
    step_offset_q4,
    compute,
    bilateral_upsample,
    inject_bounce,
    bounce_sequence,
    denoise,
    DENOISE_KERNEL,
    UPSAMPLE_SIGMA,
    UPSAMPLE_FLOOR,
    sh_eval,
)
