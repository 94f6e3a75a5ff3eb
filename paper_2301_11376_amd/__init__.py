"""Screen-space visibility-bitmask AO / indirect / ambient gather on AMD MI355X (gfx950).

The work runs in the HIP library ``libssvb.so`` (C ABI in ``include/ssvb.h``);
``binding`` marshals torch device tensors into it.  Importing this package does not load
the library; the first call that needs it does, and fails loudly if it is missing.
"""
from .binding import (  # noqa: F401
    Camera,
    Context,
    FrameArray,
    Params,
    SSVBError,
    Sequence,
    Server,
    HIT_ROUND,
    HIT_PSEUDOCODE,
    NOISE_HASH,
    NOISE_R2,
    NOISE_FIXED,
    NOISE_NAMES,
    STEPS_UNIFORM,
    STEPS_QUADRATIC,
    lib,
)
