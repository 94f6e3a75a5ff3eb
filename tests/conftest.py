import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


# tests whose oracle references are computed when collection ends (see parity.BAND_REFS)
BAND_REF_TESTS = {"test_parity_c2_1080p_full_frame": ["c2_full"],
                  "test_parity_c3_4k_fp16_band": ["c3_band_fp16", "c3_band_fp32"]}


def pytest_collection_finish(session):
    """Before any test runs (and so before any test initialises the GPU), compute the
    oracle references of the selected large-frame parity tests in forked processes."""
    names = []
    for item in session.items:
        names += BAND_REF_TESTS.get(item.originalname if hasattr(item, "originalname") else item.name, [])
    if not names or session.config.option.collectonly:
        return
    import parity
    workers = max(1, min(16, os.cpu_count() or 1))
    parity.compute_band_refs(sorted(set(names)), workers)
