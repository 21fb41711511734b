import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


TUNE_FILE = os.path.join(ROOT, "profiles", "tune_mi355x.json")


@pytest.fixture
def bench_tuning():
    """Apply the committed tune file's entry for a plan's configuration (the launch configuration
    bench.py times); with required=True the file must hold one."""
    def apply(plan, required=True):
        from paper_2105_01612_amd.autotune import apply_cached

        t = apply_cached(plan, TUNE_FILE)
        assert t is not None or not required, f"{TUNE_FILE} holds no entry for this benchmark configuration"
        return t
    return apply


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running case")


def pytest_collection_modifyitems(config, items):
    # GPU tests need a visible device; on a CPU-only host they are skipped, not failed.
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
