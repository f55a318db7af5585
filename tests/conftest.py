import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer statistical checks")


def pytest_collection_modifyitems(config, items):
    # Skip GPU tests when no GPU is visible, unless they were selected
    # explicitly ("-m gpu"): then they run and fail, so that a GPU run without
    # a visible GPU is reported as a failure rather than as skipped tests.
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    marker_expr = config.getoption("-m") or ""
    if "gpu" in marker_expr and "not gpu" not in marker_expr:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
