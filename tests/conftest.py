import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    has_gpu = None
    for item in items:
        if "gpu" in item.keywords:
            if has_gpu is None:
                try:
                    import torch
                    has_gpu = torch.cuda.is_available()
                except Exception:
                    has_gpu = False
            if not has_gpu:
                item.add_marker(pytest.mark.skip(reason="no GPU in this environment"))
