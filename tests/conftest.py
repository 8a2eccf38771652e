import os
import sys

import pytest

if os.environ.get("PYTEST_XDIST_WORKER"):
    # worker processes share the CPUs: a few threads each for torch's CPU kernels
    os.environ.setdefault("OMP_NUM_THREADS", "2")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.hookimpl(tryfirst=True)
def pytest_cmdline_main(config):
    """A run that deselects the GPU tests is CPU work only (the oracle and its pins,
    the host logic, the CPU build of the library, each test in its own state):
    unless ``-n`` is given it spreads the tests over worker processes."""
    opt = config.option
    if not hasattr(opt, "numprocesses") or opt.numprocesses is not None or os.environ.get("PYTEST_XDIST_WORKER"):
        return None
    if "not gpu" not in (opt.markexpr or "").replace("  ", " ") or getattr(opt, "collectonly", False):
        return None
    opt.numprocesses = max(1, min(6, (os.cpu_count() or 2) - 2))
    return None


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
