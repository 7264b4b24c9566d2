import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running (still part of the default suite)")


def _have_gpu() -> bool:
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _have_gpu():
        return
    skip = pytest.mark.skip(reason="no GPU visible in this process")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def orc():
    import oracle
    if not os.path.exists(oracle.lib_path()):
        oracle.build()
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def rocrand_philox(tmp_path_factory):
    """Path of a host program that evaluates rocRAND's Philox4x32-10 block function.

    Built from tests/helpers/rocrand_philox.cpp with hipcc (host code only);
    skipped where hipcc or the rocRAND headers are absent.
    """
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not (os.path.exists(hipcc) and os.path.exists(hdr)):
        pytest.skip("hipcc / rocRAND headers not available")
    out = tmp_path_factory.mktemp("rocrand") / "rocrand_philox"
    src = os.path.join(ROOT, "tests", "helpers", "rocrand_philox.cpp")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-w", src, "-o", str(out)],
                   check=True, capture_output=True)
    return str(out)
