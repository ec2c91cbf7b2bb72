import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def rocrand_ref():
    """Path of a host program that prints rocRAND Philox4x32-10 blocks."""
    src = os.path.join(ROOT, "tests", "helpers", "rocrand_philox_ref.cpp")
    out_dir = os.path.join(ROOT, "tests", "_build")
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, "rocrand_philox_ref")
    if not os.path.exists(exe) or os.path.getmtime(exe) < os.path.getmtime(src):
        hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
        if not os.path.exists(hipcc):
            pytest.skip("hipcc not available to build the rocRAND reference")
        subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", src, "-o", exe + ".tmp"],
                       check=True, capture_output=True)
        os.replace(exe + ".tmp", exe)
    return exe
