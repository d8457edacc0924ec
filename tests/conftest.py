import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_jobs = {"proc": None, "dir": None}


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def _gpu_tests_selected(config) -> bool:
    expr = (config.getoption("markexpr") or "").replace(" ", "")
    if "notgpu" in expr:
        return False
    return os.path.exists("/dev/kfd")


def pytest_sessionstart(session):
    """Start the full-size oracle computations (CPU only, in a separate
    process) before any test initialises the GPU, so the full-size parity
    tests find their expected results ready."""
    if not _gpu_tests_selected(session.config):
        return
    d = tempfile.mkdtemp(prefix="vox_oracle_")
    _jobs["dir"] = d
    _jobs["proc"] = subprocess.Popen(
        [sys.executable, "-m", "tests.oracle_jobs", d, "arbitrary4m_euclid", "arbitrary4m", "scenes"],
        cwd=ROOT, stdout=subprocess.DEVNULL, stderr=open(os.path.join(d, "jobs.log"), "w"))


def pytest_sessionfinish(session, exitstatus):
    p = _jobs["proc"]
    if p is not None and p.poll() is None:
        p.terminate()
        try:
            p.wait(timeout=10)
        except subprocess.TimeoutExpired:
            p.kill()


@pytest.fixture(scope="session")
def oracle_jobs_dir():
    if _jobs["dir"] is None:
        pytest.skip("full-size oracle jobs were not started in this session")
    return _jobs["dir"]
