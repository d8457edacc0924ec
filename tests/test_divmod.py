"""The exact division behind every kernel's evaluation of eq. (3) (Section 3):
quotient and remainder of (2 k a + N - neg) / 2N from a float reciprocal
estimate biased downwards and one integer correction.  The library's own
helper is built for the host and run with the reciprocal off by -1, 0 and
+1 ulp, for every divisor below 2^16 at every quotient boundary (CPU only)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "divmod_check.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("dmc") / "divmod_check")
    # Host code only; no contraction of the float product into anything else.
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-ffp-contract=off", "-pthread",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2009_09500_amd", "csrc"),
                           "-o", out, SRC])
    return out


def _run(driver, *args):
    r = subprocess.run([driver] + [str(a) for a in args], capture_output=True, text=True)
    words = r.stdout.split()
    return r.returncode, int(words[1]), int(words[3]), r.stdout


def test_every_divisor_every_quotient_boundary(driver):
    rc, cases, bad, out = _run(driver, 65536, min(8, os.cpu_count() or 1))
    # 65534 divisors x 3 estimates x (2 numerators per quotient + 65 more).
    assert cases > 65534 * 3 * 2 * 16384, out
    assert rc == 0 and bad == 0, out


def test_unbiased_estimate_is_caught(driver):
    """Without the downward scaling the +1 ulp estimate overshoots some
    quotients: the check must see it."""
    rc, cases, bad, out = _run(driver, 4096, min(8, os.cpu_count() or 1), "unbiased")
    assert rc == 1 and bad > 0, out
