"""The ABI and layout tests again, against a host-sanitizer build of the
library: the host sources under AddressSanitizer and
UndefinedBehaviorSanitizer (g++), the kernel objects of the ordinary build
unchanged.  Each run is a child process with the sanitizer runtime preloaded;
it must pass with no sanitizer report, and the child is checked to have
really loaded the sanitized library and the runtime."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer", "SUMMARY: UndefinedBehavior")


@pytest.fixture(scope="module")
def san():
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    from paper_2110_01409_amd import build_sanitized as bs
    try:
        bs.build()
    except FileNotFoundError as e:
        pytest.skip(str(e))
    return bs


def test_sanitized_library_is_what_the_child_loads(san):
    code = ("import ctypes, os; ctypes.CDLL(os.environ['DG_LIBRARY']); "
            "maps = open('/proc/self/maps').read(); "
            "print('asan' if 'libasan' in maps else 'no-asan', 'san-lib' if 'libdg_san' in maps else 'no-lib')")
    r = subprocess.run([sys.executable, "-c", code], env=san.env(), capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split() == ["asan", "san-lib"], r.stdout


def test_abi_and_layout_under_sanitizers(san):
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_plan.py")],
                       cwd=ROOT, env=san.env(), capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert " passed" in r.stdout, out[-2000:]
    for rep in REPORTS:
        assert rep not in out, out[-4000:]
