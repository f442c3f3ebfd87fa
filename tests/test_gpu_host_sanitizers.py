"""The C-ABI driver (tests/host_sanitizers/capi_driver.cpp) built with the
host code of the library under AddressSanitizer and UndefinedBehavior-
Sanitizer (GPU code as in the product; `build()` builds both): every entry
point and its error paths on small oil-water and black-oil grids, the
network's entry points and the caller allocator, with no sanitizer report
and every call returning what it should."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "host_sanitizers", "capi_driver")


def test_capi_under_host_sanitizers():
    if not os.path.exists(DRIVER):
        pytest.fail("the sanitized C-ABI driver is not built (run __graft_entry__.build())")
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([DRIVER], capture_output=True, text=True, timeout=240, env=env)
    print(p.stdout[-2000:], p.stderr[-4000:], flush=True)
    assert "ERROR: AddressSanitizer" not in p.stderr
    assert "runtime error:" not in p.stderr
    assert p.returncode == 0
    assert "all checks passed" in p.stdout
