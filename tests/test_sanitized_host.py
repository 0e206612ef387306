"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): the library is rebuilt with the host compilation instrumented
(build.SANITIZE_FLAGS) and the ABI, reduced-basis table and batch-planner tests
run against it in a child process with the sanitizer runtime preloaded.  Any
out-of-bounds access, use after free or undefined behaviour in the argument
validation, workspace carving, table construction or planning aborts the child."""

import os
import shutil
import subprocess
import sys

import pytest

from paper_2010_03598_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow

CHILD_TESTS = ["tests/test_abi.py", "tests/test_pe_host.py", "tests/test_batched_host.py"]

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
from paper_2010_03598_amd import _lib
_lib.load()
maps = open("/proc/self/maps").read()
assert _lib.LIB_PATH in maps, "the sanitizer build is not the loaded library"
assert "libclang_rt.asan" in maps, "the sanitizer runtime is not loaded"
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", *{tests!r}]))
"""


def stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    return any(os.path.getmtime(s) > t for s in build.sources() + [
        os.path.join(build.INCLUDE, "kgrape.h")])


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc is needed for the sanitizer build")
def test_host_code_under_address_and_ub_sanitizers():
    lib = build.SANITIZED_LIB
    if stale(lib):
        build.build(sanitized=True)
    env = dict(os.environ)
    env.update({"LD_PRELOAD": build.asan_runtime(),
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
                "KG_LIBRARY": lib})
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, tests=CHILD_TESTS)],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=1200)
    assert r.returncode == 0, r.stdout[-4000:]
