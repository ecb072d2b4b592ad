"""The host side of the library under AddressSanitizer and
UndefinedBehaviorSanitizer: the CPU-side ABI tests (argument checks, plan
caches, workspace layouts, batch grouping, the serving layer's checks) run
against a build whose host sources (plan.cpp, server.cpp) carry both
sanitizers, with the toolchain's ASan runtime preloaded.

CPU only: the run adds a preload of its own, so it is skipped where the
environment already preloads something (a GPU host's harness).
"""
import os
import subprocess
import sys

import pytest

from paper_1702_01904_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))


def test_host_abi_tests_pass_under_asan_and_ubsan():
    rt = B.asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime in the HIP toolchain")
    if os.environ.get("LD_PRELOAD") or os.path.exists("/etc/ld.so.preload"):
        pytest.skip("the environment preloads a library already")
    if not all(os.path.exists(os.path.join(B.OUT_DIR, os.path.splitext(s)[0] + ".o"))
               for s in B.SOURCES):
        B.build()
    lib = B.build_sanitized()
    env = dict(os.environ, PRISM_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(HERE, "test_abi_host.py")],
                       env=env, capture_output=True, text=True, timeout=900, cwd=os.path.dirname(HERE))
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert " passed" in r.stdout and "failed" not in r.stdout
