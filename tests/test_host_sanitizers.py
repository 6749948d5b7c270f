"""The library's host code (option validation, Algorithm 1 hierarchy, the
workspace sizing pass, argument checks) under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/host_check.cpp linked against solver.cpp
compiled with both sanitizers on its host side.  CPU only."""
import os
import shutil
import subprocess

import pytest

from paper_2508_09589_amd import build as B


def test_host_code_is_clean_under_asan_and_ubsan():
    if shutil.which(B._hipcc()) is None and not os.path.exists(B._hipcc()):
        pytest.skip("hipcc not available")
    kern = [os.path.join(B.BUILD, os.path.splitext(x)[0] + ".o") for x in B.SOURCES]
    if not all(os.path.exists(k) for k in kern):
        B.build(jobs=4)
    exe = B.build_host_check()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host_check ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
