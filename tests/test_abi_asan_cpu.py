"""The C ABI's host code under AddressSanitizer: the library rebuilt with the
sanitizer on its host compilation only (tests/asan_lib.py) runs the CPU ABI
tests (loading, exported symbols, every argument check that returns before a
GPU is touched) in a child process with the sanitizer runtime preloaded."""
import os
import subprocess
import sys

import pytest

import asan_lib

ROOT = asan_lib.ROOT


def test_abi_checks_run_clean_under_address_sanitizer():
    rt = asan_lib.runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this ROCm")
    lib = asan_lib.build()
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               MFFV_LIBRARY=lib, PYTHONPATH=ROOT)
    # the child loads the sanitized library, not the product one
    probe = subprocess.run([sys.executable, "-c",
                            "from paper_2408_03452_amd import mffv; print(mffv.lib()._name)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0, probe.stderr[-2000:]
    assert probe.stdout.strip().endswith("libmffv_asan.so"), probe.stdout
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
